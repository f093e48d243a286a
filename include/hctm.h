/*
 * hctm.h -- C ABI of the Hermitian-symmetric CTMRG library (libhctm.so).
 *
 * Method: arXiv:2410.11596, "Exploiting the Hermitian symmetry in tensor
 * network algorithms".  A real iPEPS tensor A (Sec. II A) defines the double
 * layer a = sum_s A (x) A (Fig. 1b).  Joining each ket leg with its bra leg
 * gives a leg of dimension D^2 on which the bra-ket swap S acts; for real A
 * the double layer is invariant under S on all four legs (Fig. 1e-f), so in
 * the eigenbasis of S (Sec. II B) the double layer, the corners C and the
 * edges T of the CTMRG environment (Fig. 1d) are Z2 block sparse.  The
 * library runs directional CTMRG in that basis, block by block, on one
 * AMD Instinct MI355X (gfx950), in FP64.  CTM_FORM_DENSE runs the same code
 * on the unrotated, one-sector network (the non-symmetric reference form).
 *
 * Conventions shared by all calls
 *  - Every call returns CTM_OK (0) or an error code; no exception crosses the
 *    ABI.  ctm_last_error() gives a message for the last failing call.
 *  - After an error raised while work was running on the GPU, the context is
 *    poisoned: every call except ctm_free/ctm_last_error returns CTM_E_STATE.
 *  - Host arrays are plain row-major FP64 buffers owned by the caller; the
 *    library copies inputs at the call and writes outputs before returning.
 *  - Device memory: the context owns all device memory it allocates.  If
 *    ctm_opts.workspace is set, the library carves its buffers out of that
 *    caller-owned device allocation (at least ctm_workspace_size bytes) and
 *    allocates nothing else of that size; the caller keeps it alive until
 *    ctm_free.
 *  - Streams: work is issued on ctm_opts.stream (a hipStream_t) or on a
 *    stream owned by the context.  Calls that return host data synchronise
 *    that stream.
 *  - One context may be used by one host thread at a time.
 *
 * Tensor layout: A is d x D x D x D x D, legs [s, u, l, d, r] (physical,
 * up, left, down, right).  A joined bra-ket leg index is K = k*D + kbar
 * (ket index k, bra index kbar).
 *
 * Unit cell: the network may repeat an Lx x Ly cell of different tensors
 * A(x, y), x = 0..Lx-1 to the right, y = 0..Ly-1 downwards (periodic).  The
 * paper's method is stated for one tensor; on a cell every site keeps its own
 * corners and edges, and a move sweeps the columns (or rows) of the cell in
 * turn, each cut taking its projectors from the 2 x 2 block of sites next to
 * it.  With Lx = Ly = 1 (the default) this is the one-site algorithm.
 */
#ifndef HCTM_H
#define HCTM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctm_ctx ctm_ctx;

enum {
  CTM_OK = 0,
  CTM_E_ARG = 1,     /* invalid argument (sizes, pointers, options) */
  CTM_E_NOMEM = 2,   /* device allocation failed or workspace too small */
  CTM_E_HIP = 3,     /* HIP runtime error */
  CTM_E_NUMERIC = 4, /* non-finite input, or a factorisation that broke down */
  CTM_E_STATE = 5    /* context poisoned by an earlier error */
};

enum { CTM_FORM_Z2 = 0, CTM_FORM_DENSE = 1 };

/* Arithmetic of the block products of the moves (enlarged corners, halves,
 * projectors, renormalisation).  CTM_PREC_FP32: operands rounded to FP32,
 * FP32 matrix-core products and accumulation, FP64 results.
 * CTM_PREC_BF16X3: each operand split into BF16 parts x = hi + lo, the
 * products hi*hi + hi*lo + lo*hi on the BF16 matrix cores with FP32
 * accumulation (about 2^-16 relative per product).  In both the truncated
 * SVD, the normalisations and the observables stay FP64, and a run is brought
 * back to the FP64 fixed point by further iterations in FP64
 * (ctm_set_precision). */
enum { CTM_PREC_FP64 = 0, CTM_PREC_FP32 = 1, CTM_PREC_BF16X3 = 2 };

typedef struct {
  int form;                    /* CTM_FORM_Z2 (default) or CTM_FORM_DENSE */
  int Lx, Ly;                  /* unit cell, each in [1, 4] (default 1 x 1) */
  const double* boundary;      /* host, D*D vector b[K] tracing the open boundary
                                  legs of the initial 3x3 patch; NULL selects
                                  b = sum_k |k k> (the open boundary).  In the Z2
                                  form b must be swap symmetric, b[k*D+l] = b[l*D+k]. */
  double svd_rel_cutoff;       /* keep singular values > cutoff * largest (default 1e-12) */
  int svd_iters;               /* at most this many subspace iterations per truncated
                                  SVD (default 12; twice that in the C4v scheme); fewer
                                  once the basis has converged */
  int form_m;                  /* 0 (default): apply the decomposed matrix through the
                                  enlarged corners when few iterations are expected;
                                  1: always form it (H_d H_u) first */
  int precision;               /* CTM_PREC_FP64 (default), CTM_PREC_FP32 or CTM_PREC_BF16X3 */
  int c4v;                     /* 1: the C4v-symmetric scheme (Sec. II A) for a tensor
                                  invariant under the rotations and reflections of the
                                  square (checked to 1e-12 relative; 1 x 1 cell only):
                                  one corner C and one edge T stand for all four, and an
                                  iteration is one absorption C' = V^T Q V,
                                  T' = V^T (T a) V with V the dominant eigenvectors
                                  (largest |eigenvalue|) of the symmetric enlarged
                                  corner Q = C T T a, per sector in the Z2 form.
                                  0 (default): the directional moves */
  unsigned long long seed;     /* seed of the subspace-iteration start blocks */
  int profile;                 /* 1: time every GEMM launch with HIP events (ctm_gemm_stats) */
  void* stream;                /* hipStream_t or NULL */
  void* workspace;             /* caller-owned device memory or NULL */
  size_t workspace_bytes;
} ctm_opts;

/* Fill *o with the defaults above. */
int ctm_opts_default(ctm_opts* o);

/* Device bytes a context with these sizes needs (for ctm_opts.workspace). */
int ctm_workspace_size(int d, int D, int chi, const ctm_opts* o, size_t* bytes);

/*
 * Create a context: copies A (host, Lx*Ly tensors of d*D^4 doubles, legs
 * [s,u,l,d,r], site (x, y) at offset (y*Lx + x)*d*D^4), forms the double
 * layers in the eigenbasis of the swap (Sec. II B) and the initial
 * environment of boundary dimension D^2 (every site's 3x3 patch traced with
 * the boundary vector).  chi >= 1 is the boundary dimension kept after each
 * truncation (Sec. II A).  Requires 1 <= d <= 16, 1 <= D <= 8,
 * 1 <= chi <= 4096, finite A; *out is NULL on failure.
 */
int ctm_init(ctm_ctx** out, const double* A, int d, int D, int chi, const ctm_opts* o);

/*
 * Run n_iter CTMRG iterations; one iteration is a left, right, top and
 * bottom move, each absorbing the columns or rows of double-layer tensors of
 * the cell and truncating every grown bond back to chi with per-sector SVD
 * projectors.  After every iteration the corner spectra are compared with the
 * previous ones (see ctm_converged).
 */
int ctm_step(ctm_ctx* c, int n_iter);

/* Precision of the block products of the following ctm_step calls
 * (CTM_PREC_FP64, CTM_PREC_FP32 or CTM_PREC_BF16X3); the environment is
 * kept. */
int ctm_set_precision(ctm_ctx* c, int precision);

/*
 * delta = max over the four corners of every site of || s_new - s_old ||_2,
 * s the singular values of a corner divided by their sum and padded with
 * zeros to chi, between the last two iterations (+inf before the second).
 * converged = (delta < tol).  Synchronises.
 */
int ctm_converged(ctm_ctx* c, double tol, int* converged, double* delta);

/* One-site reduced density matrix rho[s][s'] of site (x, y) of the cell
 * (host, d*d), trace one. */
int ctm_rdm_1site(ctm_ctx* c, int x, int y, double* rho);

/*
 * Two-site RDM of a nearest-neighbour pair, rho[(s1 s2)][(s1' s2')] (host,
 * d^4), trace one.  dir 0: the pair (x, y)-(x+1, y), 1: the pair
 * (x, y)-(x, y+1), the first site first.  In the Z2 form both RDMs are
 * symmetric by construction: only the even (symmetric) part of an impurity
 * couples to the even environment, and pairs of odd (antisymmetric) parts are
 * combined so that the result is invariant under the joint ket-bra swap.
 */
int ctm_rdm_2site(ctm_ctx* c, int x, int y, int dir, double* rho);

/* E = mean over the sites of Tr(rho_h h) + Tr(rho_v h), for a bond operator
 * h (host, d^2 x d^2). */
int ctm_energy(ctm_ctx* c, const double* h, double* e);

/* Release everything; NULL is accepted. */
void ctm_free(ctm_ctx* c);

/* Message of the last error on this context (never NULL). */
const char* ctm_last_error(const ctm_ctx* c);

/* ---- diagnostics used by the tests ------------------------------------ */

/* One-site environment of site (x, y) with the centre removed (Sec. III A),
 * back in the plain basis, normalised so that <eps, a> = 1; host, D^8
 * doubles ordered [U, L, Dn, R] with joined indices K = k*D + kbar. */
int ctm_env_epsilon(ctm_ctx* c, int x, int y, double* eps);

/* Hermitian symmetry error S_err = ||e - e^dag|| / ||e + e^dag|| (Sec. III A),
 * the largest over the sites. */
int ctm_s_err(ctm_ctx* c, double* s_err);

/* ln of the partition function per site, kappa = Z11 Z00 / (Z10 Z01);
 * 1 x 1 cell only (CTM_E_ARG otherwise). */
int ctm_log_kappa(ctm_ctx* c, double* ln_kappa);

/* Number of truncations run so far (one per cut: a move of an Lx x Ly cell
 * truncates Lx*Ly cuts). */
int ctm_num_records(ctm_ctx* c, int* n);

/*
 * Record of truncation m (0-based, in the order run): the kept singular
 * values of the decomposed matrix, merged over both sectors in descending
 * order and divided by the largest, and the kept sector sizes.  s: host array
 * of at least cap doubles.  info (may be NULL): 8 ints, the frame of the move
 * (0 left, 1 top, 2 right, 3 bottom), the column swept and the row of the cut
 * in the coordinates of that frame, then for the even and the odd sector the
 * subspace iterations run (0: the block was decomposed directly) and the
 * Jacobi sweeps of the final small SVD, and 1 if the matrix was applied
 * through the enlarged corners instead of being formed (see form_m).
 */
int ctm_record(ctm_ctx* c, int m, double* s, int cap, int* n, int* k_even, int* k_odd, int* info);

/* Current boundary bond on side 0..3 (top, right, bottom, left) of site
 * (x, y): the bond of the edge tensor's first leg (T1's left, T2's up, T3's
 * right, T4's down leg), its even and odd sizes. */
int ctm_sector_dims(ctm_ctx* c, int x, int y, int side, int* chi_even, int* chi_odd);

/* GPU seconds of the last ctm_step call per phase of the moves:
 * t[0] enlarged corners, t[1] half-system products and M, t[2] truncated SVD
 * (subspace iteration, Jacobi, selection), t[3] projectors, renormalisation
 * and normalisation.  *n = 4. */
int ctm_timing(ctm_ctx* c, double* t, int cap, int* n);

/* Profile mode only (ctm_opts.profile = 1): algorithmic FP64 GEMM flops
 * (2*M*N*K per block product), summed GEMM launch durations in seconds and
 * the number of launches since the last reset; reset != 0 clears them. */
int ctm_gemm_stats(ctm_ctx* c, double* flops, double* seconds, long long* launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* HCTM_H */
