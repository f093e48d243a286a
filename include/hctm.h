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

/* Device bytes a context with these sizes needs (for ctm_opts.workspace):
 * the double layers and the environment tensors C, T of Sec. II A for every
 * site, the enlarged corners, and the work arrays of the truncations.  It
 * grows as (chi D^2)^2.  Errors: CTM_E_ARG for sizes or options that ctm_init
 * would refuse; a size too large for the device is not an error here (the
 * allocation in ctm_init reports CTM_E_NOMEM). */
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
 * Run n_iter CTMRG iterations (Sec. II A: the boundary grows by absorbing
 * rows and columns, and every grown bond of dimension chi D^2 is truncated
 * back to chi by an SVD; Sec. II B, points (1)-(3): in the swap eigenbasis
 * every product and SVD runs per parity sector and the truncation keeps the
 * symmetry).  One iteration is a left, right, top and bottom move, each
 * absorbing the columns or rows of double-layer tensors of the cell and
 * truncating every grown bond back to chi with per-sector SVD projectors.
 * After every iteration the corner spectra are compared with the previous
 * ones (see ctm_converged).  Work is enqueued on the context's stream; the
 * call reads back small values (kept counts, stopping tests) and returns
 * when the iterations are done.  Errors: CTM_E_ARG for n_iter < 0;
 * CTM_E_NUMERIC (context poisoned) if a decomposition breaks down.
 */
int ctm_step(ctm_ctx* c, int n_iter);

/* Precision of the block products of the following ctm_step calls
 * (CTM_PREC_FP64, CTM_PREC_FP32 or CTM_PREC_BF16X3); the environment is
 * kept.  The paper computes in FP64 throughout; the lower precisions are an
 * option of this library for the products of Sec. II A, with FP64 iterations
 * afterwards to reach the FP64 fixed point.  Errors: CTM_E_ARG for another
 * value, or for FP32 or BF16X3 on a complex-tensor context (FP64 only). */
int ctm_set_precision(ctm_ctx* c, int precision);

/*
 * Convergence of the environment (the boundary tensors of Sec. II A,
 * Fig. 1d, approach a fixed point as the iterations grow the system):
 * delta = max over the four corners of every site of || s_new - s_old ||_2,
 * s the singular values of a corner divided by their sum and padded with
 * zeros to max(chi, D^2), between the last iteration and the one before
 * (the initial environment before the first; +inf before any).
 * converged = (delta < tol).  Either output may be NULL.  Synchronises.
 */
int ctm_converged(ctm_ctx* c, double tol, int* converged, double* delta);

/*
 * Current spectrum of corner `corner` (0 C1 up-left, 1 C2 up-right, 2 C3
 * down-right, 3 C4 down-left; the corner matrices of Sec. II A, Fig. 1d) of
 * site (x, y): the singular values of both
 * sectors merged in descending order, divided by their sum, zero padded;
 * *n = its length max(chi, D^2).  s: host array of cap >= *n doubles, or
 * NULL to query *n.  These are the vectors ctm_converged compares.
 */
int ctm_corner_spectrum(ctm_ctx* c, int x, int y, int corner, double* s, int cap, int* n);
/* (The paper names no convergence measure; the change of these spectra is
 * the one used here.  Errors: CTM_E_ARG for a bad site or corner, or
 * cap < *n with s not NULL.  Synchronises.) */

/*
 * Health of the truncations run so far (Sec. II B, point (3); Sec. III A):
 * *unconverged = truncations in which a sector's subspace iteration reached
 * ctm_opts.svd_iters iterations without passing its residual test (the
 * iterate is used as it stands); *multiplet_splits = truncations whose chi
 * cut separated two values within a relative 1e-10 of each other (the first
 * discarded value above the cutoff), where the kept space is not unique.
 * Either output may be NULL.
 */
int ctm_svd_health(ctm_ctx* c, int* unconverged, int* multiplet_splits);

/* One-site reduced density matrix rho[s][s'] of site (x, y) of the cell
 * (host, d*d, row-major), trace one: the one-site environment (Sec. III A)
 * closed with A[s] (x) A[s'] (Sec. II A, Fig. 1b).  In the Z2 form only
 * the symmetric impurity (A[s] (x) A[s'] + A[s'] (x) A[s]) / 2 enters, the
 * only part that is even under the swap of Sec. II B, so rho is symmetric
 * (Hermitian) bit for bit.  Errors: CTM_E_ARG for a site outside the cell or
 * a NULL rho.  Synchronises. */
int ctm_rdm_1site(ctm_ctx* c, int x, int y, double* rho);

/*
 * Two-site RDM of a nearest-neighbour pair (Sec. I and Sec. II B point (3):
 * reduced density matrices are the observables whose Hermiticity the swap
 * symmetry protects), rho[(s1 s2)][(s1' s2')] (host, d^4, row-major), trace
 * one.  Errors: CTM_E_ARG for a bad site, dir or a NULL rho.  Synchronises.
 * dir 0: the pair (x, y)-(x+1, y), 1: the pair
 * (x, y)-(x, y+1), the first site first.  In the Z2 form both RDMs are
 * symmetric by construction: only the even (symmetric) part of an impurity
 * couples to the even environment, and pairs of odd (antisymmetric) parts are
 * combined so that the result is invariant under the joint ket-bra swap.
 */
int ctm_rdm_2site(ctm_ctx* c, int x, int y, int dir, double* rho);

/* Energy per site of a nearest-neighbour Hamiltonian (Sec. III: the
 * Heisenberg model's energy is the benchmark observable): E = mean over the
 * sites of Tr(rho_h h) + Tr(rho_v h), rho the two-site RDMs above, for a bond
 * operator h (host, d^2 x d^2 row-major, read only).  Errors: CTM_E_ARG for
 * NULL pointers.  Synchronises. */
int ctm_energy(ctm_ctx* c, const double* h, double* e);

/* ---- complex tensors (Sec. II C) ---------------------------------------
 * For a complex A the double layer a = sum_s A[s] (x) conj(A[s]) is not swap
 * invariant, but in the eigenbasis of the swap its blocks of even total
 * parity are real and those of odd total parity imaginary (Sec. II C), and so
 * is every tensor of the contraction.  The library holds each such tensor as
 * two real block tensors (the real even-total blocks and the imaginary parts
 * of the odd-total blocks: the real representation with the extra leg of
 * dimension 2 and the multiplication rule f of Sec. II C) and multiplies them
 * with four half-size real block products where complex dense arithmetic
 * needs four full-size ones.  The truncation decomposes the real matrix
 * D^-1 M D, D = diag(i^parity), whose SVD gives that of M; every kept state is
 * then even.  Z2 form, 1 x 1 cell, directional moves and FP64 only; the RDMs
 * are Hermitian by construction.  ctm_step, ctm_converged,
 * ctm_corner_spectrum, ctm_record*, ctm_sector_dims, ctm_energy (real h),
 * ctm_timing and ctm_free apply as for a real tensor; ctm_rdm_1site/2site,
 * ctm_env_epsilon, ctm_s_err and ctm_log_kappa return CTM_E_ARG. */

/* Device bytes of a complex-tensor context (ctm_opts.workspace). */
int ctm_workspace_size_complex(int d, int D, int chi, const ctm_opts* o, size_t* bytes);

/* Create a context for the complex tensor A = A_re + i A_im (host, d*D^4
 * doubles each, legs [s,u,l,d,r], copied), whose double layer has the
 * real/imaginary block structure of Sec. II C.  Requires 1 <= d <= 8,
 * 1 <= D <= 8, 1 <= chi <= 4096, finite entries; ctm_opts as for ctm_init
 * with form CTM_FORM_Z2, a 1 x 1 cell, c4v = 0 and CTM_PREC_FP64 (else
 * CTM_E_ARG). */
int ctm_init_complex(ctm_ctx** out, const double* A_re, const double* A_im, int d, int D, int chi,
                     const ctm_opts* o);

/* Hermitian one-site RDM (Sec. II C; Hermitian by construction as Sec. II B
 * point (3) promises for the symmetric basis) of a complex-tensor context,
 * rho = rho_re + i rho_im
 * (host, d*d each, row-major), trace one: the entries on and above the
 * diagonal from the environment, the others their conjugates.  (x, y) must
 * be (0, 0).  Synchronises. */
int ctm_rdm_1site_complex(ctm_ctx* c, int x, int y, double* rho_re, double* rho_im);

/* Hermitian two-site RDM (Sec. II C, as ctm_rdm_1site_complex)
 * [(s1 s2)][(s1' s2')] of a complex-tensor context
 * (host, d^4 each), dir 0 horizontal, 1 vertical; (x, y) must be (0, 0).
 * Synchronises. */
int ctm_rdm_2site_complex(ctm_ctx* c, int x, int y, int dir, double* rho_re, double* rho_im);

/* Release everything; NULL is accepted.  (Resource handling of this
 * library; no passage of the paper.) */
void ctm_free(ctm_ctx* c);

/* Message of the last error on this context, or of the calling thread's last
 * failed ctm_init for NULL (never NULL).  (Error handling of this library;
 * no passage of the paper.) */
const char* ctm_last_error(const ctm_ctx* c);

/* ---- diagnostics used by the tests ------------------------------------ */

/* One-site environment of site (x, y) with the centre removed (Sec. III A),
 * back in the plain basis, normalised so that <eps, a> = 1; host, D^8
 * doubles ordered [U, L, Dn, R] with joined indices K = k*D + kbar. */
int ctm_env_epsilon(ctm_ctx* c, int x, int y, double* eps);

/* Hermitian symmetry error S_err = ||e - e^dag|| / ||e + e^dag|| (Sec. III A),
 * the largest over the sites. */
int ctm_s_err(ctm_ctx* c, double* s_err);

/* ln of the partition function per site of the double-layer network of
 * Sec. II A (Fig. 1), kappa = Z11 Z00 / (Z10 Z01) from the converged
 * environment: Z11 the 3x3 patch with the centre tensor, Z00 the four
 * corners alone, Z10 and Z01 the patches with one row or one column of
 * edges.  The paper prints no formula for it; this is the standard one.
 * 1 x 1 cell only (CTM_E_ARG otherwise).  Synchronises. */
int ctm_log_kappa(ctm_ctx* c, double* ln_kappa);

/* Number of truncations (the SVD cuts of Sec. II A) run so far, one per
 * cut: a move of an Lx x Ly cell truncates Lx*Ly cuts. */
int ctm_num_records(ctm_ctx* c, int* n);

/* Status bits of truncation m (the per-sector SVDs of Sec. II B point
 * (3)): 1 (2) the even (odd) sector's subspace
 * iteration reached its cap without passing the residual test, 4 the chi cut
 * split a near-degenerate multiplet (see ctm_svd_health). */
int ctm_record_status(ctm_ctx* c, int m, int* status);

/*
 * Record of truncation m (0-based, in the order run; Sec. II A truncation,
 * per sector as in Sec. II B point (3)): the kept singular
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
 * right, T4's down leg), its even and odd sizes (the Z2 sectors of
 * Sec. II B; the plain form reports all states as even). */
int ctm_sector_dims(ctm_ctx* c, int x, int y, int side, int* chi_even, int* chi_odd);

/* GPU seconds of the last ctm_step call per phase of the moves:
 * t[0] enlarged corners, t[1] half-system products and M, t[2] truncated SVD
 * (subspace iteration, Jacobi, selection), t[3] projectors, renormalisation
 * and normalisation, t[4] the corner spectra of the convergence test.
 * *n = 5. */
int ctm_timing(ctm_ctx* c, double* t, int cap, int* n);

/* Measurement of the block products whose cost Sec. III B compares (no
 * passage defines it).  Profile mode only (ctm_opts.profile = 1):
 * algorithmic FP64 GEMM flops
 * (2*M*N*K per block product), the summed durations in seconds of the GEMM
 * kernel launches (a HIP event right before and right after each) and their
 * number since the last reset; reset != 0 clears them (and the reduction
 * figures below). */
int ctm_gemm_stats(ctm_ctx* c, double* flops, double* seconds, long long* launches, int reset);

/* Measurement, as ctm_gemm_stats.  Profile mode only: the summed
 * durations and the number of the split-K
 * reductions that follow GEMM launches whose K was split over workgroups. */
int ctm_gemm_reduce_stats(ctm_ctx* c, double* seconds, long long* launches);

#ifdef __cplusplus
}
#endif

#endif /* HCTM_H */
