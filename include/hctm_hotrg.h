/*
 * hctm_hotrg.h -- HOTRG on the double-layer network of a real iPEPS, in the
 * eigenbasis of the bra-ket swap (Z2 form) or in the plain basis.
 *
 * The paper treats HOTRG (higher-order tensor renormalisation group) beside
 * CTMRG and states that the Z2 structure of the rotated double layer carries
 * over to its steps (Sec. II A); it measures HOTRG's Hermitian symmetry error
 * with a probe tensor b (Sec. III A, Fig. 3) and its speed-up (Fig. 4(c),
 * (d)).  The steps are those of the standard method:
 *
 *  - A step joins two copies of the current tensor T[u,l,d,r] along the
 *    vertical bond, M[u,l1,l2,d,r1,r2] = sum_m T[u,l1,m,r1] T[m,l2,d,r2], and
 *    cuts the fused left legs (l1,l2) and right legs (r1,r2) back to chi with
 *    one isometry U: T'[u,x,d,y] = sum U[(l1 l2),x] M U[(r1 r2),y].
 *  - U holds the dominant eigenvectors of the Gram matrix of M with rows
 *    (l1,l2), or of the one with rows (r1,r2), whichever discards the smaller
 *    sum of eigenvalues (the left one on a tie, i.e. when the two differ by
 *    at most 1e-10 of their common trace ||M||_F^2).  Kept: min(chi,
 *    #{lambda > cutoff * lambda_max}) over the merged spectrum of both
 *    sectors, ties even first.  In the Z2 form the Gram matrices are block
 *    diagonal and each sector is decomposed on its own: up to 141 rows by
 *    one-sided Jacobi, larger sectors (up to 4096 rows) by subspace iteration
 *    with Rayleigh-Ritz (every third iteration) until the leading chi Ritz
 *    pairs have residuals below 1e-12 of the largest eigenvalue.
 *  - T' is divided by its Frobenius norm n_j and turned by a quarter turn
 *    (the right leg becomes the upper one), so that steps alternate between
 *    the two lattice directions.
 *  - After k steps T stands for a torus of 2^k sites:
 *    ln Z / N = ln n_0 + sum_j ln(n_j) / 2^j + ln(Tr T) / 2^k,
 *    Tr T = sum T[u,l,u,l], n_0 the norm of the initial double layer.
 *  - Symmetry probe (optional): one tensor of the network replaced by b
 *    (as a D^4 x D^4 matrix between the ket and the bra indices of
 *    [u,l,d,r]: +1 above the diagonal, -1 below) or by |b| (1 off the
 *    diagonal).  In each step the impurity is joined (above) with a pure
 *    tensor using the pure step's U and n_j.  The symmetry error is
 *    |Z_b| / Z_|b|.  b is odd under the bra-ket swap, so in the Z2 form it
 *    has only blocks of odd total parity and Z_b vanishes identically.
 *
 * Memory: the context allocates its device memory at hotrg_init (largest
 * buffers (max(chi, D^2))^5 doubles, two of them).  Errors are the CTM_E_*
 * codes of hctm.h; an error raised while GPU work ran poisons the context.
 * One context may be used by one host thread at a time.
 */
#ifndef HCTM_HOTRG_H
#define HCTM_HOTRG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hotrg_ctx hotrg_ctx;

typedef struct {
  int form;              /* CTM_FORM_Z2 (default) or CTM_FORM_DENSE */
  double svd_rel_cutoff; /* eigenvalues kept above cutoff * largest (default 1e-12) */
  int probes;            /* 1: carry the impurities b and |b| (hotrg_sym_error) */
  void* stream;          /* hipStream_t or NULL (a stream owned by the context) */
} hotrg_opts;

/* Fill *o with the defaults above. */
int hotrg_opts_default(hotrg_opts* o);

/*
 * Create a context: copies A (host, d*D^4 doubles, legs [s,u,l,d,r]) and
 * forms the double layer (Sec. II A, Fig. 1b; in the eigenbasis of the swap
 * in the Z2 form, Sec. II B) as the initial tensor, divided by its norm.  Requires 1 <= d <= 16, 1 <= D <= 6,
 * 1 <= chi, max(chi, D^2) <= 64; finite A.  *out is NULL on failure.
 */
int hotrg_init(hotrg_ctx** out, const double* A, int d, int D, int chi, const hotrg_opts* o);

/* Run n >= 0 coarse-graining steps (Sec. II A; per parity sector in the Z2
 * form, Sec. II B point (3)).  A step fails with CTM_E_ARG (before any GPU work of
 * that step) if a sector of a Gram matrix exceeds 4096 rows, the limit of
 * the eigensolver (only the plain form at chi = 64 reaches it exactly), and
 * with CTM_E_NUMERIC (context poisoned) if the Jacobi step of a Rayleigh-Ritz
 * projection does not converge.  A Gram sector whose rank is below the
 * subspace block is not an error: its missing directions have eigenvalue
 * zero and fall below the cutoff. */
int hotrg_step(hotrg_ctx* c, int n);

/* ln Z per site of the torus of 2^k sites after k steps (the formula in the
 * file comment; the paper prints none, it is the standard one).
 * Synchronises. */
int hotrg_log_z(hotrg_ctx* c, double* lnz);

/* Probe mode only (the symmetry probe of Sec. III A, Fig. 3):
 * z_b = Z_b / Z, z_abs = Z_|b| / Z and err = |z_b| / |z_abs| (any pointer
 * may be NULL).  Synchronises. */
int hotrg_sym_error(hotrg_ctx* c, double* err, double* z_b, double* z_abs);

/*
 * Bond energy (Sec. III: the Heisenberg model's energy is the observable the
 * paper reports): h (host, d^2 x d^2 doubles, row-major, h[(s1 s2),(s1' s2')],
 * site 1 above site 2 on a vertical bond, ket indices s, bra indices s') is
 * written as sum_{a,b} |a><b| (x) O_ab with O_ab[s2,s2'] = h[(a s2),(b s2')]
 * (in the Z2 form regrouped into symmetric and antisymmetric pairs, the
 * mixed ones vanishing); every term puts the impurities
 * a[O] = sum O[s,s'] A[s] (x) A[s'] on two vertically adjacent sites, joined
 * in the first step and carried like the probes.  Must be called before the
 * first step; d <= 4.  A second call replaces the operator.
 */
int hotrg_set_bond(hotrg_ctx* c, const double* h);

/* <h> on a vertical bond after at least one step (hotrg_set_bond first).
 * Synchronises. */
int hotrg_energy(hotrg_ctx* c, double* e);

/*
 * One-site RDM (Hermitian by construction in the Z2 form, Sec. II B point
 * (3)): carries the impurities a[|s><s'|] (in the Z2 form only the
 * symmetric parts (|s><s'| + |s'><s|)/2, s <= s', whose double layers are
 * even: the RDM is symmetric by construction).  Must be called before the
 * first step; d <= 4.
 */
int hotrg_track_rdm1(hotrg_ctx* c);

/* rho[s][s'] (host, d*d), trace one, after hotrg_track_rdm1.  Synchronises. */
int hotrg_rdm1(hotrg_ctx* c, double* rho);

/* Number of steps run (one truncation each, Sec. II A). */
int hotrg_num_records(hotrg_ctx* c, int* n);

/*
 * Step i: the kept eigenvalues (merged, descending, divided by the largest;
 * at most cap written, *n the full count), kept states per sector (plain
 * form: all in k_even), side = 0 if the left Gram matrix gave U, 1 the right;
 * discarded[0..1] = discarded weight of the left and the right one.
 */
int hotrg_record(hotrg_ctx* c, int i, double* spectrum, int cap, int* n, int* k_even, int* k_odd, int* side,
                 double* discarded);

/* Last error message of c (or of the calling thread's last failed init for
 * NULL).  (Error handling of this library; no passage of the paper.) */
const char* hotrg_last_error(const hotrg_ctx* c);

/* Release everything; NULL is accepted.  (Resource handling; no passage.) */
void hotrg_free(hotrg_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* HCTM_HOTRG_H */
