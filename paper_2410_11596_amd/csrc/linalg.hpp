// Small dense FP64 linear algebra used by the per-sector truncated SVD.
#pragma once
#include "hctm_internal.hpp"

namespace hctm {

struct SmallProb {
  double* a;       // matrix operated on (row-major, leading dim lda)
  double* b;       // Cholesky: R^-1 (ld ldb); Jacobi: accumulated right vectors (n x n) or null
  int m, n, lda, ldb;
  double rel;      // Cholesky: relative diagonal shift; Jacobi: orthogonality tolerance
  int max_sweeps;  // Jacobi only
  int* info;       // Cholesky: first failing pivot (1-based) or 0; Jacobi: sweeps (<0: no convergence)
  double* sv;      // Jacobi: singular values, descending
  int* perm;       // Jacobi: column of the j-th largest
  double* vlog;    // Jacobi: rotation log (jacobi_log_doubles), enables the LDS kernel with V
  int flags;       // Cholesky: 1 = factor the unit-diagonal Gram D^-1 G D^-1 (D = sqrt diag G);
                   // Rinv is then D^-1 R^-1 (sv must point to n doubles of scratch).
                   // Jacobi: kJacPairAbs = a pair of columns counts as orthogonal once
                   // |x_i . x_j| <= rel * max(|x_i|^2, |x_j|^2) (instead of rel |x_i| |x_j|)
  int pre;         // Jacobi (LDS kernel): the last pre columns are first orthogonalised among
                   // themselves (0: not); their sweep count goes to info[1]
  double* work;    // Jacobi: m*n doubles of device scratch (enables the L2 kernel for n <= 256)
};

// For the eigenvectors of a symmetric positive semi-definite X (X V = V L):
// one-sided Jacobi on X orthogonalises the columns of X V, whose norms are the
// eigenvalues, so relative orthogonality of two columns of very different
// norms lies below the rounding floor; measured against the larger of the two
// it is reached, and it bounds the mixing of two eigenvectors by about
// rel / (1 - (lambda_j / lambda_i)^2).
constexpr int kJacPairAbs = 2;

constexpr int kMaxSmall = 16;
struct SmallBatch {
  SmallProb p[kMaxSmall];
  int n;
};

struct SelectArgs {
  const double* sv0;
  const double* sv1;
  int n0, n1;    // trusted values per sector
  int chi;
  double tau;
  int* out_k;    // [k_even, k_odd]
  double* out_s; // [s_max, first discarded value or -1, last kept value]
  double* isq0;  // 1/sqrt(s) of the kept values, sector 0
  double* isq1;
  double* isv0;  // 1/s of the kept values
  double* isv1;
};

// corner spectra of one site: merge the two sector spectra of each corner,
// divide by the sum, pad to len; delta = max_c || new_c - old_c ||_2 (if
// have_old), or the maximum of that and the incoming *delta (accumulate)
struct SpecArgs {
  const double* sv[8];  // corner c sector P at sv[2c+P]
  int nsv[8];
  double* spec_new;     // 4 x len
  const double* spec_old;
  int len;
  int have_old;
  int accumulate;
  double* delta;
};
void corner_spectra_delta(const SpecArgs& a, hipStream_t s);

void fill(double* p, double v, size_t n, hipStream_t s);
// p[r * ld + c] *= alpha for r < rows, c < cols
void scale_block(double* p, int rows, int cols, long long ld, double alpha, hipStream_t s);
void random_fill(double* p, size_t n, uint64_t seed, hipStream_t s);
void norm2(const double* p, size_t n, double* out, double* part, hipStream_t s);
void sumsq(const double* p, size_t n, double* out, double* part, hipStream_t s);
void scale_inv(double* p, size_t n, const double* nrm, hipStream_t s);
void chol_inv(const std::vector<SmallProb>& probs, hipStream_t s);
void jacobi(const std::vector<SmallProb>& probs, hipStream_t s);
size_t jacobi_log_doubles(int n, int max_sweeps);
// out[0] = max_i |A_i - B_i|, out[1] = max_i |A_i| over the first k columns
// (n rows); out (two doubles) must be zero before
void col_resid(const double* A, int lda, const double* B, int ldb, int n, int k, double* out, hipStream_t s);
void gather_cols(const double* X, int ldx, const int* perm, const double* sv, int m, int k, double* U, int ldu,
                 hipStream_t s);
// out[c] = || GU[:, c] - lam[c] U[:, c] ||_2 for the first k columns (n rows, leading dim ld)
void ritz_resid(const double* GU, const double* U, const double* lam, int n, int ld, int k, double* out,
                hipStream_t s);
void select_states(const SelectArgs& a, hipStream_t s);

}  // namespace hctm
