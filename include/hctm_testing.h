/*
 * hctm_testing.h -- kernel-level entry points of libhctm.so, exported so that
 * the tests can check each building block of the CTMRG move on its own.
 * All pointers are device pointers; stream is a hipStream_t (NULL = the
 * default stream).  Each call only enqueues work and returns CTM_OK (0) or
 * CTM_E_ARG / CTM_E_HIP; callers synchronise the stream themselves.
 */
#ifndef HCTM_TESTING_H
#define HCTM_TESTING_H

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha * op(A) op(B) * diag(cscale) + beta * C, FP64 on the matrix
 * cores (the block products of Sec. II B).  Row-major storage: ta = 0 means
 * A[m*lda + k], ta = 1 means A[k*lda + m]; tb = 0 means B[k*ldb + n], tb = 1
 * means B[n*ldb + k].  cscale may be NULL. */
int hctm_dev_gemm(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb, int ldc,
                  int ta, int tb, double alpha, double beta, const double* cscale, void* stream);

/* Strided copy of a dense box of rank r <= 6: out[sum x_j ostr_j] =
 * in[sum x_j istr_j] (the permute-and-reshape step between block products). */
int hctm_dev_copy(const double* in, double* out, int r, const int* dims, const long long* istr,
                  const long long* ostr, void* stream);

/* Rinv = R^-1 with G + rel*max(diag G)*I = R^T R (R upper triangular);
 * G (n x n) is overwritten; info[0] = 0 unless a pivot was not positive. */
int hctm_dev_chol_inv(double* G, double* Rinv, int n, double rel, int* info, void* stream);

/* One-sided Jacobi SVD of X (m x n, row-major, overwritten by U*Sigma in
 * column order); sv = singular values descending, perm = their columns,
 * sweeps[0] = sweeps used (negative: no convergence within max_sweeps). */
int hctm_dev_jacobi(double* X, int m, int n, double tol, int max_sweeps, double* sv, int* perm, int* sweeps,
                    void* stream);

#ifdef __cplusplus
}
#endif

#endif
