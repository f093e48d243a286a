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
 * means B[n*ldb + k].  cscale may be NULL.  scratch (may be NULL): device
 * doubles the kernel may use to split a long K over several workgroups. */
int hctm_dev_gemm(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb, int ldc,
                  int ta, int tb, double alpha, double beta, const double* cscale, double* scratch,
                  long long scratch_doubles, void* stream);

/* op(A) op(B) (M x N, FP64) with a scattered output, the form the enlarged
 * corners use to write their product straight into a permuted layout: with
 * row = i0 T + i1 and col = i2 R + i3, element (row, col) of
 * alpha op(A) op(B) + beta C is stored at
 * C + i0 strides[0] + i1 strides[1] + i2 strides[2] + i3 strides[3]
 * (strides: host array of 4).  T must divide M and R divide N; the caller's
 * strides must map distinct elements to distinct addresses inside C. */
int hctm_dev_gemm_scatter(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb,
                          int ta, int tb, double alpha, double beta, int T, int R, const long long* strides,
                          void* stream);

/* The same with the operands rounded to FP32 and FP32 matrix-core products
 * and accumulation (CTM_PREC_FP32); C, alpha, beta and cscale stay FP64. */
int hctm_dev_gemm_f32(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb, int ldc,
                      int ta, int tb, double alpha, double beta, const double* cscale, double* scratch,
                      long long scratch_doubles, void* stream);

/* The same with BF16x3 split products (CTM_PREC_BF16X3). */
int hctm_dev_gemm_bf16x3(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb,
                         int ldc, int ta, int tb, double alpha, double beta, const double* cscale, double* scratch,
                         long long scratch_doubles, void* stream);

/* Probes of the chip's own ceilings (reported beside the published peaks;
 * measurement only, no passage of the paper).
 * hctm_dev_mfma_probe: blocks workgroups of four waves, each wave issuing
 * 32 * iters rounds of eight independent FP64 16 x 16 x 4 matrix-core products
 * with no memory traffic; sink (device, blocks * 256 doubles) receives the
 * sums so that the work is kept; *flops (host, may be NULL) = the flops
 * executed.  The caller times the launch on its stream.
 * hctm_dev_stream_probe: out[0..n) = in[0..n) (device, 16-byte aligned,
 * not overlapping) with 16-byte loads and stores; CTM_E_ARG if misaligned. */
int hctm_dev_mfma_probe(double* sink, int blocks, int iters, double* flops, void* stream);
int hctm_dev_stream_probe(const double* in, double* out, long long n, void* stream);

/* Strided copy of a dense box of rank r <= 6: out[sum x_j ostr_j] =
 * in[sum x_j istr_j] (the permute-and-reshape step between the block
 * products of Sec. II B). */
int hctm_dev_copy(const double* in, double* out, int r, const int* dims, const long long* istr,
                  const long long* ostr, void* stream);

/* CholeskyQR step of the truncated SVD (the SVD of Sec. II A, done per
 * sector as in Sec. II B point (3), by subspace iteration here):
 * Rinv = R^-1 with G + rel*max(diag G)*I = R^T R (R upper triangular);
 * G (n x n) is overwritten; info[0] = 0 unless a pivot was not positive. */
int hctm_dev_chol_inv(double* G, double* Rinv, int n, double rel, int* info, void* stream);

/* The small SVD of the truncation (Sec. II A, per sector as in Sec. II B
 * point (3)): one-sided Jacobi SVD of X (m x n, row-major, overwritten by U*Sigma in
 * column order); sv = singular values descending, perm = their columns,
 * sweeps[0] = sweeps used (negative: no convergence within max_sweeps).
 * If V is not NULL (X square), V (n x n, row-major) receives the product of
 * the rotations, so that X_in V = X_out; vlog then needs
 * hctm_dev_jacobi_log_doubles(n, max_sweeps) doubles of scratch.
 * pre (2 <= pre < n; else ignored): the last pre columns are first
 * orthogonalised among themselves, sweeps[1] = the sweeps of that phase
 * (sweeps then holds 2 ints).  The result is the same decomposition; only
 * the number of rotations changes.  work (m * n doubles, or NULL): device
 * scratch that lets blocks with 160 < n <= 256 or m * n > 19968 (m <= 256)
 * run with one wave per column pair on an L2-resident column-major copy;
 * without it such blocks take the slow global-memory kernel (which ignores
 * pre and vlog). */
int hctm_dev_jacobi(double* X, int m, int n, double tol, int max_sweeps, int pre, double* sv, int* perm,
                    int* sweeps, double* V, double* vlog, double* work, void* stream);

/* Scratch doubles needed by hctm_dev_jacobi's rotation log. */
long long hctm_dev_jacobi_log_doubles(int n, int max_sweeps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decomposition as hctm_dev_jacobi with vlog (when V is requested) and work
 * (when m, n <= 256) taken from a static device buffer of 4 Mi doubles
 * (32 MiB) that the library holds on every device it runs on; it allocates
 * nothing.  The caller passes the inputs and outputs as for hctm_dev_jacobi.
 * Returns CTM_E_ARG, before any work is enqueued, when the rotation log plus
 * the copy (hctm_dev_jacobi_log_doubles(n, max_sweeps) + m * n doubles)
 * exceed the buffer.  All calls on one device share that buffer and it keeps
 * the last call's contents (nothing in it needs to start at zero): calls
 * that may overlap on one device (different streams or host threads) race
 * and must be serialised by the caller. */
int hctm_dev_jacobi_noalloc(double* X, int m, int n, double tol, int max_sweeps, int pre, double* sv, int* perm,
                            int* sweeps, double* V, void* stream);

#ifdef __cplusplus
}
#endif

#endif
