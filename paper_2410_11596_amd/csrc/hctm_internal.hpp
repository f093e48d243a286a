// Internal interfaces of the HIP implementation (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace hctm {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HCTM_HIP(x)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw ::hctm::Error(3, std::string(#x) + " failed: " + hipGetErrorString(e_));    \
  } while (0)

// ----------------------------------------------------------------- GEMM ----
// C = alpha * op(A) op(B) * diag(cscale) + beta * C, all FP64, row-major
// storage with leading dimensions.  ta = 0: A[m*lda + k]; ta = 1: A[k*lda + m].
// tb = 0: B[k*ldb + n]; tb = 1: B[n*ldb + k].  cscale may be null.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int lda, ldb, ldc;
  int ta, tb;
  double alpha, beta;
  const double* cscale;
  const double* rscale;  // optional per-row scale of the product
  int prec;              // 0: FP64; 1: operands rounded to FP32, FP32 MFMA and accumulation;
                         // 2: BF16x3 (operands split into BF16 hi + lo, hi*hi + hi*lo + lo*hi
                         //    on BF16 MFMA with FP32 accumulation)
  // Optional scattered output (sc_rn > 0): the rows of the product are sc_rn
  // legs (row-major; the sizes of all but the first in sc_rd) and the columns
  // sc_cn legs (sizes in sc_cd), each of one to three; element (row, col) is
  // stored at C + sum of leg index * stride (sc_rs, sc_cs; ldc unused).  So a
  // product is written straight into a layout with its legs permuted.  Such
  // a product is not split over K and must have K > 0.
  int sc_rn, sc_cn;
  int sc_rd[2], sc_cd[2];
  long long sc_rs[3], sc_cs[3];
};
// Optional observer of the kernels gemm() launches, called on the host right
// before (phase 0) and after (phase 1) each launch: kind 0 a GEMM kernel
// (flops = algorithmic 2 M N K of its problems), kind 1 a split-K reduction.
struct GemmObserver {
  virtual void mark(int kind, int phase, double flops) = 0;
  virtual ~GemmObserver() = default;
};
// scratch (optional): device doubles for split-K partial tiles.
void gemm(const std::vector<GemmDesc>& probs, hipStream_t s, double* scratch = nullptr, long long scratch_cap = 0,
          GemmObserver* obs = nullptr);

// ---------------------------------------------------------------- probes ----
// FP64 MFMA issue probe: blocks workgroups of four waves, 32 * iters rounds
// of eight independent 16 x 16 x 4 products each; sink gets blocks * 256
// doubles.  Returns the flops it executes.
double mfma_probe(double* sink, int blocks, int iters, hipStream_t s);
// out[0..n) = in[0..n) with 16-byte accesses (in and out 16-byte aligned).
void stream_probe(const double* in, double* out, long long n, hipStream_t s);

// -------------------------------------------------------------- permute ----
// Strided copy of one dense block: out[sum_j x_j ostr_j] = in[sum_j x_j istr_j]
// for x in the box dims[0..r).  Used for every leg permutation of a
// block-sparse tensor (one job per parity block).
constexpr int kMaxRank = 6;
struct CopyJob {
  const double* in;
  double* out;
  int r;
  int dims[kMaxRank];
  long long istr[kMaxRank];
  long long ostr[kMaxRank];
};
void copy_jobs(const std::vector<CopyJob>& jobs, hipStream_t s);

}  // namespace hctm
