// FP64 grouped GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// Every contraction of the method is a dense product of parity blocks (the
// cost model of Sec. II B: two half-size block products instead of one full
// product).  One launch takes a list of independent problems; the grid is the
// concatenation of their output tiles (and K slices).
//
// Tile: BM x BN per workgroup of 256 threads (4 wave64 in a 2 x 2 layout),
// K step 16.  128 x 64 (FP64; 128 x 128 for the FP32 and BF16x3 products)
// for the large block products; 64 x 64 when the
// problems are too small to fill the 256 CUs; and when the 64 x 64 tiles are
// too few (the tall n x l products and the l x l Gram matrices of the
// subspace iteration) the K range is split over several workgroups, about
// four per CU in all, whose partial tiles are summed in a fixed order by a
// second kernel with one thread per output element (deterministic, no
// atomics).  Operands are
// staged through LDS in k-major order so that one MFMA fragment read is a
// contiguous row per 16 lanes; loads for step k+1 are issued into registers
// before the MFMAs of step k.
//
// MFMA 16x16x4 operand layout (measured on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; its four accumulator values are
// D[l / 16 + 4 * v][l % 16] (FP64) or D[4 * (l / 16) + v][l % 16] (FP32),
// v = 0..3.  The same kernel runs with FP32 operands in LDS and FP32 MFMAs
// (CTM_PREC_FP32); the epilogue is FP64 either way.
#include <algorithm>

#include "hctm_internal.hpp"

namespace hctm {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BK = 16;
constexpr int NT = 256;
constexpr int kMaxGroup = 16;

struct Prob {
  const double* A;
  const double* B;
  double* C;
  const double* cscale;
  const double* rscale;
  double* part;  // split-K partial tiles (ksplit x M x N), null if ksplit == 1
  double alpha, beta;
  int M, N, K, lda, ldb, ldc, ta, tb;
  int tiles_m, tiles_n, ksplit, kchunk, tile_start;
  // scattered output (GemmDesc); sc_rn == 0: row-major C with ldc
  int sc_rn, sc_cn;
  int sc_rd[2], sc_cd[2];
  long long sc_rs[3], sc_cs[3];
};

// offset of index x of a run of n legs (row-major, sizes of all but the
// first in d) with strides s
__device__ __forceinline__ long long leg_offset(int x, int n, const int* d, const long long* s) {
  if (n == 1) return (long long)x * s[0];
  if (n == 2) {
    const int q = x / d[0];
    return (long long)q * s[0] + (long long)(x - q * d[0]) * s[1];
  }
  const int q = x / d[1];
  const int i0 = q / d[0];
  return (long long)i0 * s[0] + (long long)(q - i0 * d[0]) * s[1] + (long long)(x - q * d[1]) * s[2];
}

struct Group {
  Prob p[kMaxGroup];
  int n;
  int total;
};
static_assert(sizeof(Group) <= 4096, "a launch's problem list must fit the kernel arguments");

// Load a BK x ROWS slab of op(X) (k-major) into registers.
template <int ROWS>
__device__ __forceinline__ void load_tile(const double* __restrict__ X, int ld, int trans, int rows, int kend,
                                          int r0, int k0, double (&reg)[ROWS * BK / NT]) {
  constexpr int PER = ROWS * BK / NT;
  const int t = threadIdx.x;
  if (!trans) {
    // X[r][k], k contiguous
    constexpr int TPR = BK / PER;
    const int r = r0 + t / TPR;
    const int kb = k0 + (t % TPR) * PER;
    const double* src = X + (long long)r * ld + kb;
    const bool rok = r < rows;
    if (rok && kb + PER <= kend && ((((uintptr_t)src) & 15) == 0)) {
      const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
      for (int i = 0; i < PER / 2; ++i) {
        double2 v = s2[i];
        reg[2 * i] = v.x;
        reg[2 * i + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i) reg[i] = (rok && kb + i < kend) ? src[i] : 0.0;
    }
  } else {
    // X[k][r], r contiguous: 16 threads per k row
    const int k = k0 + t / 16;
    const int rb = r0 + (t % 16) * PER;
    const double* src = X + (long long)k * ld + rb;
    const bool kok = k < kend;
    if (kok && rb + PER <= rows && ((((uintptr_t)src) & 15) == 0)) {
      const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
      for (int i = 0; i < PER / 2; ++i) {
        double2 v = s2[i];
        reg[2 * i] = v.x;
        reg[2 * i + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i) reg[i] = (kok && rb + i < rows) ? src[i] : 0.0;
    }
  }
}

template <int ROWS, typename CT>
__device__ __forceinline__ void store_tile(CT* __restrict__ S, int trans, const double (&reg)[ROWS * BK / NT]) {
  constexpr int PER = ROWS * BK / NT;
  constexpr int PITCH = ROWS + 4;
  const int t = threadIdx.x;
  if (!trans) {
    constexpr int TPR = BK / PER;
    const int r = t / TPR;
    const int kb = (t % TPR) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) S[(kb + i) * PITCH + r] = (CT)reg[i];
  } else {
    const int k = t / 16;
    const int rb = (t % 16) * PER;
#pragma unroll
    for (int i = 0; i < PER; ++i) S[k * PITCH + rb + i] = (CT)reg[i];
  }
}

typedef float v4f __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 in the compute type: FP64 (v_mfma_f64_16x16x4f64) or FP32
// (v_mfma_f32_16x16x4f32, FP32 products and accumulation); both take one
// element of A and of B per lane and give four accumulator values per lane
template <typename CT>
struct Mfma;
// Accumulator value v of lane (lk = l / 16, l % 16) holds row row(lk, v) of
// the 16 x 16 block (measured on gfx950: lk + 4v for FP64, 4 lk + v for FP32).
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ v4d op(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ v4f op(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

// BF16x3: x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to
// nearest even); the MFMA v_mfma_f32_16x16x16bf16 takes four consecutive k
// per lane: lane l supplies A[l % 16][4 (l / 16) + q] and B[4 (l / 16) + q][l % 16],
// q = 0..3, and holds D[4 (l / 16) + v][l % 16] as the FP32 MFMA does.
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rn(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ float bf16_to_float(short h) {
  return __uint_as_float(((unsigned)(unsigned short)h) << 16);
}

__device__ __forceinline__ void split_bf16(float x, short& hi, short& lo) {
  hi = bf16_rn(x);
  lo = bf16_rn(x - bf16_to_float(hi));
}

// One output tile of the grouped GEMM; CT = type of the staged operands and
// of the MFMA (the output is FP64 either way); SPLIT (with CT = float): the
// BF16x3 products.
template <int BM, int BN, typename CT, bool SPLIT = false>
__device__ __forceinline__ void gemm_tile(const Group& g, CT* As, CT* Bs) {
  constexpr int PA = BM + 4, PB = BN + 4;
  constexpr int WM = BM / 2, WN = BN / 2;  // per-wave sub-tile
  constexpr int TI = WM / 16, TJ = WN / 16;
  typedef typename Mfma<CT>::acc_t acc_t;

  // XCD-aware order: blocks are dealt to the 8 XCDs round robin; give each
  // XCD a contiguous range of tiles so that neighbouring tiles share its L2.
  int b = blockIdx.x;
  const int T = g.total;
  const int full = (T / 8) * 8;
  if (b < full) b = (b & 7) * (T / 8) + (b >> 3);

  int pi = 0;
#pragma unroll 1
  for (int i = 1; i < g.n; ++i)
    if (b >= g.p[i].tile_start) pi = i;
  const Prob& P = g.p[pi];
  int tile = b - P.tile_start;
  const int ks = tile % P.ksplit;
  tile /= P.ksplit;
  const int tm = tile / P.tiles_n, tn = tile % P.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = ks * P.kchunk;
  const int kend = min(P.K, kbeg + P.kchunk);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int li = lane & 15, lk = lane >> 4;

  acc_t acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  double ra[BM * BK / NT], rb[BN * BK / NT];
  load_tile<BM>(P.A, P.lda, P.ta, P.M, kend, m0, kbeg, ra);
  // B is stored [k][n] (tb=0, n contiguous) or [n][k] (tb=1): the roles of
  // the two layouts are swapped with respect to A.
  load_tile<BN>(P.B, P.ldb, !P.tb, P.N, kend, n0, kbeg, rb);
  store_tile<BM>(As, P.ta, ra);
  store_tile<BN>(Bs, !P.tb, rb);
  __syncthreads();

#pragma unroll 1
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      load_tile<BM>(P.A, P.lda, P.ta, P.M, kend, m0, k0 + BK, ra);
      load_tile<BN>(P.B, P.ldb, !P.tb, P.N, kend, n0, k0 + BK, rb);
    }
    if constexpr (SPLIT) {
      // one BF16 MFMA covers the 16 k of the slab: lane takes k = 4 lk + q
      static_assert(BK == 16, "one BF16 MFMA per K step");
      v4s ah[TI], al[TI], bh[TJ], bl[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          short h, l;
          split_bf16(As[(4 * lk + q) * PA + wm + i * 16 + li], h, l);
          ah[i][q] = h;
          al[i][q] = l;
        }
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          short h, l;
          split_bf16(Bs[(4 * lk + q) * PB + wn + j * 16 + li], h, l);
          bh[j][q] = h;
          bl[j][q] = l;
        }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          // the small terms first
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        CT af[TI], bf[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i) af[i] = As[(kk + lk) * PA + wm + i * 16 + li];
#pragma unroll
        for (int j = 0; j < TJ; ++j) bf[j] = Bs[(kk + lk) * PB + wn + j * 16 + li];
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) acc[i][j] = Mfma<CT>::op(af[i], bf[j], acc[i][j]);
      }
    }
    __syncthreads();
    if (more) {
      store_tile<BM>(As, P.ta, ra);
      store_tile<BN>(Bs, !P.tb, rb);
    }
    __syncthreads();
  }

  // epilogue: lane holds D[row(lk, v)][li] of every 16x16 tile
  if (P.ksplit > 1) {
    double* part = P.part + (long long)ks * P.M * P.N;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const int col = n0 + wn + j * 16 + li;
        if (col >= P.N) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = m0 + wm + i * 16 + Mfma<CT>::row(lk, v);
          if (row < P.M) part[(long long)row * P.N + col] = (double)acc[i][j][v];
        }
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i) {
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int col = n0 + wn + j * 16 + li;
      if (col >= P.N) continue;
      const double cs = P.cscale ? P.cscale[col] : 1.0;
      // column part of the output address
      const long long cpart = P.sc_rn ? leg_offset(col, P.sc_cn, P.sc_cd, P.sc_cs) : col;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + i * 16 + Mfma<CT>::row(lk, v);
        if (row >= P.M) continue;
        double val = P.alpha * (double)acc[i][j][v] * cs;
        if (P.rscale) val *= P.rscale[row];
        const long long rpart = P.sc_rn ? leg_offset(row, P.sc_rn, P.sc_rd, P.sc_rs) : (long long)row * P.ldc;
        double* c = P.C + rpart + cpart;
        if (P.beta != 0.0) val += P.beta * *c;
        *c = val;
      }
    }
  }
}

template <int BM, int BN>
__global__ __launch_bounds__(NT, 2) void gemm_f64_kernel(Group g) {
  __shared__ double As[BK * (BM + 4)];
  __shared__ double Bs[BK * (BN + 4)];
  gemm_tile<BM, BN, double>(g, As, Bs);
}

template <int BM, int BN>
__global__ __launch_bounds__(NT, 2) void gemm_f32_kernel(Group g) {
  __shared__ float As[BK * (BM + 4)];
  __shared__ float Bs[BK * (BN + 4)];
  gemm_tile<BM, BN, float>(g, As, Bs);
}

template <int BM, int BN>
__global__ __launch_bounds__(NT, 2) void gemm_bf16x3_kernel(Group g) {
  __shared__ float As[BK * (BM + 4)];
  __shared__ float Bs[BK * (BN + 4)];
  gemm_tile<BM, BN, float, true>(g, As, Bs);
}

// Sum the K slices of split problems in slice order and apply the epilogue.
__global__ void splitk_reduce_kernel(Group g) {
  const Prob& P = g.p[blockIdx.y];
  if (P.ksplit <= 1) return;
  const long long n = (long long)P.M * P.N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < P.ksplit; ++k) s += P.part[(long long)k * n + e];
    const int row = (int)(e / P.N), col = (int)(e % P.N);
    double val = P.alpha * s;
    if (P.cscale) val *= P.cscale[col];
    if (P.rscale) val *= P.rscale[row];
    double* c = P.C + (long long)row * P.ldc + col;
    if (P.beta != 0.0) val += P.beta * *c;
    *c = val;
  }
}

// C = beta * C for problems with K == 0 (nothing to multiply).
__global__ void scale_c_kernel(double* C, int M, int N, int ldc, double beta) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)M * N) return;
  const int r = (int)(idx / N), c = (int)(idx % N);
  double* p = C + (long long)r * ldc + c;
  *p = beta == 0.0 ? 0.0 : beta * *p;
}

long long tiles(const GemmDesc& d, int bm, int bn) {
  return (long long)((d.M + bm - 1) / bm) * ((d.N + bn - 1) / bn);
}

}  // namespace

namespace {
void gemm_one_type(const std::vector<GemmDesc>& probs, int prec, hipStream_t s, double* scratch,
                   long long scratch_cap, GemmObserver* obs) {
  // tile shape for the whole call, from how many workgroups it yields: the
  // large tile when it alone fills the chip (FP64: 128 x 64, measured faster
  // than 128 x 128 on the 2592^3 to 8192^3 block products, 55-65 against
  // 46-59 TFLOP/s; FP32 and BF16x3: 128 x 128), else 64 x 64
  constexpr long long kFill = 240;  // about one workgroup per CU
  const int big_n = prec == 0 ? 64 : 128;
  long long tbig = 0, t64 = 0;
  for (const GemmDesc& d : probs)
    if (d.M > 0 && d.N > 0 && d.K > 0) {
      tbig += tiles(d, 128, big_n);
      t64 += tiles(d, 64, 64);
    }
  const int cfg = tbig >= kFill ? 0 : 1;  // 0: 128 x big_n, 1: 64 x 64
  const int bm = cfg == 0 ? 128 : 64, bn = cfg == 0 ? big_n : 64;
  long long part_used = 0;

  Group g;
  g.n = 0;
  g.total = 0;
  bool any_split = false;
  long long split_mn = 0;
  auto flush = [&]() {
    if (g.n == 0) return;
    double f = 0.0;
    for (int i = 0; i < g.n; ++i) f += 2.0 * g.p[i].M * g.p[i].N * (double)g.p[i].K;
    if (obs) obs->mark(0, 0, f);
    if (prec == 0 && cfg == 0)
      hipLaunchKernelGGL((gemm_f64_kernel<128, 64>), dim3(g.total), dim3(NT), 0, s, g);
    else if (prec == 0)
      hipLaunchKernelGGL((gemm_f64_kernel<64, 64>), dim3(g.total), dim3(NT), 0, s, g);
    else if (prec == 1 && cfg == 0)
      hipLaunchKernelGGL((gemm_f32_kernel<128, 128>), dim3(g.total), dim3(NT), 0, s, g);
    else if (prec == 1)
      hipLaunchKernelGGL((gemm_f32_kernel<64, 64>), dim3(g.total), dim3(NT), 0, s, g);
    else if (cfg == 0)
      hipLaunchKernelGGL((gemm_bf16x3_kernel<128, 128>), dim3(g.total), dim3(NT), 0, s, g);
    else
      hipLaunchKernelGGL((gemm_bf16x3_kernel<64, 64>), dim3(g.total), dim3(NT), 0, s, g);
    HCTM_HIP(hipGetLastError());
    if (obs) obs->mark(0, 1, f);
    if (any_split) {
      // one thread per output element of the largest split problem
      const unsigned gx = (unsigned)std::min<long long>(2048, (split_mn + 255) / 256);
      if (obs) obs->mark(1, 0, 0.0);
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3(gx, g.n), dim3(256), 0, s, g);
      HCTM_HIP(hipGetLastError());
      if (obs) obs->mark(1, 1, 0.0);
    }
    g.n = 0;
    g.total = 0;
    part_used = 0;
    any_split = false;
    split_mn = 0;
  };
  for (const GemmDesc& d : probs) {
    if (d.M <= 0 || d.N <= 0) continue;
    if (d.K <= 0) {
      if (d.sc_rn > 0) throw Error(1, "gemm: a scattered output needs K > 0");
      const long long n = (long long)d.M * d.N;
      hipLaunchKernelGGL(scale_c_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d.C, d.M, d.N, d.ldc,
                         d.beta);
      HCTM_HIP(hipGetLastError());
      continue;
    }
    if (g.n == kMaxGroup) flush();
    Prob& p = g.p[g.n];
    p.A = d.A;
    p.B = d.B;
    p.C = d.C;
    p.cscale = d.cscale;
    p.rscale = d.rscale;
    p.alpha = d.alpha;
    p.beta = d.beta;
    p.M = d.M;
    p.N = d.N;
    p.K = d.K;
    p.lda = d.lda;
    p.ldb = d.ldb;
    p.ldc = d.ldc;
    p.ta = d.ta;
    p.tb = d.tb;
    p.tiles_m = (d.M + bm - 1) / bm;
    p.tiles_n = (d.N + bn - 1) / bn;
    const bool sc = d.sc_rn >= 1 && d.sc_rn <= 3 && d.sc_cn >= 1 && d.sc_cn <= 3;
    if (d.sc_rn != 0 && !sc) throw Error(1, "gemm: a scattered output takes one to three legs each side");
    p.sc_rn = sc ? d.sc_rn : 0;
    p.sc_cn = sc ? d.sc_cn : 0;
    for (int q = 0; q < 2; ++q) {
      p.sc_rd[q] = d.sc_rd[q];
      p.sc_cd[q] = d.sc_cd[q];
    }
    for (int q = 0; q < 3; ++q) {
      p.sc_rs[q] = d.sc_rs[q];
      p.sc_cs[q] = d.sc_cs[q];
    }
    // split K when the call has too few output tiles and this K is long
    int ks = 1;
    if (cfg == 1 && t64 < 4 * kFill && scratch && !p.sc_rn) {
      const long long want = (4 * kFill + t64 - 1) / t64;  // about 4 workgroups per CU
      const long long maxk = d.K / 64;  // at least 64 of K per slice
      ks = (int)std::max<long long>(1, std::min(want, maxk));
      while (ks > 1 && part_used + (long long)ks * d.M * d.N > scratch_cap) --ks;
    }
    p.ksplit = ks;
    p.kchunk = ks > 1 ? (((d.K + ks - 1) / ks + BK - 1) / BK) * BK : d.K;
    if (ks > 1) {
      p.ksplit = (d.K + p.kchunk - 1) / p.kchunk;
      p.part = scratch + part_used;
      part_used += (long long)p.ksplit * d.M * d.N;
      any_split = true;
      split_mn = std::max(split_mn, (long long)d.M * d.N);
    } else {
      p.part = nullptr;
    }
    p.tile_start = g.total;
    g.total += p.tiles_m * p.tiles_n * p.ksplit;
    g.n++;
  }
  flush();
}
}  // namespace

void gemm(const std::vector<GemmDesc>& probs, hipStream_t s, double* scratch, long long scratch_cap,
          GemmObserver* obs) {
  // problems of different arithmetic go to separate launches (all problems
  // of one call are independent)
  std::vector<GemmDesc> by[3];
  for (const GemmDesc& d : probs) by[(d.prec >= 0 && d.prec <= 2) ? d.prec : 0].push_back(d);
  for (int p = 0; p < 3; ++p)
    if (!by[p].empty()) gemm_one_type(by[p], p, s, scratch, scratch_cap, obs);
}

}  // namespace hctm
