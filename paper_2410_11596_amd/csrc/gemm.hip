// FP64 grouped GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
// Every contraction of the method is a dense product of parity blocks (the
// cost model of Sec. II B: two half-size block products instead of one full
// product).  One launch takes a list of independent problems; the grid is the
// concatenation of their output tiles.
//
// Tile: 128 x 128 per workgroup of 256 threads (4 wave64), K step 16, each
// wave owns a 64 x 64 sub-tile = 4 x 4 MFMA 16x16 accumulators.  Operands are
// staged through LDS in k-major order so that one MFMA fragment read is a
// contiguous 128-byte row per 16 lanes.  Loads for step k+1 are issued into
// registers before the MFMAs of step k.
//
// MFMA 16x16x4 f64 operand layout (measured on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; its four accumulator values are
// D[l / 16 + 4 * v][l % 16], v = 0..3.
#include "hctm_internal.hpp"

namespace hctm {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int NT = 256;
constexpr int LDA_S = BM + 4;   // LDS row pitch (doubles), padded
constexpr int LDB_S = BN + 4;
constexpr int kMaxGroup = 16;

struct Prob {
  const double* A;
  const double* B;
  double* C;
  const double* cscale;
  const double* rscale;
  double alpha, beta;
  int M, N, K, lda, ldb, ldc, ta, tb;
  int tiles_n, tile_start;
};

struct Group {
  Prob p[kMaxGroup];
  int n;
  int total;
};

// Load a BK x BM slab of op(A) (k-major) into registers: 8 doubles per thread.
__device__ __forceinline__ void load_tile(const double* __restrict__ X, int ld, int trans, int rows, int K,
                                          int r0, int k0, double (&reg)[8]) {
  const int t = threadIdx.x;
  if (!trans) {
    // X[r][k], k contiguous: thread -> row r0 + t/2, k = k0 + (t%2)*8 .. +8
    const int r = r0 + (t >> 1);
    const int kb = k0 + (t & 1) * 8;
    const double* src = X + (long long)r * ld + kb;
    const bool rok = r < rows;
    if (rok && kb + 8 <= K && ((((uintptr_t)src) & 15) == 0)) {
      const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double2 v = s2[i];
        reg[2 * i] = v.x;
        reg[2 * i + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) reg[i] = (rok && kb + i < K) ? src[i] : 0.0;
    }
  } else {
    // X[k][r], r contiguous: thread -> k = k0 + t/16, r = r0 + (t%16)*8 .. +8
    const int k = k0 + (t >> 4);
    const int rb = r0 + (t & 15) * 8;
    const double* src = X + (long long)k * ld + rb;
    const bool kok = k < K;
    if (kok && rb + 8 <= rows && ((((uintptr_t)src) & 15) == 0)) {
      const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double2 v = s2[i];
        reg[2 * i] = v.x;
        reg[2 * i + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) reg[i] = (kok && rb + i < rows) ? src[i] : 0.0;
    }
  }
}

__device__ __forceinline__ void store_tile(double* __restrict__ S, int pitch, int trans, const double (&reg)[8]) {
  const int t = threadIdx.x;
  if (!trans) {
    const int r = t >> 1;
    const int kb = (t & 1) * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) S[(kb + i) * pitch + r] = reg[i];
  } else {
    const int k = t >> 4;
    const int rb = (t & 15) * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) S[k * pitch + rb + i] = reg[i];
  }
}

__global__ __launch_bounds__(NT, 2) void gemm_f64_kernel(Group g) {
  __shared__ double As[BK * LDA_S];
  __shared__ double Bs[BK * LDB_S];

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
  const int tile = b - P.tile_start;
  const int tm = tile / P.tiles_n, tn = tile % P.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int li = lane & 15, lk = lane >> 4;

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  double ra[8], rb[8];
  load_tile(P.A, P.lda, P.ta, P.M, P.K, m0, 0, ra);
  // B is stored [k][n] (tb=0, n contiguous) or [n][k] (tb=1): the roles of
  // the two layouts are swapped with respect to A.
  load_tile(P.B, P.ldb, !P.tb, P.N, P.K, n0, 0, rb);
  store_tile(As, LDA_S, P.ta, ra);
  store_tile(Bs, LDB_S, !P.tb, rb);
  __syncthreads();

#pragma unroll 1
  for (int k0 = 0; k0 < P.K; k0 += BK) {
    const bool more = k0 + BK < P.K;
    if (more) {
      load_tile(P.A, P.lda, P.ta, P.M, P.K, m0, k0 + BK, ra);
      load_tile(P.B, P.ldb, !P.tb, P.N, P.K, n0, k0 + BK, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[(kk + lk) * LDA_S + wm + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[(kk + lk) * LDB_S + wn + j * 16 + li];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      store_tile(As, LDA_S, P.ta, ra);
      store_tile(Bs, LDB_S, !P.tb, rb);
    }
    __syncthreads();
  }

  // epilogue: lane holds D[lk + 4*v][li] of every 16x16 tile
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn + j * 16 + li;
      if (col >= P.N) continue;
      const double cs = P.cscale ? P.cscale[col] : 1.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + i * 16 + lk + 4 * v;
        if (row >= P.M) continue;
        double val = P.alpha * acc[i][j][v] * cs;
        if (P.rscale) val *= P.rscale[row];
        double* c = P.C + (long long)row * P.ldc + col;
        if (P.beta != 0.0) val += P.beta * *c;
        *c = val;
      }
    }
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

}  // namespace

void gemm(const std::vector<GemmDesc>& probs, hipStream_t s) {
  Group g;
  g.n = 0;
  g.total = 0;
  auto flush = [&]() {
    if (g.n == 0) return;
    hipLaunchKernelGGL(gemm_f64_kernel, dim3(g.total), dim3(NT), 0, s, g);
    HCTM_HIP(hipGetLastError());
    g.n = 0;
    g.total = 0;
  };
  for (const GemmDesc& d : probs) {
    if (d.M <= 0 || d.N <= 0) continue;
    if (d.K <= 0) {
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
    p.tiles_n = (d.N + BN - 1) / BN;
    p.tile_start = g.total;
    g.total += ((d.M + BM - 1) / BM) * p.tiles_n;
    g.n++;
  }
  flush();
}

}  // namespace hctm
