// Small dense FP64 kernels for the truncated SVD of a parity block:
//   * reductions and scalings (Frobenius normalisation of C and T),
//   * a counter-based random start block for subspace iteration,
//   * Cholesky + triangular inverse of a small Gram matrix (CholeskyQR),
//   * one-sided (Hestenes) Jacobi SVD of a small square matrix,
//   * the merge of the two parity spectra and the truncation to chi.
// Each small problem is owned by one workgroup; several independent problems
// (the two parity sectors, the four corners) go in one launch.
#include <algorithm>
#include <cmath>

#include "hctm_internal.hpp"
#include "linalg.hpp"

namespace hctm {
namespace {

constexpr int NT = 1024;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

// ----------------------------------------------------------- reductions ----
__global__ void sumsq_partial_kernel(const double* __restrict__ p, long long n, double* __restrict__ part) {
  __shared__ double red[16];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = p[i];
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int n, double* __restrict__ out, int take_sqrt) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = take_sqrt ? sqrt(s) : s;
}

__global__ void scale_inv_kernel(double* __restrict__ p, long long n, const double* __restrict__ nrm) {
  const double f = 1.0 / *nrm;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] *= f;
}

__global__ void scale_block_kernel(double* p, int rows, int cols, long long ld, double alpha) {
  const long long n = (long long)rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    p[(e / cols) * ld + e % cols] *= alpha;
}

__global__ void fill_kernel(double* p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// splitmix64 (Steele, Lea, Flood 2014), mapped to a uniform double in [-1, 1)
__device__ __forceinline__ double rng_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void random_kernel(double* p, long long n, uint64_t seed) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = rng_uniform(seed, (uint64_t)i);
}

// ------------------------------------------------ Cholesky and inverse ----
// G (n x n, row-major, symmetric positive semidefinite) -> Rinv with
// G + shift*I = R^T R, R upper triangular; Rinv = R^-1 (upper, row-major).
// shift = rel * max_i G_ii.  The factorisation is the outer-product form
// a_ik -= a_ij a_kj / a_jj (one barrier per column), L = column / sqrt(pivot).
// Small problems keep both packed triangles (L and its inverse) in LDS.
constexpr int kLdsTri = 10153;  // doubles per packed triangle in LDS (n <= 142)

__device__ __forceinline__ int tri(int i, int k) { return i * (i + 1) / 2 + k; }

__device__ __forceinline__ void tri_decode(int e, int& i, int& k) {
  int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= e) ++r;
  while (r * (r + 1) / 2 > e) --r;
  i = r;
  k = e - r * (r + 1) / 2;
}

template <bool LDS>
__device__ void chol_inv_body(const SmallProb& P, double* Lp, double* Xp) {
  const int n = P.n, ld = P.lda, ldr = P.ldb;
  double* G = P.a;
  double* Ri = P.b;
  const int tid = threadIdx.x;
  __shared__ double red[16];
  __shared__ int bad_s;
  // packed-triangle accessors (LDS or global scratch in the lower part of G)
  auto Lr = [&](int i, int k) -> double& { return LDS ? Lp[tri(i, k)] : G[(long long)i * ld + k]; };
  auto Xr = [&](int i, int k) -> double& { return LDS ? Xp[tri(i, k)] : Ri[(long long)k * ldr + i]; };

  // optional symmetric diagonal scaling to a unit-diagonal Gram matrix
  const bool scale = (P.flags & 1) != 0;
  double* dsc = P.sv;
  if (scale) {
    for (int i = tid; i < n; i += NT) {
      const double g = G[(long long)i * ld + i];
      dsc[i] = g > 0.0 ? sqrt(g) : 1.0;
    }
    __syncthreads();
    if (!LDS) {
      for (long long e = tid; e < (long long)n * n; e += NT) {
        const int i = (int)(e / n), k = (int)(e % n);
        if (k <= i) G[(long long)i * ld + k] /= dsc[i] * dsc[k];
      }
      __syncthreads();
    }
  }
  double dmax = 0.0;
  for (int i = tid; i < n; i += NT) {
    const double g = G[(long long)i * ld + i];
    dmax = fmax(dmax, (scale && LDS) ? g / (dsc[i] * dsc[i]) : g);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  if (tid == 0) bad_s = 0;
  __syncthreads();
  dmax = 0.0;
  for (int i = 0; i < NT / 64; ++i) dmax = fmax(dmax, red[i]);
  const double shift = P.rel * dmax;
  // pivots at or below this are numerically dependent columns: they are
  // dropped (zero column of L, zero row and column of the inverse)
  const double thresh = 1e-27 * dmax;
  if (LDS) {
    for (int e = tid; e < n * (n + 1) / 2; e += NT) {
      int i, k;
      tri_decode(e, i, k);
      const double g = G[(long long)i * ld + k];
      Lp[e] = (scale ? g / (dsc[i] * dsc[k]) : g) + (i == k ? shift : 0.0);
    }
  } else {
    for (int i = tid; i < n; i += NT) G[(long long)i * ld + i] += shift;
  }
  __syncthreads();

  for (int j = 0; j < n; ++j) {
    const double djj = Lr(j, j);
    if (djj > thresh) {
      const int m = n - j - 1;
      const double inv = 1.0 / djj;
      for (int e = tid; e < m * (m + 1) / 2; e += NT) {
        int i, k;
        tri_decode(e, i, k);
        i += j + 1;
        k += j + 1;
        Lr(i, k) -= Lr(i, j) * Lr(k, j) * inv;
      }
    }
    __syncthreads();
  }
  // scale columns: L_ij = a_ij / sqrt(d_j), dropped columns set to zero
  for (int e = tid; e < n * (n + 1) / 2; e += NT) {
    int i, k;
    tri_decode(e, i, k);
    if (i == k) continue;
    const double dk = Lr(k, k);
    Lr(i, k) = dk > thresh ? Lr(i, k) / sqrt(dk) : 0.0;
  }
  __syncthreads();
  for (int j = tid; j < n; j += NT) {
    const double dj = Lr(j, j);
    if (!(dj > thresh)) atomicAdd(&bad_s, 1);
    Lr(j, j) = dj > thresh ? sqrt(dj) : 0.0;
  }
  __syncthreads();
  if (tid == 0 && P.info) *P.info = bad_s;

  // X = L^-1 (lower), from the last column to the first:
  // X[i][j] = -(sum_{k=j+1..i} X[i][k] L[k][j]) / L[j][j], i > j; X[j][j] = 1/L[j][j]
  const int lane = tid & 63, wave = tid >> 6;
  for (int j = n - 1; j >= 0; --j) {
    const double ljj = Lr(j, j);
    for (int i = j + 1 + wave; i < n; i += NT / 64) {
      double t = 0.0;
      for (int k = j + 1 + lane; k <= i; k += 64) t += Xr(i, k) * Lr(k, j);
      t = wave_sum(t);
      if (lane == 0) Xr(i, j) = ljj > 0.0 ? -t / ljj : 0.0;
    }
    if (tid == 0) Xr(j, j) = ljj > 0.0 ? 1.0 / ljj : 0.0;
    __syncthreads();
  }
  // Rinv = D^-1 X^T (upper)
  if (LDS) {
    for (int e = tid; e < n * n; e += NT) {
      const int c = e / n, i = e % n;  // Rinv[c][i] = X[i][c] / d[c]
      Ri[(long long)c * ldr + i] = (c <= i) ? Xp[tri(i, c)] / (scale ? dsc[c] : 1.0) : 0.0;
    }
  } else {
    for (int e = tid; e < n * n; e += NT) {
      const int c = e / n, i = e % n;
      if (c > i)
        Ri[(long long)c * ldr + i] = 0.0;
      else if (scale)
        Ri[(long long)c * ldr + i] /= dsc[c];
    }
  }
}

// Register-resident version for n <= 32 R: thread (ty, tx) of a 32 x 32 grid
// owns rows i = ty + 32 a and columns k = tx + 32 c (a, c < R) of the matrix.
// Factorisation: at step j the pivot column j is read from a double-buffered
// LDS vector written by its owners during step j-1 (one barrier per step).
// Inverse: right-looking forward substitution for all right-hand sides at
// once, X = L^-1, with row j of X broadcast the same way.
template <int R>
__device__ void chol_inv_regs(const SmallProb& P, double* Lpk, double* buf) {
  const int n = P.n, ld = P.lda, ldr = P.ldb;
  const double* G = P.a;
  double* Ri = P.b;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  __shared__ double red[16];
  __shared__ int bad_s;
  const bool scale = (P.flags & 1) != 0;
  double* dsc = P.sv;
  if (scale)
    for (int i = tid; i < n; i += NT) {
      const double g = G[(long long)i * ld + i];
      dsc[i] = g > 0.0 ? sqrt(g) : 1.0;
    }
  if (tid == 0) bad_s = 0;
  __syncthreads();
  double dmax = 0.0;
  for (int i = tid; i < n; i += NT) {
    const double g = G[(long long)i * ld + i];
    dmax = fmax(dmax, scale ? g / (dsc[i] * dsc[i]) : g);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  __syncthreads();
  dmax = 0.0;
  for (int i = 0; i < NT / 64; ++i) dmax = fmax(dmax, red[i]);
  const double shift = P.rel * dmax;
  const double thresh = 1e-27 * dmax;

  double a[R][R];
#pragma unroll
  for (int u = 0; u < R; ++u)
#pragma unroll
    for (int v = 0; v < R; ++v) {
      const int i = ty + 32 * u, k = tx + 32 * v;
      double x = 0.0;
      if (i < n && k <= i) {
        x = G[(long long)i * ld + k];
        if (scale) x /= dsc[i] * dsc[k];
        if (i == k) x += shift;
      }
      a[u][v] = x;
    }
  // column 0 to the buffer
  if (tx == 0)
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = ty + 32 * u;
      if (i < n) buf[i] = a[u][0];
    }
  __syncthreads();

  for (int j = 0; j < n; ++j) {
    const double* cur = buf + (j & 1) * 32 * R;
    double* nxt = buf + ((j + 1) & 1) * 32 * R;
    const double djj = cur[j];
    const double inv = djj > thresh ? 1.0 / djj : 0.0;
    double ci[R], ck[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = ty + 32 * u;
      ci[u] = (i > j && i < n) ? cur[i] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < R; ++v) {
      const int k = tx + 32 * v;
      ck[v] = (k > j && k < n && 32 * v + 31 > j) ? cur[k] * inv : 0.0;
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (32 * u + 31 <= j) continue;  // whole row block finished (uniform)
#pragma unroll
      for (int v = 0; v < R; ++v) {
        if (32 * v + 31 <= j || v > u) continue;  // finished or above the diagonal
        a[u][v] -= ci[u] * ck[v];                 // zero outside j < k <= i
      }
    }
    // owners of column j keep its final values (rows >= j) in the packed store
#pragma unroll
    for (int v = 0; v < R; ++v) {
      if (tx + 32 * v != j) continue;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int i = ty + 32 * u;
        if (i >= j && i < n) Lpk[i * (i + 1) / 2 + j] = (i == j) ? djj : cur[i];
      }
    }
    // owners of column j+1 publish it (final after this update)
#pragma unroll
    for (int v = 0; v < R; ++v) {
      if (tx + 32 * v != j + 1) continue;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int i = ty + 32 * u;
        if (i >= j + 1 && i < n) nxt[i] = a[u][v];
      }
    }
    __syncthreads();
  }
  // L = column / sqrt(pivot); dropped columns (pivot <= thresh) become zero
  for (int e = tid; e < n * (n + 1) / 2; e += NT) {
    int i, k;
    tri_decode(e, i, k);
    if (i == k) continue;
    const double dk = Lpk[k * (k + 1) / 2 + k];
    Lpk[e] = dk > thresh ? Lpk[e] / sqrt(dk) : 0.0;
  }
  __syncthreads();
  for (int j = tid; j < n; j += NT) {
    const double dj = Lpk[j * (j + 1) / 2 + j];
    if (!(dj > thresh)) atomicAdd(&bad_s, 1);
    Lpk[j * (j + 1) / 2 + j] = dj > thresh ? sqrt(dj) : 0.0;
  }
  __syncthreads();
  if (tid == 0 && P.info) *P.info = bad_s;

  // X = L^-1: b holds B (identity minus the applied updates) for (i, c), c <= i
  double (&b)[R][R] = a;
#pragma unroll
  for (int u = 0; u < R; ++u)
#pragma unroll
    for (int v = 0; v < R; ++v) b[u][v] = (ty + 32 * u == tx + 32 * v) ? 1.0 : 0.0;
  // row 0 of X
  if (ty == 0)
#pragma unroll
    for (int v = 0; v < R; ++v) {
      const int c = tx + 32 * v;
      const double l00 = Lpk[0];
      if (c == 0) {
        const double x = l00 > 0.0 ? b[0][v] / l00 : 0.0;
        b[0][v] = x;
        buf[0] = x;
      }
    }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double* xr = buf + (j & 1) * 32 * R;
    double* nxt = buf + ((j + 1) & 1) * 32 * R;
    double lij[R], xc[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = ty + 32 * u;
      lij[u] = (i > j && i < n) ? Lpk[i * (i + 1) / 2 + j] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < R; ++v) {
      const int c = tx + 32 * v;
      xc[v] = (c <= j) ? xr[c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (32 * u + 31 <= j) continue;  // rows <= j are final (uniform)
#pragma unroll
      for (int v = 0; v < R; ++v) {
        if (32 * v > j || v > u) continue;  // only columns c <= j change
        b[u][v] -= lij[u] * xc[v];
      }
    }
    // owners of row j+1 finalise it and publish
    if (j + 1 < n) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int i = ty + 32 * u;
        if (i != j + 1) continue;
        const double lii = Lpk[i * (i + 1) / 2 + i];
#pragma unroll
        for (int v = 0; v < R; ++v) {
          const int c = tx + 32 * v;
          if (c <= i) {
            const double x = lii > 0.0 ? b[u][v] / lii : 0.0;
            b[u][v] = x;
            nxt[c] = x;
          }
        }
      }
    }
    __syncthreads();
  }
  // Rinv[c][i] = X[i][c] / d[c] (upper), zero below the diagonal
#pragma unroll
  for (int u = 0; u < R; ++u)
#pragma unroll
    for (int v = 0; v < R; ++v) {
      const int i = ty + 32 * u, c = tx + 32 * v;
      if (i < n && c < n) {
        double x = c <= i ? b[u][v] : 0.0;
        if (scale && c <= i) x /= dsc[c];
        Ri[(long long)c * ldr + i] = x;
      }
    }
}

__global__ __launch_bounds__(NT) void chol_inv_regs_kernel(SmallBatch b) {
  __shared__ double Lpk[160 * 161 / 2];
  __shared__ double buf[2 * 32 * 5];
  const SmallProb& P = b.p[blockIdx.x];
  const int R = (P.n + 31) / 32;
  if (R <= 1)
    chol_inv_regs<1>(P, Lpk, buf);
  else if (R == 2)
    chol_inv_regs<2>(P, Lpk, buf);
  else if (R == 3)
    chol_inv_regs<3>(P, Lpk, buf);
  else if (R == 4)
    chol_inv_regs<4>(P, Lpk, buf);
  else
    chol_inv_regs<5>(P, Lpk, buf);
}

// ------------------------------------- Cholesky inverse, one elimination ----
// 1/x and 1/sqrt(x) from the hardware estimates and two Newton steps each
// (the estimates are good to far more than 2^-14, so two steps reach the
// rounding level).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double rsq_nr(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// R^-1 of G = R^T R for n <= 256, one workgroup per matrix: a GS x GS grid
// of threads (GS = 16 up to n = 64, else 32: more waves hide more latency), thread (ty, tx) holding the
// entries (ty + GS u, tx + GS v), u >= v, in registers.  The elimination of G
// (G = L_u D L_u^T, L_u unit lower) and the inverse X = L_u^-1 run in the same
// sweep over the columns and in the same registers.  With multipliers
// m_i = G_ij / d_j (i > j), step j updates
//   entries (i, k), k > j (still G):        G_ik -= m_i G_kj
//   entries (i, k), k < j (S, see below):   S_ik -= m_i S_jk
// and leaves column j alone.  S_ic = -d_c X_ic is X with column c scaled by
// -d_c: the update of X is linear in each column, and at step c the value
// held at (i, c), G_ic = m_i d_c, is exactly -d_c X_ic = -d_c (-m_i).  So the
// column-to-X transition costs nothing.  At the end X_ic = -S_ic / d_c and
// R^-1[c][i] = X_ic / sqrt(d_i).
//
// Two columns (J, J+1) per step.  Their owners publish V1[k] = G_kJ (k >= J),
// S_Jk (k < J) and V2[k] = G_k,J+1 (k >= J+1), S_J+1,k (k < J); an odd n is
// padded with a dead pivot.  Step J+1 sees column J+1 and row J+1 as updated
// by step J: d' = G_J+1,J+1 - m_J+1 G_J+1,J, multipliers
// m'_i = (G_i,J+1 - m_i G_J+1,J) / d' and vector w2_k = G_k,J+1 - m_k G_J+1,J
// (k > J+1), 0 (k = J+1), G_J+1,J (k = J: column J is S from step J+1 on),
// S_J+1,k - m_J+1 S_Jk (k < J); step J's vector w1 is V1 with 0 at J.  Phase
// A computes m, m', w1, w2 once per index into LDS; phase B applies both
// rank-one updates in one pass over the registers and publishes the next
// pair.  Two barriers per pair of columns.  Pivots d_j <= 1e-27 max(diag)
// drop their column: zero multipliers, and row and column of X zero (as in
// chol_inv_regs).
constexpr int kGjMaxN = 256;
#ifndef HCTM_GJ16_MAX
#define HCTM_GJ16_MAX 64
#endif
constexpr int kGj16Max = HCTM_GJ16_MAX;  // largest n on the 16 x 16 grid

template <int GS, int R>
__device__ void chol_gj(const SmallProb& P, double* buf, double* red, int* bad) {
  constexpr int NTC = GS * GS, NWV = NTC / 64, L = GS * R;
  const int n = P.n, ld = P.lda, ldr = P.ldb;
  const double* G = P.a;
  double* Ri = P.b;
  const int tid = threadIdx.x, tx = tid % GS, ty = tid / GS;
  const bool scale = (P.flags & 1) != 0;
  double* dsc = P.sv;
  // buf: V1, V2 (published columns), M1, M2 (multipliers), W1, W2 (vectors)
  double* V1 = buf;
  double* V2 = buf + L;
  double* M1 = buf + 2 * L;
  double* M2 = buf + 3 * L;
  double* W1 = buf + 4 * L;
  double* W2 = buf + 5 * L;
  if (scale)
    for (int i = tid; i < n; i += NTC) {
      const double g = G[(long long)i * ld + i];
      dsc[i] = g > 0.0 ? sqrt(g) : 1.0;
    }
  if (tid == 0) *bad = 0;
  for (int i = tid; i < 6 * L; i += NTC) buf[i] = 0.0;
  __syncthreads();
  double dmax = 0.0;
  for (int i = tid; i < n; i += NTC) {
    const double g = G[(long long)i * ld + i];
    dmax = fmax(dmax, scale ? g / (dsc[i] * dsc[i]) : g);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  __syncthreads();
  dmax = red[0];
#pragma unroll
  for (int w = 1; w < NWV; ++w) dmax = fmax(dmax, red[w]);
  const double shift = P.rel * dmax;
  const double thresh = 1e-27 * dmax;

  double a[R][R];  // a[u][v] used for u >= v only
#pragma unroll
  for (int u = 0; u < R; ++u)
#pragma unroll
    for (int v = 0; v <= u; ++v) {
      const int i = ty + GS * u, k = tx + GS * v;
      double x = 0.0;
      if (i < n && k <= i) {
        x = G[(long long)i * ld + k];
        if (scale) x /= dsc[i] * dsc[k];
        if (i == k) x += shift;
      }
      a[u][v] = x;
    }
  if (tx == 0)
#pragma unroll
    for (int u = 0; u < R; ++u) V1[ty + GS * u] = a[u][0];  // column 0
  if (tx == 1)
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = ty + GS * u;
      if (i >= 1) V2[i] = a[u][0];  // column 1
    }
  __syncthreads();

  for (int J = 0; J < n; J += 2) {
    // phase A: multipliers and update vectors, one index per thread
    {
      const double dJ = V1[J], g1 = V1[J + 1], e2 = V2[J + 1];
      const double inv = dJ > thresh ? rcp_nr(dJ) : 0.0;
      const double mJ1 = g1 * inv;
      const double d2 = e2 - mJ1 * g1;
      const double inv2 = d2 > thresh ? rcp_nr(d2) : 0.0;
      for (int t = tid; t < L; t += NTC) {
        const double v1 = V1[t], v2 = V2[t];
        const double x1 = v1 * inv;
        const double y2 = fma(-x1, g1, v2);  // G_t,J+1 - m_t G_J+1,J
        M1[t] = t > J ? x1 : 0.0;
        M2[t] = t > J + 1 ? y2 * inv2 : 0.0;
        W1[t] = t == J ? 0.0 : v1;
        W2[t] = t > J + 1 ? y2 : (t == J + 1 ? 0.0 : (t == J ? g1 : fma(-mJ1, v1, v2)));
      }
    }
    __syncthreads();
    // phase B: both rank-one updates; rows <= J are final
    const int jb = J / GS;
    double m1[R], m2[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      m1[u] = M1[ty + GS * u];
      m2[u] = M2[ty + GS * u];
    }
#pragma unroll
    for (int v = 0; v < R; ++v) {
      const double w1 = W1[tx + GS * v], w2 = W2[tx + GS * v];
#pragma unroll
      for (int u = v; u < R; ++u) {
        if (u < jb) continue;  // uniform
        a[u][v] = fma(-m2[u], w2, fma(-m1[u], w1, a[u][v]));
      }
    }
    // publish the next pair of columns (their entries are final now)
    const int J2 = J + 2;
    if (J2 < n) {
      const int b2 = J2 / GS, l2 = J2 % GS;  // J2 + 1 is in the same block
#pragma unroll
      for (int v = 0; v < R; ++v) {
        if (v != b2) continue;  // uniform
        if (tx == l2)
#pragma unroll
          for (int u = v; u < R; ++u) {
            const int i = ty + GS * u;
            if (i >= J2) V1[i] = a[u][v];
          }
        if (tx == l2 + 1)
#pragma unroll
          for (int u = v; u < R; ++u) {
            const int i = ty + GS * u;
            if (i >= J2 + 1) V2[i] = a[u][v];
          }
        if (ty == l2)
#pragma unroll
          for (int c = 0; c <= v; ++c) {
            const int k = tx + GS * c;
            if (k < J2) V1[k] = a[v][c];
          }
        if (ty == l2 + 1)
#pragma unroll
          for (int c = 0; c <= v; ++c) {
            const int k = tx + GS * c;
            if (k < J2) V2[k] = a[v][c];
          }
      }
    }
    __syncthreads();
  }
  // the pivots d_i sit on the diagonal: gather them through LDS
  double* dg = M1;
  if (tx == ty)
#pragma unroll
    for (int u = 0; u < R; ++u) dg[ty + GS * u] = a[u][u];
  __syncthreads();
  int nbad = 0;
  double rs[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = ty + GS * u;
    const double d = i < n ? dg[i] : 1.0;
    rs[u] = d > thresh ? 1.0 / sqrt(d) : 0.0;
    if (i < n && !(d > thresh) && tx == 0) ++nbad;
  }
  if (nbad) atomicAdd(bad, nbad);
  // R^-1[c][i] = X_ic / sqrt(d_i) (/ scale of c), X_ic = -S_ic / d_c, X_ii = 1
#pragma unroll
  for (int u = 0; u < R; ++u)
#pragma unroll
    for (int v = 0; v < R; ++v) {
      const int i = ty + GS * u, c = tx + GS * v;
      if (i < n && c < n) {
        double x = 0.0;
        if (v <= u && c <= i) {
          const double dc = dg[c];
          if (c == i)
            x = rs[u];
          else
            x = dc > thresh ? -a[u][v] / dc * rs[u] : 0.0;
          if (scale) x /= dsc[c];
        }
        Ri[(long long)c * ldr + i] = x;
      }
    }
  __syncthreads();
  if (tid == 0 && P.info) *P.info = *bad;
}

// R = ceil(max n / GS) of the batch; smaller problems carry zero blocks
template <int GS, int R>
__global__ __launch_bounds__(GS * GS) void chol_gj_kernel(SmallBatch b) {
  __shared__ double buf[6 * GS * R];
  __shared__ double red[GS * GS / 64];
  __shared__ int bad;
  chol_gj<GS, R>(b.p[blockIdx.x], buf, red, &bad);
}

__global__ __launch_bounds__(NT) void chol_inv_kernel(SmallBatch b) {
  __shared__ double Lp[kLdsTri];
  __shared__ double Xp[kLdsTri];
  const SmallProb& P = b.p[blockIdx.x];
  if (P.n * (P.n + 1) / 2 <= kLdsTri)
    chol_inv_body<true>(P, Lp, Xp);
  else
    chol_inv_body<false>(P, nullptr, nullptr);
}

// ------------------------------------------------- one-sided Jacobi SVD ----
// Orthogonalises the columns of X (m x n, row-major, leading dim ld) by plane
// rotations in round-robin order, one pair per wave at a time.  On exit:
// sv[j] = j-th largest column norm, perm[j] = its column.
__global__ __launch_bounds__(NT) void jacobi_kernel(SmallBatch b) {
  const SmallProb& P = b.p[blockIdx.x];
  const int m = P.m, n = P.n, ld = P.lda;
  double* X = P.a;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = NT / 64;
  __shared__ int any_rot;
  __shared__ double nrm[1024];

  // optional accumulation of the right vectors: V (n x n, row-major, ld n)
  double* Vm = P.b;
  if (Vm)
    for (long long e = threadIdx.x; e < (long long)n * n; e += NT) Vm[e] = (e / n == e % n) ? 1.0 : 0.0;
  const int n2 = n + (n & 1);
  const int mr = n2 - 1;  // rotating players; player n2-1 fixed
  const double tol = P.rel;
  const int pairabs = P.flags & kJacPairAbs;
  // columns below m*eps*||X||_F are rounding noise: pairs involving them are
  // not rotated (their norms are kept as the singular values)
  __shared__ double red[16];
  double f2 = 0.0;
  for (long long e = threadIdx.x; e < (long long)m * n; e += NT) {
    const double x = X[(e / n) * ld + (e % n)];
    f2 += x * x;
  }
  f2 = block_sum(f2, red);
  const double small2 = f2 * (2.3e-16 * m) * (2.3e-16 * m);
  int sweep = 0;
  for (sweep = 0; sweep < P.max_sweeps; ++sweep) {
    if (threadIdx.x == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < mr; ++r) {
      for (int pp = wave; pp < n2 / 2; pp += nw) {
        int i, j;
        if (pp == 0) {
          i = r;
          j = n2 - 1;
        } else {
          i = (r + pp) % mr;
          j = (r - pp + mr) % mr;
        }
        if (i >= n || j >= n) continue;
        if (i > j) {
          const int t = i;
          i = j;
          j = t;
        }
        double a = 0.0, bb = 0.0, g = 0.0;
        for (int k = lane; k < m; k += 64) {
          const double xi = X[(long long)k * ld + i], xj = X[(long long)k * ld + j];
          a += xi * xi;
          bb += xj * xj;
          g += xi * xj;
        }
        a = wave_sum(a);
        bb = wave_sum(bb);
        g = wave_sum(g);
        if (fmin(a, bb) <= small2 || fabs(g) <= (pairabs ? tol * fmax(a, bb) : tol * sqrt(a) * sqrt(bb))) continue;
        const double zeta = (bb - a) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
        for (int k = lane; k < m; k += 64) {
          const double xi = X[(long long)k * ld + i], xj = X[(long long)k * ld + j];
          X[(long long)k * ld + i] = c * xi - s * xj;
          X[(long long)k * ld + j] = s * xi + c * xj;
        }
        if (Vm)
          for (int k = lane; k < n; k += 64) {
            const double vi = Vm[(long long)k * n + i], vj = Vm[(long long)k * n + j];
            Vm[(long long)k * n + i] = c * vi - s * vj;
            Vm[(long long)k * n + j] = s * vi + c * vj;
          }
        if (lane == 0) any_rot = 1;
      }
      __syncthreads();
    }
    const int rot = any_rot;
    __syncthreads();
    if (!rot) break;
  }
  if (threadIdx.x == 0 && P.info) *P.info = sweep < P.max_sweeps ? sweep : -sweep;

  // column norms and descending order (ties: lower index first)
  for (int j = threadIdx.x; j < n; j += NT) {
    double s = 0.0;
    for (int k = 0; k < m; ++k) {
      const double x = X[(long long)k * ld + j];
      s += x * x;
    }
    nrm[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += NT) {
    const double v = nrm[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double w = nrm[i];
      rank += (w > v) || (w == v && i < j);
    }
    P.sv[rank] = v;
    P.perm[rank] = j;
  }
}

// LDS-resident one-sided Jacobi for m * n <= kJacLds: X is held column-major
// in LDS; 16 lanes work on one column pair (a wave on four pairs at a time).
// The plane rotations of every round are logged (cos, sin per pair) so that
// the right vectors can be rebuilt in parallel afterwards (jacobi_v_kernel).
constexpr int kJacLds = 19968;  // doubles of LDS for X (n = m <= 141)

// Sum over the 16 lanes of a DPP row, result in every lane: swap neighbours,
// swap pairs (quad permutations), then the mirrored half row and row.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 8 lanes of a half DPP row (swap neighbours, swap pairs, then
// the mirrored half row), result in all 8 lanes.
__device__ __forceinline__ double sum8(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  return v;
}

// Sum over the LANES (8 or 16) lanes of a group inside a DPP row; the 16-lane
// sum adds the mirrored row to the half-row sums.
template <int LANES>
__device__ __forceinline__ double sum_lanes(double v) {
  static_assert(LANES == 8 || LANES == 16, "a column pair takes 8 or 16 lanes");
  v = sum8(v);
  if constexpr (LANES == 16) v += dpp_move<0x140>(v);  // row_mirror
  return v;
}

// Round-robin pairing of n2 (even) columns: round r pairs column n2-1 with r
// and (r + p) with (r - p) modulo n2 - 1 for p = 1 .. n2/2 - 1.
__device__ __forceinline__ void rr_pair(int r, int pp, int n2, int& i, int& j) {
  const int mr = n2 - 1;
  if (pp == 0) {
    i = r;
    j = n2 - 1;
  } else {
    i = r + pp;
    if (i >= mr) i -= mr;
    j = r - pp;
    if (j < 0) j += mr;
  }
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
}

// One group of kJacLanes lanes per column pair; each lane keeps its rows of the two
// columns in registers between the dot product and the rotation.  Squared
// column norms are kept in LDS and recomputed only for the columns a
// rotation changed, so a round needs one dot product per pair.
// Workgroup of the LDS kernel: 1024 threads, 16 lanes per column pair, so
// that every pair of a round (up to 128 columns) is rotated at once (measured
// 27-31 % faster than 256 threads with 8 lanes per pair on 76-141 columns)
constexpr int kJacNT = 1024;
constexpr int kJacLanes = 16;
constexpr int kJacMaxRows = 160;                 // rows of a matrix the LDS kernel takes
constexpr int kJacRowsMax = kJacMaxRows / kJacLanes;  // rows per lane at that size
// Rows per lane of the kernel instance for m rows (the row loops are unrolled
// to this length, so small matrices take a short instance).
inline int jacobi_rows_per_lane(int m) { return m <= 64 ? 4 : (m <= 128 ? 8 : kJacRowsMax); }

typedef double v4d __attribute__((ext_vector_type(4)));

// Every pair of the columns c0 .. c0 + nn - 1 of Xs at once: the Gram matrix
// X^T X on the matrix cores (v_mfma_f64_16x16x4f64; lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[l / 16 + 4 v][l % 16]),
// each off-diagonal entry against the pair test of the sweeps (with the cached
// squared norms).  True if no pair would rotate, i.e. the next sweep would
// rotate nothing.  Called by all threads of the workgroup.
__device__ bool gram_orthogonal(const double* Xs, const double* nrm, int* fail, int m, int c0, int nn, double tol,
                                double small2, int pairabs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  if (threadIdx.x == 0) *fail = 0;
  __syncthreads();
  const int nt = (nn + 15) / 16, ntiles = nt * (nt + 1) / 2;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < ntiles; t += nwave) {  // wave-uniform
    int ti = 0, rem = t;
    while (rem >= nt - ti) {
      rem -= nt - ti;
      ++ti;
    }
    const int tj = ti + rem;
    const int ci = 16 * ti + li, cj = 16 * tj + li;
    const bool oki = ci < nn, okj = cj < nn;
    const double* xi = Xs + (long long)(c0 + (oki ? ci : 0)) * m;
    const double* xj = Xs + (long long)(c0 + (okj ? cj : 0)) * m;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int r0 = 0; r0 < m; r0 += 4) {
      const int r = r0 + lk;
      const double a = (oki && r < m) ? xi[r] : 0.0;
      const double b = (okj && r < m) ? xj[r] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    bool bad = false;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * ti + lk + 4 * v, j = 16 * tj + li;
      if (i < j && j < nn) {
        const double g = acc[v];
        const double a2 = nrm[c0 + i], b2 = nrm[c0 + j];
        if (fmin(a2, b2) > small2 && fabs(g) > (pairabs ? tol * fmax(a2, b2) : tol * sqrt(a2) * sqrt(b2))) bad = true;
      }
    }
    if (bad) *fail = 1;
  }
  __syncthreads();
  const bool ok = *fail == 0;
  __syncthreads();
  return ok;
}

// Sweeps of round-robin rotations over the columns c0 .. c0 + nn - 1 of Xs
// (column-major, m rows) until no pair would rotate; rotations logged as
// (sweep, round, pair) from lg.  After a sweep that rotated, the pair test
// is run on all pairs at once on the Gram matrix (gram_orthogonal), so that
// the sweep that would only confirm convergence is not run.  Returns the
// sweeps done (logged), negated when max_sweeps ran out first.
template <int ROWS>
__device__ int jacobi_sweeps(double* Xs, double* nrm, int* any_rot, int m, int c0, int nn, double tol,
                             double small2, int pairabs, int max_sweeps, double2* lg) {
  const int tid = threadIdx.x;
  const int n2 = nn + (nn & 1), npairs = n2 / 2, rounds = n2 - 1;
  const int sub = tid & (kJacLanes - 1), grp = tid / kJacLanes, ngrp = kJacNT / kJacLanes;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) *any_rot = 0;
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
      double2* lr = lg ? lg + ((long long)sweep * rounds + r) * npairs : nullptr;
      for (int pp = grp; pp < npairs; pp += ngrp) {
        int i, j;
        rr_pair(r, pp, n2, i, j);
        double c = 1.0, sn = 0.0;
        if (j < nn) {
          i += c0;
          j += c0;
          double* xi = Xs + i * m;
          double* xj = Xs + j * m;
          double u[ROWS], v[ROWS];
          double g = 0.0;
#pragma unroll
          for (int q = 0; q < ROWS; ++q) {
            const int k = sub + kJacLanes * q;
            u[q] = k < m ? xi[k] : 0.0;
            v[q] = k < m ? xj[k] : 0.0;
            g = fma(u[q], v[q], g);
          }
          g = sum_lanes<kJacLanes>(g);
          const double a = nrm[i], bb = nrm[j];
          // sqrt(a) sqrt(b), not sqrt(a b): near-zero blocks (a sector that
          // the state leaves empty up to rounding) would underflow the product
          if (fmin(a, bb) > small2 && fabs(g) > (pairabs ? tol * fmax(a, bb) : tol * sqrt(a) * sqrt(bb))) {
            const double zeta = (bb - a) * rcp_nr(2.0 * g);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
            c = rsq_nr(fma(t, t, 1.0));
            sn = c * t;
            double a2 = 0.0, b2 = 0.0;
#pragma unroll
            for (int q = 0; q < ROWS; ++q) {
              const int k = sub + kJacLanes * q;
              const double x = c * u[q] - sn * v[q], y = sn * u[q] + c * v[q];
              if (k < m) {
                xi[k] = x;
                xj[k] = y;
              }
              a2 = fma(x, x, a2);
              b2 = fma(y, y, b2);
            }
            // exact norms of the rotated columns (the update a - t g loses
            // relative accuracy when a column is nearly emptied)
            a2 = sum_lanes<kJacLanes>(a2);
            b2 = sum_lanes<kJacLanes>(b2);
            if (sub == 0) {
              nrm[i] = a2;
              nrm[j] = b2;
              *any_rot = 1;
            }
          }
        }
        if (sub == 0 && lr) lr[pp] = make_double2(c, sn);
      }
      __syncthreads();
    }
    const int rot = *any_rot;
    __syncthreads();
    if (!rot) return sweep + 1;  // the converged sweep is logged too (identity rotations)
    if (gram_orthogonal(Xs, nrm, any_rot, m, c0, nn, tol, small2, pairabs)) return sweep + 1;
  }
  return -max_sweeps;
}

// Offset (in (c, s) pairs) of the log of the leading phase over the trailing
// columns: after the room for max_sweeps sweeps over all n columns.
__host__ __device__ inline long long jacobi_pre_log_offset(int n, int max_sweeps) {
  const long long n2 = n + (n & 1);
  return (long long)max_sweeps * (n2 - 1) * (n2 / 2);
}

// A subspace-iteration Ritz block is close to diagonal except among its
// trailing (oversampled, least converged) columns; with P.pre set, those are
// orthogonalised among themselves first (short sweeps), so that the sweeps
// over all columns start from nearly orthogonal columns and converge in few
// sweeps.  The result is the same one-sided Jacobi SVD (the full sweeps run
// until a sweep rotates nothing).
template <int ROWS>
__global__ __launch_bounds__(kJacNT) void jacobi_lds_kernel(SmallBatch b) {
  __shared__ double Xs[kJacLds];
  __shared__ int any_rot;
  __shared__ double red[16];
  __shared__ double nrm[160];
  const SmallProb& P = b.p[blockIdx.x];
  const int m = P.m, n = P.n, ld = P.lda;
  double* X = P.a;
  double2* rlog = reinterpret_cast<double2*>(P.b);  // rotation log or null
  const int tid = threadIdx.x;
  for (int e = tid; e < m * n; e += kJacNT) {
    const int r = e / n, c = e % n;
    Xs[c * m + r] = X[(long long)r * ld + c];
  }
  double f2 = 0.0;
  for (int e = tid; e < m * n; e += kJacNT) {
    const double x = X[(long long)(e / n) * ld + (e % n)];
    f2 += x * x;
  }
  f2 = block_sum(f2, red);  // includes barriers
  const double small2 = f2 * (2.3e-16 * m) * (2.3e-16 * m);
  const double tol = P.rel;
  for (int j = tid; j < n; j += kJacNT) {
    double s2 = 0.0;
    for (int k = 0; k < m; ++k) s2 += Xs[j * m + k] * Xs[j * m + k];
    nrm[j] = s2;
  }
  __syncthreads();
  // phase 0 over the trailing pre columns (if any), phase 1 over all; one
  // call site, so that the sweep loop is inlined once
  const int pre = (P.pre >= 2 && P.pre < n) ? P.pre : 0;
  for (int ph = pre ? 0 : 1; ph < 2; ++ph) {
    const int c0 = ph == 0 ? n - pre : 0, nn = ph == 0 ? pre : n;
    double2* lg = (rlog && ph == 0) ? rlog + jacobi_pre_log_offset(n, P.max_sweeps) : rlog;
    const int sw =
        jacobi_sweeps<ROWS>(Xs, nrm, &any_rot, m, c0, nn, tol, small2, P.flags & kJacPairAbs, P.max_sweeps, lg);
    if (tid == 0 && P.info) {
      if (ph == 0)
        P.info[1] = sw < 0 ? -sw : sw;
      else
        P.info[0] = sw;
    }
  }
  for (int j = tid; j < n; j += kJacNT) {
    double s2 = 0.0;
    for (int k = 0; k < m; ++k) s2 += Xs[j * m + k] * Xs[j * m + k];
    nrm[j] = sqrt(s2);
  }
  for (int e = tid; e < m * n; e += kJacNT) {
    const int r = e / n, c = e % n;
    X[(long long)r * ld + c] = Xs[c * m + r];
  }
  __syncthreads();
  for (int j = tid; j < n; j += kJacNT) {
    const double v = nrm[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double w = nrm[i];
      rank += (w > v) || (w == v && i < j);
    }
    P.sv[rank] = v;
    P.perm[rank] = j;
  }
}

// Jacobi for blocks too large for LDS (n, m <= 256): X is copied column-major
// into P.work (global memory; at most 512 KB, so it stays in L2), one wave
// works on one column pair with four rows per lane, the pairs a wave owns in
// a round are loaded together; column norms cached in LDS; same rotation
// order, tests, log layout, phases and Gram-matrix convergence check as the
// LDS kernel.
constexpr int kJacL2Max = 256;
constexpr int kJacL2Threads = 1024;
constexpr int kJacL2Rows = kJacL2Max / 64;  // rows per lane
constexpr int kJacL2Batch = 4;              // pairs loaded together by a wave

__device__ int jacobi_l2_sweeps(double* Xc, double* nrm, int* any_rot, int m, int c0, int nn, double tol,
                                double small2, int pairabs, int max_sweeps, double2* lg) {
  constexpr int NW = kJacL2Threads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n2 = nn + (nn & 1), npairs = n2 / 2, rounds = n2 - 1;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) *any_rot = 0;
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
      double2* lr = lg ? lg + ((long long)sweep * rounds + r) * npairs : nullptr;
      for (int p0 = wave; p0 < npairs; p0 += NW * kJacL2Batch) {
        double u[kJacL2Batch][kJacL2Rows], v[kJacL2Batch][kJacL2Rows];
        int pi[kJacL2Batch], pj[kJacL2Batch];
#pragma unroll
        for (int bq = 0; bq < kJacL2Batch; ++bq) {
          const int pp = p0 + bq * NW;
          int i = 0, j = nn;  // j >= nn: no pair
          if (pp < npairs) rr_pair(r, pp, n2, i, j);
          pi[bq] = i;
          pj[bq] = j;
          const bool live = pp < npairs && j < nn;
          const double* xi = Xc + (long long)(c0 + i) * m;
          const double* xj = Xc + (long long)(c0 + (live ? j : i)) * m;
#pragma unroll
          for (int q = 0; q < kJacL2Rows; ++q) {
            const int k = lane + 64 * q;
            u[bq][q] = (live && k < m) ? xi[k] : 0.0;
            v[bq][q] = (live && k < m) ? xj[k] : 0.0;
          }
        }
#pragma unroll
        for (int bq = 0; bq < kJacL2Batch; ++bq) {
          const int pp = p0 + bq * NW;
          if (pp >= npairs) break;  // uniform in the wave
          double c = 1.0, sn = 0.0;
          if (pj[bq] < nn) {
            const int i = c0 + pi[bq], j = c0 + pj[bq];
            double g = 0.0;
#pragma unroll
            for (int q = 0; q < kJacL2Rows; ++q) g = fma(u[bq][q], v[bq][q], g);
            g = wave_sum(g);
            const double a = nrm[i], bb = nrm[j];
            if (fmin(a, bb) > small2 && fabs(g) > (pairabs ? tol * fmax(a, bb) : tol * sqrt(a) * sqrt(bb))) {
              const double zeta = (bb - a) * rcp_nr(2.0 * g);
              const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
              c = rsq_nr(fma(t, t, 1.0));
              sn = c * t;
              double a2 = 0.0, b2 = 0.0;
              double* xi = Xc + (long long)i * m;
              double* xj = Xc + (long long)j * m;
#pragma unroll
              for (int q = 0; q < kJacL2Rows; ++q) {
                const int k = lane + 64 * q;
                const double x = c * u[bq][q] - sn * v[bq][q], y = sn * u[bq][q] + c * v[bq][q];
                if (k < m) {
                  xi[k] = x;
                  xj[k] = y;
                }
                a2 = fma(x, x, a2);
                b2 = fma(y, y, b2);
              }
              a2 = wave_sum(a2);
              b2 = wave_sum(b2);
              if (lane == 0) {
                nrm[i] = a2;
                nrm[j] = b2;
                *any_rot = 1;
              }
            }
          }
          if (lane == 0 && lr) lr[pp] = make_double2(c, sn);
        }
      }
      __syncthreads();
    }
    const int rot = *any_rot;
    __syncthreads();
    if (!rot) return sweep + 1;
    if (gram_orthogonal(Xc, nrm, any_rot, m, c0, nn, tol, small2, pairabs)) return sweep + 1;
  }
  return -max_sweeps;
}

__global__ __launch_bounds__(kJacL2Threads) void jacobi_l2_kernel(SmallBatch b) {
  __shared__ int any_rot;
  __shared__ double red[16];
  __shared__ double nrm[kJacL2Max];
  const SmallProb& P = b.p[blockIdx.x];
  const int m = P.m, n = P.n, ld = P.lda;
  double* X = P.a;
  double* Xc = P.work;
  double2* rlog = reinterpret_cast<double2*>(P.b);
  const int tid = threadIdx.x;
  double f2 = 0.0;
  for (int e = tid; e < m * n; e += kJacL2Threads) {
    const int r = e / n, c = e % n;
    const double x = X[(long long)r * ld + c];
    Xc[(long long)c * m + r] = x;
    f2 += x * x;
  }
  f2 = block_sum(f2, red);  // includes barriers (and makes Xc visible to the workgroup)
  const double small2 = f2 * (2.3e-16 * m) * (2.3e-16 * m);
  const double tol = P.rel;
  for (int j = tid; j < n; j += kJacL2Threads) {
    double s2 = 0.0;
    for (int k = 0; k < m; ++k) s2 += Xc[(long long)j * m + k] * Xc[(long long)j * m + k];
    nrm[j] = s2;
  }
  __syncthreads();
  const int pre = (P.pre >= 2 && P.pre < n) ? P.pre : 0;
  for (int ph = pre ? 0 : 1; ph < 2; ++ph) {
    const int c0 = ph == 0 ? n - pre : 0, nn = ph == 0 ? pre : n;
    double2* lg = (rlog && ph == 0) ? rlog + jacobi_pre_log_offset(n, P.max_sweeps) : rlog;
    const int sw = jacobi_l2_sweeps(Xc, nrm, &any_rot, m, c0, nn, tol, small2, P.flags & kJacPairAbs, P.max_sweeps,
                                    lg);
    if (tid == 0 && P.info) {
      if (ph == 0)
        P.info[1] = sw < 0 ? -sw : sw;
      else
        P.info[0] = sw;
    }
  }
  for (int j = tid; j < n; j += kJacL2Threads) {
    double s2 = 0.0;
    for (int k = 0; k < m; ++k) s2 += Xc[(long long)j * m + k] * Xc[(long long)j * m + k];
    nrm[j] = sqrt(s2);
  }
  for (int e = tid; e < m * n; e += kJacL2Threads) {
    const int r = e / n, c = e % n;
    X[(long long)r * ld + c] = Xc[(long long)c * m + r];
  }
  __syncthreads();
  for (int j = tid; j < n; j += kJacL2Threads) {
    const double v = nrm[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double w = nrm[i];
      rank += (w > v) || (w == v && i < j);
    }
    P.sv[rank] = v;
    P.perm[rank] = j;
  }
}

// Rebuild V (n x n, row-major, written to P.a) from the rotation log in
// P.b: rows are independent, kVRows rows per workgroup held column-major in
// LDS; the log is staged kVChunk rounds at a time so that each round reads
// LDS only.  The rotations of the leading phase over the trailing columns
// (P.pre) come first.
constexpr int kVChunk = 16;
constexpr int kVRows = 8;

// Apply the logged rotations of `sweeps` sweeps over the columns
// c0 .. c0 + nn - 1 to the rows held in Vs.
__device__ void replay_rotations(double* Vs, double2* Ls, const double2* lg, int c0, int nn, int sweeps,
                                 int rows) {
  const int n2 = nn + (nn & 1), npairs = n2 / 2, rounds = n2 - 1;
  const long long total = (long long)sweeps * rounds;
  int r = 0;
  for (long long t0 = 0; t0 < total; t0 += kVChunk) {
    const int nr = (int)min<long long>(kVChunk, total - t0);
    __syncthreads();
    for (int e = threadIdx.x; e < nr * npairs; e += 256) Ls[e] = lg[t0 * npairs + e];
    __syncthreads();
    for (int q = 0; q < nr; ++q) {
      for (int e = threadIdx.x; e < npairs * kVRows; e += 256) {
        const int pp = e / kVRows, rr = e % kVRows;
        const double2 cs = Ls[q * npairs + pp];
        if (cs.y == 0.0 || rr >= rows) continue;
        int i, j;
        rr_pair(r, pp, n2, i, j);
        if (j >= nn) continue;
        i += c0;
        j += c0;
        const double u = Vs[i * kVRows + rr], v = Vs[j * kVRows + rr];
        Vs[i * kVRows + rr] = cs.x * u - cs.y * v;
        Vs[j * kVRows + rr] = cs.y * u + cs.x * v;
      }
      if (++r == rounds) r = 0;
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void jacobi_v_kernel(SmallBatch b) {
  __shared__ double Vs[kJacL2Max * kVRows];
  __shared__ double2 Ls[kVChunk * (kJacL2Max / 2)];
  const SmallProb& P = b.p[blockIdx.y];
  const int n = P.n;
  const int sweeps = P.info ? abs(P.info[0]) : 0;
  const int pre = (P.info && P.pre >= 2 && P.pre < n) ? P.pre : 0;
  const double2* lg = reinterpret_cast<const double2*>(P.b);
  double* V = P.a;
  const int r0 = blockIdx.x * kVRows;
  if (r0 >= n) return;
  const int rows = min(kVRows, n - r0);
  for (int e = threadIdx.x; e < kVRows * n; e += 256) {
    const int c = e / kVRows, rr = e % kVRows;
    Vs[c * kVRows + rr] = (r0 + rr == c) ? 1.0 : 0.0;
  }
  if (pre)
    replay_rotations(Vs, Ls, lg + jacobi_pre_log_offset(n, P.max_sweeps), n - pre, pre, P.info[1], rows);
  replay_rotations(Vs, Ls, lg, 0, n, sweeps, rows);
  __syncthreads();
  for (int e = threadIdx.x; e < rows * n; e += 256) {
    const int rr = e / n, c = e % n;
    V[(long long)(r0 + rr) * n + c] = Vs[c * kVRows + rr];
  }
}

// U (m x k, row-major) = X[:, perm[j]] / sv[j]  (columns normalised);
// zero columns where sv == 0; plain gather if sv is null.
__global__ void gather_cols_kernel(const double* __restrict__ X, int ldx, const int* __restrict__ perm,
                                   const double* __restrict__ sv, int m, int k, double* __restrict__ U, int ldu) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)m * k) return;
  const int r = (int)(e / k), c = (int)(e % k);
  if (!sv) {
    U[(long long)r * ldu + c] = X[(long long)r * ldx + perm[c]];
    return;
  }
  const double s = sv[c];
  U[(long long)r * ldu + c] = s > 0.0 ? X[(long long)r * ldx + perm[c]] / s : 0.0;
}

// ------------------------------------------------- subspace convergence ----
// Column residuals of a subspace-iteration step: for the leading k columns,
// out[0] = max_i |A_i - B_i| and out[1] = max_i |A_i| (A = M Q_r, B its
// projection on the current left basis).  Both are written as the bit
// patterns of non-negative doubles with atomic max (the order of the bits is
// the order of the values); out must be cleared first.
__global__ __launch_bounds__(256) void col_resid_kernel(const double* __restrict__ A, int lda,
                                                        const double* __restrict__ B, int ldb, int n,
                                                        unsigned long long* out) {
  const int c = blockIdx.x;
  __shared__ double red[2][4];
  double d2 = 0.0, a2 = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const double a = A[(long long)r * lda + c], b = B[(long long)r * ldb + c];
    d2 += (a - b) * (a - b);
    a2 += a * a;
  }
  d2 = wave_sum(d2);
  a2 = wave_sum(a2);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = d2;
    red[1][w] = a2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d2 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    a2 = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    atomicMax(out, (unsigned long long)__double_as_longlong(sqrt(d2)));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(sqrt(a2)));
  }
}

// Ritz residuals: out[c] = || GU[:, c] - lam[c] U[:, c] ||_2 for c < k (n rows,
// row-major, leading dim ld); one block per column, no atomics.
__global__ __launch_bounds__(256) void ritz_resid_kernel(const double* __restrict__ GU, const double* __restrict__ U,
                                                         const double* __restrict__ lam, int n, int ld,
                                                         double* __restrict__ out) {
  const int c = blockIdx.x;
  __shared__ double red[4];
  const double l = lam[c];
  double d2 = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const double x = GU[(long long)r * ld + c] - l * U[(long long)r * ld + c];
    d2 += x * x;
  }
  d2 = wave_sum(d2);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = d2;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// --------------------------------------------------------- truncation ----
// Merge the two descending spectra (even sector first on ties) and keep
// k = min(chi, #{s > tau * s_max}) (at least one).  Writes k_even, k_odd,
// s_max, the first discarded and the last kept value, and the inverse square
// roots and inverses of the kept values per sector.  The leading chi + 1
// values of each sector are staged in LDS by all threads, one thread merges,
// all threads write the inverses.
__global__ __launch_bounds__(256) void select_kernel(SelectArgs a, int staged) {
  extern __shared__ double sh[];
  __shared__ int kk[2];
  const int c0 = min(a.n0, a.chi + 1), c1 = min(a.n1, a.chi + 1);
  const double* s0 = a.sv0;
  const double* s1 = a.sv1;
  if (staged) {  // (else the values are read where they are)
    for (int i = threadIdx.x; i < c0; i += blockDim.x) sh[i] = a.sv0[i];
    for (int i = threadIdx.x; i < c1; i += blockDim.x) sh[c0 + i] = a.sv1[i];
    s0 = sh;
    s1 = sh + c0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double v00 = c0 > 0 ? s0[0] : -1.0;
    const double v10 = c1 > 0 ? s1[0] : -1.0;
    const double smax = fmax(v00, v10);
    int i0 = 0, i1 = 0, k = 0;
    while (k < a.chi) {
      const double v0 = i0 < c0 ? s0[i0] : -1.0;
      const double v1 = i1 < c1 ? s1[i1] : -1.0;
      const bool take0 = v0 >= v1;
      const double v = take0 ? v0 : v1;
      if (v < 0.0) break;
      if (!(v > a.tau * smax) && k > 0) break;
      if (take0)
        ++i0;
      else
        ++i1;
      ++k;
    }
    a.out_k[0] = i0;
    a.out_k[1] = i1;
    a.out_s[0] = smax;
    // the first discarded and the last kept value (-1: none), for the
    // multiplet-split test at the chi cut
    const double v0 = i0 < c0 ? s0[i0] : -1.0;
    const double v1 = i1 < c1 ? s1[i1] : -1.0;
    a.out_s[1] = fmax(v0, v1);
    const double l0 = i0 > 0 ? s0[i0 - 1] : -1.0;
    const double l1 = i1 > 0 ? s1[i1 - 1] : -1.0;
    a.out_s[2] = (i0 > 0 && i1 > 0) ? fmin(l0, l1) : fmax(l0, l1);
    kk[0] = i0;
    kk[1] = i1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kk[0]; i += blockDim.x) {
    a.isq0[i] = 1.0 / sqrt(s0[i]);
    a.isv0[i] = 1.0 / s0[i];
  }
  for (int i = threadIdx.x; i < kk[1]; i += blockDim.x) {
    a.isq1[i] = 1.0 / sqrt(s1[i]);
    a.isv1[i] = 1.0 / s1[i];
  }
}

__global__ void corner_spectra_kernel(SpecArgs a) {
  __shared__ double dl[4];
  const int c = threadIdx.x;
  if (c < 4) {
    const double* s0 = a.sv[2 * c];
    const double* s1 = a.sv[2 * c + 1];
    const int n0 = a.nsv[2 * c], n1 = a.nsv[2 * c + 1];
    double tot = 0.0;
    for (int i = 0; i < n0; ++i) tot += s0[i];
    for (int i = 0; i < n1; ++i) tot += s1[i];
    if (!(tot > 0.0)) tot = 1.0;
    double* out = a.spec_new + (long long)c * a.len;
    int i0 = 0, i1 = 0;
    double d2 = 0.0;
    for (int k = 0; k < a.len; ++k) {
      const double v0 = i0 < n0 ? s0[i0] : -1.0;
      const double v1 = i1 < n1 ? s1[i1] : -1.0;
      double v;
      if (v0 < 0.0 && v1 < 0.0) {
        v = 0.0;
      } else if (v0 >= v1) {
        v = v0 / tot;
        ++i0;
      } else {
        v = v1 / tot;
        ++i1;
      }
      out[k] = v;
      if (a.have_old) {
        const double dd = v - a.spec_old[(long long)c * a.len + k];
        d2 += dd * dd;
      }
    }
    dl[c] = sqrt(d2);
  }
  __syncthreads();
  if (c == 0) {
    double v = a.have_old ? fmax(fmax(dl[0], dl[1]), fmax(dl[2], dl[3])) : 1e300;
    if (a.accumulate) v = fmax(v, *a.delta);
    *a.delta = v;
  }
}

}  // namespace

// ---------------------------------------------------------------- host ----
static unsigned grid_for(long long n, int per = 256, unsigned cap = 4096) {
  long long g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

void fill(double* p, double v, size_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for((long long)n)), dim3(256), 0, s, p, (long long)n, v);
  HCTM_HIP(hipGetLastError());
}

void scale_block(double* p, int rows, int cols, long long ld, double alpha, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  if (ld < cols) throw Error(1, "scale_block: leading dimension below the column count");
  hipLaunchKernelGGL(scale_block_kernel, dim3(grid_for((long long)rows * cols)), dim3(256), 0, s, p, rows, cols, ld,
                     alpha);
  HCTM_HIP(hipGetLastError());
}

void random_fill(double* p, size_t n, uint64_t seed, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(random_kernel, dim3(grid_for((long long)n)), dim3(256), 0, s, p, (long long)n, seed);
  HCTM_HIP(hipGetLastError());
}

void norm2(const double* p, size_t n, double* out, double* part, hipStream_t s) {
  const unsigned g = grid_for((long long)n, 256, 1024);
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3(g), dim3(256), 0, s, p, (long long)n, part);
  HCTM_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, s, part, (int)g, out, 1);
  HCTM_HIP(hipGetLastError());
}

void sumsq(const double* p, size_t n, double* out, double* part, hipStream_t s) {
  const unsigned g = grid_for((long long)n, 256, 1024);
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3(g), dim3(256), 0, s, p, (long long)n, part);
  HCTM_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, s, part, (int)g, out, 0);
  HCTM_HIP(hipGetLastError());
}

void scale_inv(double* p, size_t n, const double* nrm, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(scale_inv_kernel, dim3(grid_for((long long)n)), dim3(256), 0, s, p, (long long)n, nrm);
  HCTM_HIP(hipGetLastError());
}

void chol_inv(const std::vector<SmallProb>& probs, hipStream_t s) {
  // one-elimination register kernel for n <= 256, the LDS/global one above
  std::vector<SmallProb> small, large;
  for (const SmallProb& p : probs) (p.n <= kGjMaxN ? small : large).push_back(p);
  for (int pass = 0; pass < 2; ++pass) {
    const std::vector<SmallProb>& v = pass == 0 ? small : large;
    for (size_t i = 0; i < v.size(); i += kMaxSmall) {
      SmallBatch b;
      b.n = 0;
      for (size_t j = i; j < v.size() && b.n < kMaxSmall; ++j) b.p[b.n++] = v[j];
      if (pass == 0) {
        int nmax = 1;
        for (int q = 0; q < b.n; ++q) nmax = std::max(nmax, b.p[q].n);
        // 16 x 16 threads up to n = kGj16Max, 32 x 32 beyond
        switch (nmax <= kGj16Max ? (nmax + 15) / 16 : 10 + (nmax + 31) / 32) {
          case 1: hipLaunchKernelGGL((chol_gj_kernel<16, 1>), dim3(b.n), dim3(256), 0, s, b); break;
          case 2: hipLaunchKernelGGL((chol_gj_kernel<16, 2>), dim3(b.n), dim3(256), 0, s, b); break;
          case 3: hipLaunchKernelGGL((chol_gj_kernel<16, 3>), dim3(b.n), dim3(256), 0, s, b); break;
          case 4: hipLaunchKernelGGL((chol_gj_kernel<16, 4>), dim3(b.n), dim3(256), 0, s, b); break;
          case 5: hipLaunchKernelGGL((chol_gj_kernel<16, 5>), dim3(b.n), dim3(256), 0, s, b); break;
          case 6: hipLaunchKernelGGL((chol_gj_kernel<16, 6>), dim3(b.n), dim3(256), 0, s, b); break;
          case 7: hipLaunchKernelGGL((chol_gj_kernel<16, 7>), dim3(b.n), dim3(256), 0, s, b); break;
          case 8: hipLaunchKernelGGL((chol_gj_kernel<16, 8>), dim3(b.n), dim3(256), 0, s, b); break;
          case 9: hipLaunchKernelGGL((chol_gj_kernel<16, 9>), dim3(b.n), dim3(256), 0, s, b); break;
          case 13: hipLaunchKernelGGL((chol_gj_kernel<32, 3>), dim3(b.n), dim3(1024), 0, s, b); break;
          case 14: hipLaunchKernelGGL((chol_gj_kernel<32, 4>), dim3(b.n), dim3(1024), 0, s, b); break;
          case 15: hipLaunchKernelGGL((chol_gj_kernel<32, 5>), dim3(b.n), dim3(1024), 0, s, b); break;
          case 16: hipLaunchKernelGGL((chol_gj_kernel<32, 6>), dim3(b.n), dim3(1024), 0, s, b); break;
          case 17: hipLaunchKernelGGL((chol_gj_kernel<32, 7>), dim3(b.n), dim3(1024), 0, s, b); break;
          default: hipLaunchKernelGGL((chol_gj_kernel<32, 8>), dim3(b.n), dim3(1024), 0, s, b); break;
        }
      } else
        hipLaunchKernelGGL(chol_inv_kernel, dim3(b.n), dim3(NT), 0, s, b);
      HCTM_HIP(hipGetLastError());
    }
  }
}

size_t jacobi_log_doubles(int n, int max_sweeps) {
  // (c, s) per pair per round: the sweeps over all columns, then those of the
  // leading phase over the trailing columns (at most as many)
  return 4 * (size_t)jacobi_pre_log_offset(n, max_sweeps);
}

void jacobi(const std::vector<SmallProb>& probs, hipStream_t s) {
  // LDS kernel where X fits in LDS, L2 kernel up to 256 x 256 with a scratch
  // copy, global-memory kernel otherwise; with V requested, the first two
  // log their rotations and V is rebuilt in parallel afterwards
  std::vector<SmallProb> lds, l2, glob;
  for (const SmallProb& p : probs) {
    if (p.n > 1024) throw Error(1, "jacobi: too many columns");
    const bool logok = !p.b || p.vlog;
    if ((long long)p.m * p.n <= kJacLds && p.n <= 160 && p.m <= kJacMaxRows && logok)
      lds.push_back(p);
    else if (p.work && p.m <= kJacL2Max && p.n <= kJacL2Max && logok)
      l2.push_back(p);
    else
      glob.push_back(p);
  }
  for (int kind = 0; kind < 2; ++kind) {
    const std::vector<SmallProb>& v = kind == 0 ? lds : l2;
    for (size_t i = 0; i < v.size(); i += kMaxSmall) {
      SmallBatch b, bv;
      b.n = bv.n = 0;
      int nmax = 0;
      for (size_t j = i; j < v.size() && b.n < kMaxSmall; ++j) {
        SmallProb p = v[j];
        p.b = v[j].b ? p.vlog : nullptr;  // the Jacobi kernel writes the rotation log
        b.p[b.n++] = p;
        if (v[j].b) {
          SmallProb q = v[j];
          q.a = v[j].b;  // V output
          q.b = v[j].vlog;
          bv.p[bv.n++] = q;
          nmax = std::max(nmax, q.n);
        }
      }
      int mmax = 0;
      for (int j = 0; j < b.n; ++j) mmax = std::max(mmax, b.p[j].m);
      const int rows = jacobi_rows_per_lane(mmax);
      if (kind == 0 && rows == 4)
        hipLaunchKernelGGL(jacobi_lds_kernel<4>, dim3(b.n), dim3(kJacNT), 0, s, b);
      else if (kind == 0 && rows == 8)
        hipLaunchKernelGGL(jacobi_lds_kernel<8>, dim3(b.n), dim3(kJacNT), 0, s, b);
      else if (kind == 0)
        hipLaunchKernelGGL(jacobi_lds_kernel<kJacRowsMax>, dim3(b.n), dim3(kJacNT), 0, s, b);
      else
        hipLaunchKernelGGL(jacobi_l2_kernel, dim3(b.n), dim3(kJacL2Threads), 0, s, b);
      HCTM_HIP(hipGetLastError());
      if (bv.n > 0) {
        hipLaunchKernelGGL(jacobi_v_kernel, dim3((nmax + kVRows - 1) / kVRows, bv.n), dim3(256), 0, s, bv);
        HCTM_HIP(hipGetLastError());
      }
    }
  }
  for (size_t i = 0; i < glob.size(); i += kMaxSmall) {
    SmallBatch b;
    b.n = 0;
    for (size_t j = i; j < glob.size() && b.n < kMaxSmall; ++j) b.p[b.n++] = glob[j];
    hipLaunchKernelGGL(jacobi_kernel, dim3(b.n), dim3(NT), 0, s, b);
    HCTM_HIP(hipGetLastError());
  }
}

void col_resid(const double* A, int lda, const double* B, int ldb, int n, int k, double* out, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(col_resid_kernel, dim3(k), dim3(256), 0, s, A, lda, B, ldb, n,
                     reinterpret_cast<unsigned long long*>(out));
  HCTM_HIP(hipGetLastError());
}

void ritz_resid(const double* GU, const double* U, const double* lam, int n, int ld, int k, double* out,
                hipStream_t s) {
  if (k <= 0 || n <= 0) return;
  hipLaunchKernelGGL(ritz_resid_kernel, dim3(k), dim3(256), 0, s, GU, U, lam, n, ld, out);
  HCTM_HIP(hipGetLastError());
}

void gather_cols(const double* X, int ldx, const int* perm, const double* sv, int m, int k, double* U, int ldu,
                 hipStream_t s) {
  const long long n = (long long)m * k;
  if (n == 0) return;
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, ldx, perm, sv, m, k,
                     U, ldu);
  HCTM_HIP(hipGetLastError());
}

void corner_spectra_delta(const SpecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(corner_spectra_kernel, dim3(1), dim3(64), 0, s, a);
  HCTM_HIP(hipGetLastError());
}

void select_states(const SelectArgs& a, hipStream_t s) {
  if (a.chi < 1 || a.chi > 8192 || a.n0 < 0 || a.n1 < 0) throw Error(1, "select_states: sizes out of range");
  size_t lds = sizeof(double) * (size_t)(std::min(a.n0, a.chi + 1) + std::min(a.n1, a.chi + 1));
  const int staged = lds <= 48 * 1024 ? 1 : 0;
  if (!staged) lds = 0;
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), lds, s, a, staged);
  HCTM_HIP(hipGetLastError());
}

}  // namespace hctm
