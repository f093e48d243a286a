// Small dense FP64 kernels for the truncated SVD of a parity block:
//   * reductions and scalings (Frobenius normalisation of C and T),
//   * a counter-based random start block for subspace iteration,
//   * Cholesky + triangular inverse of a small Gram matrix (CholeskyQR),
//   * one-sided (Hestenes) Jacobi SVD of a small square matrix,
//   * the merge of the two parity spectra and the truncation to chi.
// Each small problem is owned by one workgroup; several independent problems
// (the two parity sectors, the four corners) go in one launch.
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
        if (fmin(a, bb) <= small2 || fabs(g) <= tol * sqrt(a) * sqrt(bb)) continue;
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

// --------------------------------------------------------- truncation ----
// Merge the two descending spectra (even sector first on ties) and keep
// k = min(chi, #{s > tau * s_max}) (at least one).  Writes k_even, k_odd,
// s_max and the inverse square roots of the kept values per sector.
__global__ void select_kernel(SelectArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double s0 = a.n0 > 0 ? a.sv0[0] : -1.0;
  const double s1 = a.n1 > 0 ? a.sv1[0] : -1.0;
  const double smax = fmax(s0, s1);
  int i0 = 0, i1 = 0, k = 0;
  while (k < a.chi) {
    const double v0 = i0 < a.n0 ? a.sv0[i0] : -1.0;
    const double v1 = i1 < a.n1 ? a.sv1[i1] : -1.0;
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
  for (int i = 0; i < i0; ++i) {
    a.isq0[i] = 1.0 / sqrt(a.sv0[i]);
    a.isv0[i] = 1.0 / a.sv0[i];
  }
  for (int i = 0; i < i1; ++i) {
    a.isq1[i] = 1.0 / sqrt(a.sv1[i]);
    a.isv1[i] = 1.0 / a.sv1[i];
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
  if (c == 0) *a.delta = a.have_old ? fmax(fmax(dl[0], dl[1]), fmax(dl[2], dl[3])) : 1e300;
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
  for (size_t i = 0; i < probs.size(); i += kMaxSmall) {
    SmallBatch b;
    b.n = 0;
    for (size_t j = i; j < probs.size() && b.n < kMaxSmall; ++j) b.p[b.n++] = probs[j];
    hipLaunchKernelGGL(chol_inv_kernel, dim3(b.n), dim3(NT), 0, s, b);
    HCTM_HIP(hipGetLastError());
  }
}

void jacobi(const std::vector<SmallProb>& probs, hipStream_t s) {
  for (size_t i = 0; i < probs.size(); i += kMaxSmall) {
    SmallBatch b;
    b.n = 0;
    for (size_t j = i; j < probs.size() && b.n < kMaxSmall; ++j) {
      if (probs[j].n > 1024) throw Error(1, "jacobi: too many columns");
      b.p[b.n++] = probs[j];
    }
    hipLaunchKernelGGL(jacobi_kernel, dim3(b.n), dim3(NT), 0, s, b);
    HCTM_HIP(hipGetLastError());
  }
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
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(64), 0, s, a);
  HCTM_HIP(hipGetLastError());
}

}  // namespace hctm
