// Construction kernels: the double layer in the eigenbasis of the swap
// (Sec. II A-B), the traced boundary environment, and small reductions used
// by the observables.
#include "hctm_internal.hpp"
#include "tensor.hpp"

namespace hctm {
namespace {

// out[a1,a2,a3,a4] = sum over the <= 2 entries of each basis row
//   c1 c2 c3 c4 * X[K1,K2,K3,K4],
// X[K1..K4] = sum_p w_p Aket_p[k1,k2,k3,k4] Abra_p[kb1,kb2,kb3,kb4], K = k*D + kb.
// The tensors A (d x D^4) are staged in LDS.
__global__ __launch_bounds__(256) void double_layer_basis_kernel(DLArgs g) {
  extern __shared__ double sA[];
  const int D = g.D, q = D * D;
  const int D4 = D * D * D * D;
  for (int i = threadIdx.x; i < g.d * D4; i += blockDim.x) sA[i] = g.A[i];
  __syncthreads();
  const long long n = (long long)q * q * q * q;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    int a[4];
    long long t = e;
    for (int i = 3; i >= 0; --i) {
      a[i] = (int)(t % q);
      t /= q;
    }
    double acc = 0.0;
    // loop over the <= 16 combinations of basis entries
    for (int c = 0; c < 16; ++c) {
      double coef = 1.0;
      int K[4];
      bool ok = true;
      for (int i = 0; i < 4; ++i) {
        const int which = (c >> i) & 1;
        const int Ki = g.tab_idx[2 * a[i] + which];
        if (Ki < 0) {
          ok = false;
          break;
        }
        K[i] = Ki;
        coef *= g.tab_c[2 * a[i] + which];
      }
      if (!ok) continue;
      int ik = 0, ib = 0;
      for (int i = 0; i < 4; ++i) {
        ik = ik * D + K[i] / D;
        ib = ib * D + K[i] % D;
      }
      double x = 0.0;
      for (int p = 0; p < g.npairs; ++p) x += g.w[p] * sA[g.ket[p] * D4 + ik] * sA[g.bra[p] * D4 + ib];
      acc += coef * x;
    }
    g.out[e] = acc;
  }
}

// Apply a q x q change of basis with <= 2 entries per row to every leg of a
// plain q^4 tensor: out[a1..a4] = sum c1..c4 in[K1..K4].
__global__ __launch_bounds__(256) void basis4_kernel(const double* __restrict__ in, double* __restrict__ out, int q,
                                                     const int* __restrict__ tab_idx,
                                                     const double* __restrict__ tab_c) {
  const long long n = (long long)q * q * q * q;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    int a[4];
    long long t = e;
    for (int i = 3; i >= 0; --i) {
      a[i] = (int)(t % q);
      t /= q;
    }
    double acc = 0.0;
    for (int c = 0; c < 16; ++c) {
      double coef = 1.0;
      long long idx = 0;
      bool ok = true;
      for (int i = 0; i < 4; ++i) {
        const int which = (c >> i) & 1;
        const int Ki = tab_idx[2 * a[i] + which];
        if (Ki < 0) {
          ok = false;
          break;
        }
        coef *= tab_c[2 * a[i] + which];
        idx = idx * q + Ki;
      }
      if (ok) acc += coef * in[idx];
    }
    out[e] = acc;
  }
}

// Traced boundary in frame r: with legs of a_r = legs (j - r) mod 4 of the
// plain tensor a[u,l,d,r] and b~ = U b,
//   C[d,r] = sum_{u,l} b~[u] b~[l] a_r[u,l,d,r],  T[l,d,r] = sum_u b~[u] a_r[u,l,d,r].
__global__ __launch_bounds__(256) void init_env_kernel(const double* __restrict__ a, int q, int rot,
                                                       const double* __restrict__ b, const int* __restrict__ tab_idx,
                                                       const double* __restrict__ tab_c, double* __restrict__ C,
                                                       double* __restrict__ T) {
  extern __shared__ double bt[];
  for (int al = threadIdx.x; al < q; al += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < 2; ++w) {
      const int K = tab_idx[2 * al + w];
      if (K >= 0) s += tab_c[2 * al + w] * b[K];
    }
    bt[al] = s;
  }
  __syncthreads();
  long long st[4];
  {
    const long long s0[4] = {(long long)q * q * q, (long long)q * q, (long long)q, 1};
    for (int j = 0; j < 4; ++j) st[j] = s0[(j - rot + 4) % 4];
  }
  const long long nT = (long long)q * q * q;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nT + (long long)q * q;
       e += (long long)gridDim.x * blockDim.x) {
    if (e < nT) {
      const int l = (int)(e / ((long long)q * q)), d = (int)((e / q) % q), r = (int)(e % q);
      double s = 0.0;
      for (int u = 0; u < q; ++u) s += bt[u] * a[u * st[0] + l * st[1] + d * st[2] + r * st[3]];
      T[e] = s;
    } else {
      const long long f = e - nT;
      const int d = (int)(f / q), r = (int)(f % q);
      double s = 0.0;
      for (int u = 0; u < q; ++u) {
        const double bu = bt[u];
        if (bu == 0.0) continue;
        for (int l = 0; l < q; ++l) s += bu * bt[l] * a[u * st[0] + l * st[1] + d * st[2] + r * st[3]];
      }
      C[f] = s;
    }
  }
}

// out[j] = sum_i x_j[i] * y_j[i] for a list of vector pairs (one block each)
__global__ __launch_bounds__(256) void dots_kernel(DotBatch b, double* scratch) {
  __shared__ double red[4];
  const DotJob& J = b.j[blockIdx.y];
  double* partial = scratch + 64 * blockIdx.y;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < J.n; i += (long long)gridDim.x * blockDim.x)
    s += J.x[i] * J.y[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = red[0] + red[1] + red[2] + red[3];
    partial[blockIdx.x] = t;
  }
}

__global__ void dots_finish_kernel(DotBatch b, const double* scratch, int nparts) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= b.n) return;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += scratch[64 * j + i];
  *b.j[j].out = s;
}

// Index of the pair (s <= s') among the d(d+1)/2 ordered pairs, and of
// (s < s') among the d(d-1)/2 strict pairs.
__device__ __forceinline__ int pair_le(int s, int t, int d) { return s * d - s * (s - 1) / 2 + (t - s); }
__device__ __forceinline__ int pair_lt(int s, int t, int d) { return s * (d - 1) - s * (s - 1) / 2 + (t - s - 1); }

__global__ void assemble_rho_kernel(const double* __restrict__ dots, int d, int mode, double* __restrict__ rho) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = (mode <= 1) ? d : d * d;
  if (mode == 0) {
    for (int i = 0; i < d * d; ++i) rho[i] = dots[i];
  } else if (mode == 1) {
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t) rho[s * d + t] = dots[s <= t ? pair_le(s, t, d) : pair_le(t, s, d)];
  } else if (mode == 2) {
    for (int s1 = 0; s1 < d; ++s1)
      for (int s2 = 0; s2 < d; ++s2)
        for (int t1 = 0; t1 < d; ++t1)
          for (int t2 = 0; t2 < d; ++t2)
            rho[(s1 * d + s2) * n + (t1 * d + t2)] = dots[(s1 * d + t1) * d * d + (s2 * d + t2)];
  } else {
    // dots: first the sym-sym block [P1][P2] with P = pair_le, then the
    // anti-anti block [Q1][Q2] with Q = pair_lt.
    const int ns = d * (d + 1) / 2, na = d * (d - 1) / 2;
    const double* ss = dots;
    const double* aa = dots + ns * ns;
    for (int s1 = 0; s1 < d; ++s1)
      for (int s2 = 0; s2 < d; ++s2)
        for (int t1 = 0; t1 < d; ++t1)
          for (int t2 = 0; t2 < d; ++t2) {
            const int P1 = s1 <= t1 ? pair_le(s1, t1, d) : pair_le(t1, s1, d);
            const int P2 = s2 <= t2 ? pair_le(s2, t2, d) : pair_le(t2, s2, d);
            double v = ss[P1 * ns + P2];
            if (s1 != t1 && s2 != t2) {
              const int Q1 = s1 < t1 ? pair_lt(s1, t1, d) : pair_lt(t1, s1, d);
              const int Q2 = s2 < t2 ? pair_lt(s2, t2, d) : pair_lt(t2, s2, d);
              const double sg = ((s1 < t1) == (s2 < t2)) ? 1.0 : -1.0;
              v += sg * aa[Q1 * na + Q2];
            }
            rho[(s1 * d + s2) * n + (t1 * d + t2)] = v;
          }
  }
  double tr = 0.0;
  for (int i = 0; i < n; ++i) tr += rho[i * n + i];
  for (int i = 0; i < n * n; ++i) rho[i] /= tr;
}

// Hermitian RDMs of a complex tensor from real dot products (see
// assemble_rho_complex in tensor.hpp): the entries on and above the diagonal
// are formed, those below are their conjugates, the diagonal is real; then
// everything is divided by the trace.
__global__ void assemble_rho_complex_kernel(const double* __restrict__ dots, int d, int two_site,
                                            double* __restrict__ re, double* __restrict__ im) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = two_site ? d * d : d;
  for (int I = 0; I < n; ++I)
    for (int J = I; J < n; ++J) {
      double vr, vi;
      if (!two_site) {
        const double* t = dots + 4 * pair_le(I, J, d);
        vr = t[0] - t[1];
        vi = t[2] - t[3];
      } else {
        const int s1 = I / d, s2 = I % d, t1 = J / d, t2 = J % d;
        const double* t = dots + 8 * ((s1 * d + t1) * d * d + (s2 * d + t2));
        const double l1r1 = t[0] - t[1], l2r2 = t[2] - t[3], l1r2 = t[4] - t[5], l2r1 = t[6] - t[7];
        vr = l1r1 - l2r2;
        vi = l1r2 + l2r1;
      }
      if (I == J) vi = 0.0;
      re[I * n + J] = vr;
      im[I * n + J] = vi;
      re[J * n + I] = vr;
      im[J * n + I] = -vi;
    }
  double tr = 0.0;
  for (int i = 0; i < n; ++i) tr += re[i * n + i];
  for (int i = 0; i < n * n; ++i) {
    re[i] /= tr;
    im[i] /= tr;
  }
}

__global__ void trace_products_kernel(const double* __restrict__ rho, int nrho, const double* __restrict__ h, int n,
                                      double* __restrict__ e) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < nrho; ++k)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) s += rho[(long long)k * n * n + i * n + j] * h[j * n + i];
  *e = s;
}

__global__ void swap_asym_kernel(const double* __restrict__ x, int D, double* __restrict__ part) {
  __shared__ double r1[4], r2[4];
  const int q = D * D;
  const long long n = (long long)q * q * q * q;
  double num = 0.0, den = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    long long t = e, se = 0, mul = 1;
    for (int i = 0; i < 4; ++i) {
      const int K = (int)(t % q);
      t /= q;
      const int sw = (K % D) * D + K / D;
      se += sw * mul;
      mul *= q;
    }
    const double a = x[e], b = x[se];
    num += (a - b) * (a - b);
    den += (a + b) * (a + b);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    num += __shfl_xor(num, o, 64);
    den += __shfl_xor(den, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    r1[threadIdx.x >> 6] = num;
    r2[threadIdx.x >> 6] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0] + r1[1] + r1[2] + r1[3];
    part[2 * blockIdx.x + 1] = r2[0] + r2[1] + r2[2] + r2[3];
  }
}

__global__ void swap_asym_finish(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double num = 0.0, den = 0.0;
  for (int i = 0; i < nb; ++i) {
    num += part[2 * i];
    den += part[2 * i + 1];
  }
  *out = den > 0.0 ? sqrt(num / den) : 0.0;
}

struct TraceArgs {
  const double* p[8];
  int n[8], ld[8];
  int nb;
};

// one block of 256 threads: thread t sums the diagonal entries i = t mod 256
// of every block, then a fixed-order tree reduction (deterministic)
__global__ __launch_bounds__(256) void trace_blocks_kernel(TraceArgs a, double* out) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = 0; b < a.nb; ++b)
    for (int i = t; i < a.n[b]; i += 256) s += a.p[b][(long long)i * a.ld[b] + i];
  red[t] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) *out = red[0];
}

__global__ void log_ratio_kernel(const double* __restrict__ z, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  *out = log(fabs(z[0])) + log(fabs(z[1])) - log(fabs(z[2])) - log(fabs(z[3]));
}

}  // namespace

void assemble_rho(const double* dots, int d, int mode, double* rho, hipStream_t s) {
  hipLaunchKernelGGL(assemble_rho_kernel, dim3(1), dim3(64), 0, s, dots, d, mode, rho);
  HCTM_HIP(hipGetLastError());
}

void trace_products(const double* rho, int nrho, const double* h, int n, double* e, hipStream_t s) {
  hipLaunchKernelGGL(trace_products_kernel, dim3(1), dim3(64), 0, s, rho, nrho, h, n, e);
  HCTM_HIP(hipGetLastError());
}

void swap_asym(const double* x, int D, double* part, double* out, hipStream_t s) {
  const int nb = 256;
  hipLaunchKernelGGL(swap_asym_kernel, dim3(nb), dim3(256), 0, s, x, D, part);
  HCTM_HIP(hipGetLastError());
  hipLaunchKernelGGL(swap_asym_finish, dim3(1), dim3(64), 0, s, part, nb, out);
  HCTM_HIP(hipGetLastError());
}

void trace_blocks(const double* const* p, const int* n, const int* ld, int nb, double* out, hipStream_t s) {
  if (nb < 0 || nb > 8) throw Error(1, "trace_blocks: at most 8 blocks");
  TraceArgs a;
  a.nb = nb;
  for (int i = 0; i < nb; ++i) {
    a.p[i] = p[i];
    a.n[i] = n[i];
    a.ld[i] = ld[i];
  }
  hipLaunchKernelGGL(trace_blocks_kernel, dim3(1), dim3(256), 0, s, a, out);
  HCTM_HIP(hipGetLastError());
}

void log_ratio(const double* z, double* out, hipStream_t s) {
  hipLaunchKernelGGL(log_ratio_kernel, dim3(1), dim3(64), 0, s, z, out);
  HCTM_HIP(hipGetLastError());
}

void double_layer_basis(const DLArgs& g, hipStream_t s) {
  const int q = g.D * g.D;
  const long long n = (long long)q * q * q * q;
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  const size_t lds = sizeof(double) * g.d * g.D * g.D * g.D * g.D;
  if (lds > 160 * 1024) throw Error(1, "double layer: d D^4 doubles exceed the LDS of a workgroup");
  hipLaunchKernelGGL(double_layer_basis_kernel, dim3((unsigned)blocks), dim3(256), lds, s, g);
  HCTM_HIP(hipGetLastError());
}

void basis4(const double* in, double* out, int q, const int* tab_idx, const double* tab_c, hipStream_t s) {
  const long long n = (long long)q * q * q * q;
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(basis4_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, q, tab_idx, tab_c);
  HCTM_HIP(hipGetLastError());
}

void init_env(const double* a, int q, int rot, const double* b, const int* tab_idx, const double* tab_c, double* C,
              double* T, hipStream_t s) {
  const long long n = (long long)q * q * q + (long long)q * q;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(init_env_kernel, dim3((unsigned)blocks), dim3(256), sizeof(double) * q, s, a, q, rot, b, tab_idx,
                     tab_c, C, T);
  HCTM_HIP(hipGetLastError());
}

void assemble_rho_complex(const double* dots, int d, int two_site, double* re, double* im, hipStream_t s) {
  hipLaunchKernelGGL(assemble_rho_complex_kernel, dim3(1), dim3(64), 0, s, dots, d, two_site, re, im);
  HCTM_HIP(hipGetLastError());
}

void dots(const std::vector<DotJob>& jobs, double* scratch, hipStream_t s) {
  constexpr int kParts = 64;
  for (size_t i = 0; i < jobs.size(); i += kMaxDots) {
    DotBatch b;
    b.n = 0;
    for (size_t j = i; j < jobs.size() && b.n < kMaxDots; ++j) b.j[b.n++] = jobs[j];
    hipLaunchKernelGGL(dots_kernel, dim3(kParts, b.n), dim3(256), 0, s, b, scratch);
    HCTM_HIP(hipGetLastError());
    hipLaunchKernelGGL(dots_finish_kernel, dim3(1), dim3(64), 0, s, b, scratch, kParts);
    HCTM_HIP(hipGetLastError());
  }
}

}  // namespace hctm
