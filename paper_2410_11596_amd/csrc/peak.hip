// Probes of the chip's own ceilings, against which the kernels' rates are
// also reported (beside the published peaks):
//   mfma_probe: back-to-back FP64 matrix-core products (v_mfma_f64_16x16x4f64)
//     with no memory traffic, eight independent accumulators per wave, every
//     SIMD holding several waves -- the FP64 MFMA rate at the clock the chip
//     sustains under that load;
//   stream_probe: a contiguous copy with one 16-byte non-temporal load and
//     store per thread -- the HBM copy bandwidth (read + write).
#include "hctm_internal.hpp"

namespace hctm {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kProbeAcc = 8;
constexpr int kProbeRounds = 32;

__global__ __launch_bounds__(256) void mfma_probe_kernel(double* sink, int iters) {
  const int lane = threadIdx.x & 63;
  const double a = 1e-3 * (1 + (lane & 7)), b = 1e-3 * (1 + (lane >> 3));
  v4d acc[kProbeAcc];
#pragma unroll
  for (int j = 0; j < kProbeAcc; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
  // kProbeRounds rounds per loop trip, so that the loop's own bookkeeping
  // (and any register moves around it) is small beside the products
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kProbeRounds; ++r)
#pragma unroll
      for (int j = 0; j < kProbeAcc; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kProbeAcc; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  sink[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// one 16-byte element per thread over the whole grid, with non-temporal
// loads and stores (measured on this chip: 6.6 TB/s for a 1 GiB copy, against
// 6.2 with ordinary accesses and 4.3-4.5 for grid-stride loops of 2-16 K
// workgroups)
__global__ __launch_bounds__(256) void stream_probe_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                                           long long n2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) {
    const double x = __builtin_nontemporal_load(&in[i].x);
    const double y = __builtin_nontemporal_load(&in[i].y);
    __builtin_nontemporal_store(x, &out[i].x);
    __builtin_nontemporal_store(y, &out[i].y);
  }
}

}  // namespace

double mfma_probe(double* sink, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(mfma_probe_kernel, dim3(blocks), dim3(256), 0, s, sink, iters);
  HCTM_HIP(hipGetLastError());
  // 4 waves per workgroup, kProbeRounds x kProbeAcc products of 16 x 16 x 4
  // (2048 flops) per loop trip
  return (double)blocks * 4 * iters * kProbeRounds * kProbeAcc * 2048.0;
}

void stream_probe(const double* in, double* out, long long n, hipStream_t s) {
  const long long n2 = n / 2;
  if ((n2 + 255) / 256 > 0x7fffffffLL) throw Error(1, "stream probe: too many elements");
  const unsigned blocks = (unsigned)((n2 + 255) / 256);
  if (n2 > 0) {
    hipLaunchKernelGGL(stream_probe_kernel, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const double2*>(in),
                       reinterpret_cast<double2*>(out), n2);
    HCTM_HIP(hipGetLastError());
  }
  if (n & 1) HCTM_HIP(hipMemcpyAsync(out + n - 1, in + n - 1, sizeof(double), hipMemcpyDeviceToDevice, s));
}

}  // namespace hctm
