// Strided block copies: the "permute and reshape" step that moves parity
// blocks between the matrix views required by consecutive block products.
//
// A job copies one dense box; on the host, dimensions that are contiguous in
// both the source and the destination are merged first.  If the innermost
// (stride-1) dimension of source and destination coincide the copy streams
// along it; otherwise a 32 x 32 tile is staged through LDS so that both the
// reads and the writes are coalesced.  A destination-fast dimension shorter
// than the tile (a parity block of a double-layer leg, D^2 / 2 entries) is
// joined with the next destination dimension when the two are contiguous in
// the destination, so that a tile's writes are whole 256-byte runs.  Index
// arithmetic is 32-bit where a launch's element counts allow it.
#include <algorithm>

#include "hctm_internal.hpp"

namespace hctm {
namespace {

constexpr int TT = 32;
constexpr int kMaxJobs = 16;

struct KJob {
  const double* in;
  double* out;
  int nouter;
  int odims[kMaxRank];
  long long oi[kMaxRank], oo[kMaxRank];
  int na, nb;           // tiled dims: a = source-fast, b = destination-fast (na = 1 for streaming)
  long long ia, oa, ib, ob;
  int nlo;              // > 0: b = (b_hi, b_lo) with b_lo < nlo, source stride ib of b_lo and ihi of b_hi
  long long ihi;
  int tiles_a, tiles_b;
  long long start;
};

struct KBatch {
  KJob j[kMaxJobs];
  int n;
  long long total;
};

__device__ __forceinline__ int find_job(const KBatch& B, long long blk) {
  int ji = 0;
#pragma unroll 1
  for (int i = 1; i < B.n; ++i)
    if (blk >= B.j[i].start) ji = i;
  return ji;
}

// IT: unsigned (every count of the launch below 2^31) or unsigned long long
template <typename IT>
__device__ __forceinline__ void outer_offsets(const KJob& J, IT o, long long& bi, long long& bo) {
  bi = 0;
  bo = 0;
#pragma unroll 1
  for (int d = J.nouter - 1; d >= 0; --d) {
    const IT n = (IT)J.odims[d];
    const IT q = o / n;
    const IT x = o - q * n;
    o = q;
    bi += (long long)x * J.oi[d];
    bo += (long long)x * J.oo[d];
  }
}

// source offset of destination-fast index b
__device__ __forceinline__ long long b_source(const KJob& J, int b) {
  if (J.nlo == 0) return (long long)b * J.ib;
  const unsigned hi = (unsigned)b / (unsigned)J.nlo, lo = (unsigned)b - hi * (unsigned)J.nlo;
  return (long long)hi * J.ihi + (long long)lo * J.ib;
}

// transpose-type jobs: one 32x32 tile per block
template <typename IT>
__global__ __launch_bounds__(256) void copy_tile_kernel(KBatch B) {
  __shared__ double tile[TT][TT + 1];
  const long long blk = blockIdx.x;
  const KJob& J = B.j[find_job(B, blk)];
  IT local = (IT)(blk - J.start);
  const int tb = (int)(local % (IT)J.tiles_b);
  local /= (IT)J.tiles_b;
  const int ta = (int)(local % (IT)J.tiles_a);
  local /= (IT)J.tiles_a;
  long long bi, bo;
  outer_offsets<IT>(J, local, bi, bo);
  const int a0 = ta * TT, b0 = tb * TT;
  const int t = threadIdx.x;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ao = t & 31, bo_ = (t >> 5) + 8 * r;
    const int a = a0 + ao, b = b0 + bo_;
    if (a < J.na && b < J.nb) tile[bo_][ao] = J.in[bi + a * J.ia + b_source(J, b)];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int b_ = t & 31, a_ = (t >> 5) + 8 * r;
    const int a = a0 + a_, b = b0 + b_;
    if (a < J.na && b < J.nb) J.out[bo + a * J.oa + b * J.ob] = tile[b_][a_];
  }
}

// streaming jobs: element e of the flattened (outer x nb) space per thread
template <typename IT>
__global__ __launch_bounds__(256) void copy_stream_kernel(KBatch B) {
  const long long blk = blockIdx.x;
  const KJob& J = B.j[find_job(B, blk)];
  const IT e = (IT)(blk - J.start) * 256u + threadIdx.x;
  IT total = (IT)J.nb;
  for (int d = 0; d < J.nouter; ++d) total *= (IT)J.odims[d];
  if (e >= total) return;
  const IT outer = e / (IT)J.nb;
  const int x = (int)(e - outer * (IT)J.nb);
  long long bi, bo;
  outer_offsets<IT>(J, outer, bi, bo);
  J.out[bo + x * J.ob] = J.in[bi + x * J.ib];
}

struct Dim {
  int n;
  long long is, os;
};

}  // namespace

void copy_jobs(const std::vector<CopyJob>& jobs, hipStream_t s) {
  KBatch tiles, streams;
  tiles.n = streams.n = 0;
  tiles.total = streams.total = 0;
  // largest element or block count of each batch, for the index width
  long long big[2] = {0, 0};
  auto flush = [&](KBatch& b, bool tile) {
    if (b.n == 0) return;
    const bool narrow = big[tile] < (1LL << 31) && b.total * 256 < (1LL << 31);
    if (tile && narrow)
      hipLaunchKernelGGL(copy_tile_kernel<unsigned>, dim3((unsigned)b.total), dim3(256), 0, s, b);
    else if (tile)
      hipLaunchKernelGGL(copy_tile_kernel<unsigned long long>, dim3((unsigned)b.total), dim3(256), 0, s, b);
    else if (narrow)
      hipLaunchKernelGGL(copy_stream_kernel<unsigned>, dim3((unsigned)b.total), dim3(256), 0, s, b);
    else
      hipLaunchKernelGGL(copy_stream_kernel<unsigned long long>, dim3((unsigned)b.total), dim3(256), 0, s, b);
    HCTM_HIP(hipGetLastError());
    b.n = 0;
    b.total = 0;
    big[tile] = 0;
  };
  for (const CopyJob& cj : jobs) {
    // collect non-trivial dims
    std::vector<Dim> d;
    bool empty = false;
    for (int k = 0; k < cj.r; ++k) {
      if (cj.dims[k] == 0) empty = true;
      if (cj.dims[k] > 1) d.push_back({cj.dims[k], cj.istr[k], cj.ostr[k]});
    }
    if (empty) continue;
    if (d.empty()) d.push_back({1, 1, 1});
    // order by destination stride (descending), then merge dims contiguous in both
    std::stable_sort(d.begin(), d.end(), [](const Dim& x, const Dim& y) { return x.os > y.os; });
    std::vector<Dim> m;
    for (const Dim& x : d) {
      if (!m.empty()) {
        Dim& y = m.back();
        if (y.is == x.is * x.n && y.os == x.os * x.n) {
          y.n *= x.n;
          y.is = x.is;
          y.os = x.os;
          continue;
        }
      }
      m.push_back(x);
    }
    // destination-fast dim = last; source-fast = smallest source stride
    const int ib = (int)m.size() - 1;
    int ia = 0;
    for (int k = 1; k < (int)m.size(); ++k)
      if (m[k].is < m[ia].is) ia = k;
    KJob J;
    J.in = cj.in;
    J.out = cj.out;
    J.nb = m[ib].n;
    J.ib = m[ib].is;
    J.ob = m[ib].os;
    const bool tile = (ia != ib) && m[ib].is != 1;
    // a short destination-fast dim joins the next destination dim (b_hi)
    // when the two are contiguous in the destination
    int ihi = -1;
    J.nlo = 0;
    J.ihi = 0;
    if (tile && m[ib].n < TT && ib >= 1 && ib - 1 != ia && m[ib - 1].os == m[ib].os * m[ib].n &&
        (long long)m[ib - 1].n * m[ib].n < (1LL << 30)) {
      ihi = ib - 1;
      J.nlo = m[ib].n;
      J.ihi = m[ihi].is;
      J.nb = m[ihi].n * m[ib].n;
    }
    J.nouter = 0;
    for (int k = 0; k < (int)m.size(); ++k) {
      if (k == ib || k == ihi || (tile && k == ia)) continue;
      if (J.nouter >= kMaxRank) throw Error(1, "copy job rank too large");
      J.odims[J.nouter] = m[k].n;
      J.oi[J.nouter] = m[k].is;
      J.oo[J.nouter] = m[k].os;
      J.nouter++;
    }
    long long outer = 1;
    for (int k = 0; k < J.nouter; ++k) outer *= J.odims[k];
    KBatch& b = tile ? tiles : streams;
    if (b.n == kMaxJobs) flush(b, tile);
    big[tile] = std::max(big[tile], outer * J.nb * (tile ? (long long)m[ia].n : 1LL));
    if (tile) {
      J.na = m[ia].n;
      J.ia = m[ia].is;
      J.oa = m[ia].os;
      J.tiles_a = (J.na + TT - 1) / TT;
      J.tiles_b = (J.nb + TT - 1) / TT;
      J.start = b.total;
      b.total += outer * J.tiles_a * J.tiles_b;
    } else {
      J.na = 1;
      J.ia = J.oa = 0;
      J.tiles_a = J.tiles_b = 1;
      J.start = b.total;
      b.total += (outer * J.nb + 255) / 256;
    }
    b.j[b.n++] = J;
  }
  flush(tiles, true);
  flush(streams, false);
}

}  // namespace hctm
