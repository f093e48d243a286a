// Host-only check of the block planners (no GPU): a contraction written
// straight into a permuted layout (plan_contract_permuted) must put every
// element where forming the product and permuting it (plan_contract +
// plan_permute) puts it.  Both sides are evaluated on the host with a plain
// triple loop in the same summation order, so the outputs must agree bit
// for bit, and every element of the permuted tensor must be written once.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "blocks.hpp"

using namespace hctm;

// C (row-major, ldc) = A B for one product description, host memory
static void host_gemm_plain(const GemmDesc& d) {
  for (int r = 0; r < d.M; ++r)
    for (int c = 0; c < d.N; ++c) {
      double s = 0.0;
      for (int k = 0; k < d.K; ++k) s += d.A[(long long)r * d.lda + k] * d.B[(long long)k * d.ldb + c];
      d.C[(long long)r * d.ldc + c] = s;
    }
}

static void host_copy(const CopyJob& j) {
  long long n = 1;
  for (int i = 0; i < j.r; ++i) n *= j.dims[i];
  for (long long e = 0; e < n; ++e) {
    long long rem = e, io = 0, oo = 0;
    for (int i = j.r - 1; i >= 0; --i) {
      const long long x = rem % j.dims[i];
      rem /= j.dims[i];
      io += x * j.istr[i];
      oo += x * j.ostr[i];
    }
    j.out[oo] = j.in[io];
  }
}

int main() {
  std::mt19937 rng(12345);
  std::uniform_int_distribution<int> dim(0, 3);
  std::normal_distribution<double> nd;
  int planned = 0, refused = 0, cases = 0;
  for (int trial = 0; trial < 60; ++trial) {
    Leg l[5];
    for (Leg& x : l) {
      x.e = dim(rng);
      x.o = dim(rng);
      if (x.e + x.o == 0) x.e = 1;
    }
    // A [l0 l1 | k], B [k | l2 l3], C = A B [l0 l1 | l2 l3]
    BT A, B;
    A.L = Layout({l[0], l[1], l[4]}, 2);
    B.L = Layout({l[4], l[2], l[3]}, 1);
    std::vector<double> a(A.L.size + 1), b(B.L.size + 1);
    for (double& x : a) x = nd(rng);
    for (double& x : b) x = nd(rng);
    A.p = a.data();
    A.capacity = A.L.size;
    B.p = b.data();
    B.capacity = B.L.size;
    int perm[4] = {0, 1, 2, 3};
    do {
      for (int nr = 1; nr <= 3; ++nr) {
        ++cases;
        // reference: form C, then permute it
        std::vector<double> cbuf(4096), ref(4096, 0.0), got(4096, 0.0);
        BT C{Layout(), cbuf.data(), (long long)cbuf.size()};
        std::vector<GemmDesc> g;
        plan_contract(A, B, C, 1.0, 0.0, g);
        bool empty_k = false;
        for (const GemmDesc& d : g) {
          if (d.K <= 0) empty_k = true;
          host_gemm_plain(d);
        }
        BT R{Layout(), ref.data(), (long long)ref.size()};
        Layout Lo;
        Lo.r = 4;
        Lo.nr = nr;
        Lo.tp = C.L.tp;
        for (int j = 0; j < 4; ++j) Lo.leg[j] = C.L.leg[perm[j]];
        Lo.finalize();
        R.L = Lo;
        std::vector<CopyJob> jobs;
        plan_permute(C, R, perm, jobs);
        for (const CopyJob& j : jobs) host_copy(j);
        // planned: products written straight into the permuted layout
        std::vector<double> vbuf(4096);
        BT V{Layout(), vbuf.data(), (long long)vbuf.size()};
        BT O{Layout(), got.data(), (long long)got.size()};
        std::vector<GemmDesc> parts;
        const bool ok = plan_contract_permuted(A, B, V, O, perm, nr, parts);
        if (ok == empty_k) {
          std::printf("FAIL: planned %d with an empty contraction %d\n", (int)ok, (int)empty_k);
          return 1;
        }
        if (!ok) {
          ++refused;
          continue;
        }
        ++planned;
        std::vector<int> writes(got.size(), 0);
        for (const GemmDesc& d : parts) {
          if (d.sc_T <= 0 || d.sc_R <= 0 || d.M % d.sc_T || d.N % d.sc_R) {
            std::printf("FAIL: bad scatter descriptor\n");
            return 1;
          }
          for (int r = 0; r < d.M; ++r)
            for (int c = 0; c < d.N; ++c) {
              double s = 0.0;
              for (int k = 0; k < d.K; ++k) s += d.A[(long long)r * d.lda + k] * d.B[(long long)k * d.ldb + c];
              const long long at = (r / d.sc_T) * d.sc_s[0] + (r % d.sc_T) * d.sc_s[1] +
                                   (c / d.sc_R) * d.sc_s[2] + (c % d.sc_R) * d.sc_s[3];
              double* p = d.C + at;
              if (p < got.data() || p >= got.data() + O.L.size) {
                std::printf("FAIL: store outside the permuted tensor\n");
                return 1;
              }
              *p = s;
              ++writes[p - got.data()];
            }
        }
        if (!(O.L.r == R.L.r && O.L.size == R.L.size)) {
          std::printf("FAIL: layouts differ\n");
          return 1;
        }
        for (long long e = 0; e < O.L.size; ++e)
          if (writes[e] != 1 || got[e] != ref[e]) {
            std::printf("FAIL: element %lld written %d times, %g against %g\n", e, writes[e], got[e], ref[e]);
            return 1;
          }
      }
    } while (std::next_permutation(perm, perm + 4));
  }
  std::printf("ok: %d cases, %d planned, %d left to the separate copy\n", cases, planned, refused);
  return 0;
}
