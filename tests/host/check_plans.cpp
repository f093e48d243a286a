// Host-only check of the block planners (no GPU).  The per-sector products
// (plan_contract) and the block permutations (plan_permute) must agree with
// dense arithmetic on the full index space, and packing between a plain
// array and the blocks (plan_pack) must keep exactly the entries of the
// tensor's total parity.  A contraction written
// straight into a permuted layout (plan_contract_permuted) must put every
// element where forming the product and permuting it (plan_contract +
// plan_permute) puts it.  Both sides are evaluated on the host with a plain
// triple loop in the same summation order, so the outputs must agree bit
// for bit, and every element of the permuted tensor must be written once.
#include <algorithm>
#include <cmath>
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

// offset of index x of a run of n legs (row-major, sizes of all but the
// first in dd) with strides s: written out independently of the kernel's
static long long scatter_offset(int x, int n, const int* dd, const long long* s) {
  long long off = 0;
  for (int i = n - 1; i >= 0; --i) {
    const int size = i == 0 ? x + 1 : dd[i - 1];
    const int idx = i == 0 ? x : x % size;
    off += (long long)idx * s[i];
    if (i > 0) x /= size;
  }
  return off;
}

// dense array (row-major over the legs, each leg's even states first) of a
// block tensor; entries outside its blocks are zero
static std::vector<double> to_dense(const BT& x) {
  const Layout& L = x.L;
  long long n = 1;
  for (int i = 0; i < L.r; ++i) n *= L.leg[i].n();
  std::vector<double> d(n, 0.0);
  L.for_blocks([&](const int* p) {
    long long st[kMaxRank];
    const long long base = L.box(p, st);
    long long cnt = 1;
    for (int i = 0; i < L.r; ++i) cnt *= L.leg[i].d(p[i]);
    for (long long e = 0; e < cnt; ++e) {
      long long rem = e, src = base, dst = 0;
      int idx[kMaxRank];
      for (int i = L.r - 1; i >= 0; --i) {
        const int dim = L.leg[i].d(p[i]);
        idx[i] = (int)(rem % dim);
        rem /= dim;
        src += idx[i] * st[i];
      }
      for (int i = 0; i < L.r; ++i) dst = dst * L.leg[i].n() + (p[i] ? L.leg[i].e : 0) + idx[i];
      d[dst] = x.p[src];
    }
  });
  return d;
}

// the block planners against dense arithmetic: C = A B per sector equals the
// dense contraction over the shared leg, and a permutation of the blocks
// equals the dense transposition (total parities 0 and 1)
static int check_against_dense(std::mt19937& rng) {
  std::uniform_int_distribution<int> dim(0, 3);
  std::normal_distribution<double> nd;
  for (int trial = 0; trial < 40; ++trial) {
    Leg l[5];
    for (Leg& x : l) {
      x.e = dim(rng);
      x.o = dim(rng);
      if (x.e + x.o == 0) x.o = 1;
    }
    const int tpa = trial & 1, tpb = (trial >> 1) & 1;
    BT A, B;
    A.L = Layout({l[0], l[1], l[4]}, 2, tpa);
    B.L = Layout({l[4], l[2], l[3]}, 1, tpb);
    std::vector<double> a(A.L.size + 1), b(B.L.size + 1), c(8192, 0.0);
    for (double& x : a) x = nd(rng);
    for (double& x : b) x = nd(rng);
    A.p = a.data();
    B.p = b.data();
    A.capacity = A.L.size;
    B.capacity = B.L.size;
    BT C{Layout(), c.data(), (long long)c.size()};
    std::vector<GemmDesc> g;
    plan_contract(A, B, C, 1.0, 0.0, g);
    for (const GemmDesc& d : g) host_gemm_plain(d);
    const std::vector<double> da = to_dense(A), db = to_dense(B), dc = to_dense(C);
    const int n0 = l[0].n(), n1 = l[1].n(), n2 = l[2].n(), n3 = l[3].n(), nk = l[4].n();
    for (int i0 = 0; i0 < n0; ++i0)
      for (int i1 = 0; i1 < n1; ++i1)
        for (int i2 = 0; i2 < n2; ++i2)
          for (int i3 = 0; i3 < n3; ++i3) {
            double s = 0.0;
            for (int k = 0; k < nk; ++k)
              s += da[((long long)i0 * n1 + i1) * nk + k] * db[((long long)k * n2 + i2) * n3 + i3];
            const double got = dc[(((long long)i0 * n1 + i1) * n2 + i2) * n3 + i3];
            if (std::abs(got - s) > 1e-12 * (1.0 + std::abs(s))) {
              std::printf("FAIL: block contraction differs from the dense one\n");
              return 1;
            }
          }
    // permutations of C against dense transposition
    int perm[4] = {0, 1, 2, 3};
    const int n[4] = {n0, n1, n2, n3};
    do {
      for (int nr = 0; nr <= 4; ++nr) {
        std::vector<double> o(8192, 0.0);
        BT O{Layout(), o.data(), (long long)o.size()};
        Layout Lo;
        Lo.r = 4;
        Lo.nr = nr;
        Lo.tp = C.L.tp;
        for (int j = 0; j < 4; ++j) Lo.leg[j] = C.L.leg[perm[j]];
        Lo.finalize();
        O.L = Lo;
        std::vector<CopyJob> jobs;
        plan_permute(C, O, perm, jobs);
        for (const CopyJob& j : jobs) host_copy(j);
        const std::vector<double> dO = to_dense(O);
        int idx[4];
        for (idx[0] = 0; idx[0] < n0; ++idx[0])
          for (idx[1] = 0; idx[1] < n1; ++idx[1])
            for (idx[2] = 0; idx[2] < n2; ++idx[2])
              for (idx[3] = 0; idx[3] < n3; ++idx[3]) {
                long long at = 0;
                for (int j = 0; j < 4; ++j) at = at * n[perm[j]] + idx[perm[j]];
                if (dO[at] != dc[(((long long)idx[0] * n1 + idx[1]) * n2 + idx[2]) * n3 + idx[3]]) {
                  std::printf("FAIL: block permutation differs from the dense transposition\n");
                  return 1;
                }
              }
      }
    } while (std::next_permutation(perm, perm + 4));
  }
  return 0;
}

// plan_pack between a plain array and the blocks, for every rank 1..4, row
// split and total parity, the plain array both row-major and with its legs
// stored in reverse order: packing keeps exactly the entries whose leg
// parities add up to the total parity (a leg's index is odd from its even
// count on), read back by an index walk of its own; unpacking into a zeroed
// array gives the masked plain array back
static int check_pack(std::mt19937& rng) {
  std::uniform_int_distribution<int> dim(0, 3);
  std::normal_distribution<double> nd;
  for (int trial = 0; trial < 60; ++trial) {
    const int r = 1 + trial % 4;
    for (int nr = 0; nr <= r; ++nr)
      for (int tp = 0; tp <= 1; ++tp)
        for (int rev = 0; rev <= 1; ++rev) {
          BT t;
          t.L.r = r;
          t.L.nr = nr;
          t.L.tp = tp;
          for (int i = 0; i < r; ++i) {
            t.L.leg[i].e = dim(rng);
            t.L.leg[i].o = dim(rng);
            if (t.L.leg[i].n() == 0) t.L.leg[i].o = 1;
          }
          t.L.finalize();
          int n[kMaxRank];
          long long total = 1;
          for (int i = 0; i < r; ++i) total *= (n[i] = t.L.leg[i].n());
          // plain strides: row-major over the legs, or over the legs reversed
          long long ps[kMaxRank];
          long long s = 1;
          for (int k = 0; k < r; ++k) {
            const int i = rev ? k : r - 1 - k;
            ps[i] = s;
            s *= n[i];
          }
          std::vector<double> plain(total), blocks(t.L.size + 1, 0.0), back(total, 0.0);
          for (double& x : plain) x = nd(rng);
          t.p = blocks.data();
          t.capacity = t.L.size;
          std::vector<CopyJob> jobs;
          plan_pack(plain.data(), ps, t, true, jobs);
          for (const CopyJob& j : jobs) host_copy(j);
          const std::vector<double> dense = to_dense(t);  // row-major over the legs
          std::vector<CopyJob> back_jobs;
          plan_pack(back.data(), ps, t, false, back_jobs);
          for (const CopyJob& j : back_jobs) host_copy(j);
          for (long long e = 0; e < total; ++e) {
            long long rem = e, at = 0;
            int par = 0;
            for (int i = r - 1; i >= 0; --i) {
              const int x = (int)(rem % n[i]);
              rem /= n[i];
              at += x * ps[i];
              par += x >= t.L.leg[i].e;
            }
            const double want = (par % 2 == tp) ? plain[at] : 0.0;
            if (dense[e] != want || back[at] != want) {
              std::printf("FAIL: plan_pack (rank %d, split %d, parity %d, reversed %d)\n", r, nr, tp, rev);
              return 1;
            }
          }
        }
  }
  return 0;
}

// every leg order and row split of the product of A and B: written straight
// into the permuted layout against formed and permuted, bit for bit, each
// element of the permuted tensor once; returns 1 on a mismatch
static int check_permuted(const BT& A, const BT& B, int r, int& cases, int& planned, int& refused) {
  int perm[kMaxRank];
  for (int j = 0; j < r; ++j) perm[j] = j;
  do {
    for (int nr = 1; nr < r; ++nr) {
      ++cases;
      // reference: form C, then permute it
      std::vector<double> cbuf(8192), ref(8192, 0.0), got(8192, 0.0);
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
      Lo.r = r;
      Lo.nr = nr;
      Lo.tp = C.L.tp;
      for (int j = 0; j < r; ++j) Lo.leg[j] = C.L.leg[perm[j]];
      Lo.finalize();
      R.L = Lo;
      std::vector<CopyJob> jobs;
      plan_permute(C, R, perm, jobs);
      for (const CopyJob& j : jobs) host_copy(j);
      // planned: products written straight into the permuted layout
      std::vector<double> vbuf(8192);
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
        if (d.sc_rn < 1 || d.sc_rn > 3 || d.sc_cn < 1 || d.sc_cn > 3) {
          std::printf("FAIL: bad scatter descriptor\n");
          return 1;
        }
        for (int rr = 0; rr < d.M; ++rr)
          for (int c = 0; c < d.N; ++c) {
            double s = 0.0;
            for (int k = 0; k < d.K; ++k) s += d.A[(long long)rr * d.lda + k] * d.B[(long long)k * d.ldb + c];
            const long long at = scatter_offset(rr, d.sc_rn, d.sc_rd, d.sc_rs) +
                                 scatter_offset(c, d.sc_cn, d.sc_cd, d.sc_cs);
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
  } while (std::next_permutation(perm, perm + r));
  return 0;
}

int main() {
  std::mt19937 rng(12345);
  if (check_against_dense(rng)) return 1;
  if (check_pack(rng)) return 1;
  std::uniform_int_distribution<int> dim3(0, 3), dim2(0, 2);
  std::normal_distribution<double> nd;
  int planned = 0, refused = 0, cases = 0;
  // row legs | column legs of the product: 2|2 (enlarged corners, edge),
  // 3|2 and 2|3 (HOTRG's coarse step), 1|3 and 3|1
  const int shapes[5][2] = {{2, 2}, {3, 2}, {2, 3}, {1, 3}, {3, 1}};
  for (int sh = 0; sh < 5; ++sh) {
    const int nra = shapes[sh][0], ncb = shapes[sh][1], r = nra + ncb;
    const int trials = r == 4 ? 60 : 12;
    for (int trial = 0; trial < trials; ++trial) {
      Leg l[kMaxRank + 1];
      for (int i = 0; i <= r; ++i) {
        l[i].e = r == 4 ? dim3(rng) : dim2(rng);
        l[i].o = r == 4 ? dim3(rng) : dim2(rng);
        if (l[i].e + l[i].o == 0) l[i].e = 1;
      }
      // A [rows | k], B [k | cols]; leg r is the contracted one
      BT A, B;
      A.L.r = nra + 1;
      A.L.nr = nra;
      for (int i = 0; i < nra; ++i) A.L.leg[i] = l[i];
      A.L.leg[nra] = l[r];
      A.L.tp = 0;
      A.L.finalize();
      B.L.r = ncb + 1;
      B.L.nr = 1;
      B.L.leg[0] = l[r];
      for (int i = 0; i < ncb; ++i) B.L.leg[1 + i] = l[nra + i];
      B.L.tp = 0;
      B.L.finalize();
      std::vector<double> a(A.L.size + 1), b(B.L.size + 1);
      for (double& x : a) x = nd(rng);
      for (double& x : b) x = nd(rng);
      A.p = a.data();
      A.capacity = A.L.size;
      B.p = b.data();
      B.capacity = B.L.size;
      if (check_permuted(A, B, r, cases, planned, refused)) return 1;
    }
  }
  std::printf("ok: %d cases, %d planned, %d left to the separate copy\n", cases, planned, refused);
  return 0;
}
