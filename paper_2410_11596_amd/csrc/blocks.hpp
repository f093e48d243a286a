// Z2 block-sparse tensors in a fused-sector matrix layout (host bookkeeping).
//
// In the eigenbasis of the bra-ket swap every leg splits into an even and an
// odd part (Sec. II B); a tensor of total parity tp only has blocks whose leg
// parities sum to tp mod 2.  A tensor is stored as a block-diagonal matrix
// between its row legs [0, nr) and column legs [nr, r):
//   sector P = parity of the row legs; its matrix has rows[P] rows (all row
//   parity tuples of sum P, lexicographic, first leg most significant, each a
//   row-major box) and cols[P ^ tp] columns, stored row-major at off[P].
// A contraction over the column legs of A and the row legs of B is then one
// GEMM per sector, and a leg permutation / change of row-column split is a
// list of strided block copies.  The plain (one-sector) form of the method is
// the same layout with every odd dimension zero.
#pragma once
#include <array>

#include "hctm_internal.hpp"

namespace hctm {

struct Leg {
  int e = 0, o = 0;
  int d(int p) const { return p ? o : e; }
  int n() const { return e + o; }
  bool operator==(const Leg& x) const { return e == x.e && o == x.o; }
};

struct Layout {
  int r = 0, nr = 0, tp = 0;
  std::array<Leg, kMaxRank> leg{};
  long long rows[2] = {0, 0}, cols[2] = {0, 0}, off[2] = {0, 0}, size = 0;

  static long long group_size(const Leg* l, int n, int P) {
    long long s = 0;
    for (int t = 0; t < (1 << n); ++t) {
      int par = 0;
      long long b = 1;
      for (int i = 0; i < n; ++i) {
        const int p = (t >> (n - 1 - i)) & 1;
        par ^= p;
        b *= l[i].d(p);
      }
      if (par == P) s += b;
    }
    return s;
  }
  // offset of the box with parities p[0..n) inside its fused group index
  static long long group_offset(const Leg* l, int n, const int* p) {
    int want = 0, key = 0;
    for (int i = 0; i < n; ++i) {
      want ^= p[i];
      key = (key << 1) | p[i];
    }
    long long s = 0;
    for (int t = 0; t < key; ++t) {
      int par = 0;
      long long b = 1;
      for (int i = 0; i < n; ++i) {
        const int q = (t >> (n - 1 - i)) & 1;
        par ^= q;
        b *= l[i].d(q);
      }
      if (par == want) s += b;
    }
    return s;
  }

  Layout() = default;
  Layout(std::initializer_list<Leg> legs, int nrow, int total_parity = 0) {
    r = 0;
    for (const Leg& l : legs) leg[r++] = l;
    nr = nrow;
    tp = total_parity;
    finalize();
  }
  void finalize() {
    for (int P = 0; P < 2; ++P) {
      rows[P] = group_size(leg.data(), nr, P);
      cols[P] = group_size(leg.data() + nr, r - nr, P);
    }
    off[0] = 0;
    off[1] = rows[0] * cols[tp];
    size = off[1] + rows[1] * cols[1 ^ tp];
  }
  long long ld(int P) const { return cols[P ^ tp]; }

  // address (element offset) of box p and the strides of each leg inside it
  long long box(const int* p, long long* stride) const {
    int P = 0;
    for (int i = 0; i < nr; ++i) P ^= p[i];
    const long long ldv = ld(P);
    const long long ro = group_offset(leg.data(), nr, p);
    const long long co = group_offset(leg.data() + nr, r - nr, p + nr);
    long long s = 1;
    for (int i = r - 1; i >= nr; --i) {
      stride[i] = s;
      s *= leg[i].d(p[i]);
    }
    s = ldv;
    for (int i = nr - 1; i >= 0; --i) {
      stride[i] = s;
      s *= leg[i].d(p[i]);
    }
    return off[P] + ro * ldv + co;
  }

  // all parity tuples of non-zero blocks (sum == tp), skipping empty boxes
  template <class F>
  void for_blocks(F f) const {
    for (int t = 0; t < (1 << r); ++t) {
      int p[kMaxRank];
      int par = 0;
      bool empty = false;
      for (int i = 0; i < r; ++i) {
        p[i] = (t >> (r - 1 - i)) & 1;
        par ^= p[i];
        if (leg[i].d(p[i]) == 0) empty = true;
      }
      if (par != tp || empty) continue;
      f(p);
    }
  }
};

struct BT {
  Layout L;
  double* p = nullptr;
  long long capacity = 0;  // elements available at p
};

// out = in with legs permuted: out leg j = in leg perm[j]; new row split nr_out.
inline void plan_permute(const BT& in, BT& out, const int* perm, std::vector<CopyJob>& jobs) {
  const Layout& Li = in.L;
  Layout& Lo = out.L;
  for (int j = 0; j < Li.r; ++j) {
    if (!(Lo.leg[j] == Li.leg[perm[j]])) throw Error(1, "plan_permute: leg mismatch");
  }
  if (Lo.tp != Li.tp || Lo.r != Li.r) throw Error(1, "plan_permute: parity/rank mismatch");
  if (Lo.size > out.capacity) throw Error(2, "plan_permute: output capacity");
  Lo.for_blocks([&](const int* po) {
    int pi[kMaxRank];
    for (int j = 0; j < Li.r; ++j) pi[perm[j]] = po[j];
    long long so[kMaxRank], si[kMaxRank];
    const long long bo = Lo.box(po, so);
    const long long bi = Li.box(pi, si);
    CopyJob cj;
    cj.in = in.p + bi;
    cj.out = out.p + bo;
    cj.r = Li.r;
    for (int j = 0; j < Li.r; ++j) {
      cj.dims[j] = Lo.leg[j].d(po[j]);
      cj.ostr[j] = so[j];
      cj.istr[j] = si[perm[j]];
    }
    jobs.push_back(cj);
  });
}

// C[rows A | cols B] (+)= alpha * A[rows A | K] B[K | cols B], one GEMM per sector.
inline void plan_contract(const BT& A, const BT& B, BT& C, double alpha, double beta, std::vector<GemmDesc>& g) {
  const Layout& La = A.L;
  const Layout& Lb = B.L;
  const int kr = La.r - La.nr;
  if (kr != Lb.nr) throw Error(1, "plan_contract: contracted rank mismatch");
  for (int i = 0; i < kr; ++i)
    if (!(La.leg[La.nr + i] == Lb.leg[i])) throw Error(1, "plan_contract: contracted leg mismatch");
  Layout& Lc = C.L;
  Lc.r = La.nr + (Lb.r - Lb.nr);
  Lc.nr = La.nr;
  Lc.tp = La.tp ^ Lb.tp;
  for (int i = 0; i < La.nr; ++i) Lc.leg[i] = La.leg[i];
  for (int i = 0; i < Lb.r - Lb.nr; ++i) Lc.leg[La.nr + i] = Lb.leg[Lb.nr + i];
  Lc.finalize();
  if (Lc.size > C.capacity) throw Error(2, "plan_contract: output capacity");
  for (int P = 0; P < 2; ++P) {
    const int Pk = P ^ La.tp;
    GemmDesc d{};
    d.M = (int)La.rows[P];
    d.K = (int)La.cols[Pk];
    d.N = (int)Lb.cols[Pk ^ Lb.tp];
    if (d.M == 0 || d.N == 0) continue;
    d.A = A.p + La.off[P];
    d.B = B.p + Lb.off[Pk];
    d.C = C.p + Lc.off[P];
    d.lda = (int)La.ld(P);
    d.ldb = (int)Lb.ld(Pk);
    d.ldc = (int)Lc.ld(P);
    d.ta = d.tb = 0;
    d.alpha = alpha;
    d.beta = beta;
    d.cscale = nullptr;
    d.rscale = nullptr;
    g.push_back(d);
  }
}

// out = alpha (A B) + beta out with its legs permuted (out leg j = leg
// perm[j] of the product, row split nr_out), written by the products: the
// product's layout is planned at C (never written; capacity checks only),
// each dense box of the permutation becomes one product over the rows and
// columns of its box with a scattered output.  For products with one to
// three row legs and one to three column legs; false (nothing planned)
// otherwise, or when a sector's contraction is empty.
inline bool plan_contract_permuted(const BT& A, const BT& B, BT& C, BT& out, const int* perm, int nr_out,
                                   std::vector<GemmDesc>& g, double alpha = 1.0, double beta = 0.0) {
  std::vector<GemmDesc> whole;
  plan_contract(A, B, C, alpha, beta, whole);
  const Layout& Lc = C.L;
  const int r = Lc.r, nrc = Lc.nr, ncc = Lc.r - Lc.nr;
  if (nrc < 1 || nrc > 3 || ncc < 1 || ncc > 3) return false;
  // an empty contracted sector would take the plain C = 0 path of gemm(),
  // which knows nothing of the scattered layout
  for (const GemmDesc& d : whole)
    if (d.K <= 0) return false;
  Layout L;
  L.r = r;
  L.nr = nr_out;
  L.tp = Lc.tp;
  for (int j = 0; j < r; ++j) L.leg[j] = Lc.leg[perm[j]];
  L.finalize();
  out.L = L;
  std::vector<CopyJob> jobs;
  plan_permute(C, out, perm, jobs);
  std::vector<GemmDesc> parts;
  for (const CopyJob& cj : jobs) {
    // the product whose output block holds this box
    const GemmDesc* src = nullptr;
    for (const GemmDesc& d : whole)
      if (cj.in >= d.C && cj.in < d.C + (long long)d.M * d.ldc) src = &d;
    if (!src) return false;
    const long long rel = cj.in - src->C;
    const long long row0 = rel / src->ldc, col0 = rel % src->ldc;
    long long dim[kMaxRank], is[kMaxRank], os[kMaxRank];  // per leg of the product
    for (int j = 0; j < r; ++j) {
      dim[perm[j]] = cj.dims[j];
      is[perm[j]] = cj.istr[j];
      os[perm[j]] = cj.ostr[j];
    }
    // the box is row-major in the product block: rows (its row legs, stride
    // ldc for the last), columns (its column legs, stride 1 for the last)
    long long rows = 1, cols = 1;
    for (int i = nrc - 1; i >= 0; --i) {
      if (is[i] != rows * src->ldc) return false;
      rows *= dim[i];
    }
    for (int i = r - 1; i >= nrc; --i) {
      if (is[i] != cols) return false;
      cols *= dim[i];
    }
    GemmDesc d = *src;
    d.A = src->A + row0 * src->lda;
    d.B = src->B + col0;
    d.C = cj.out;
    d.M = (int)rows;
    d.N = (int)cols;
    d.sc_rn = nrc;
    d.sc_cn = ncc;
    for (int q = 0; q < 2; ++q) {
      d.sc_rd[q] = q + 1 < nrc ? (int)dim[q + 1] : 1;
      d.sc_cd[q] = q + 1 < ncc ? (int)dim[nrc + q + 1] : 1;
    }
    for (int q = 0; q < 3; ++q) {
      d.sc_rs[q] = q < nrc ? os[q] : 0;
      d.sc_cs[q] = q < ncc ? os[nrc + q] : 0;
    }
    if (d.M > 0 && d.N > 0) parts.push_back(d);
  }
  g.insert(g.end(), parts.begin(), parts.end());
  return true;
}

// Copy between a plain dense array (row-major over legs, each leg with the
// even states first) and the blocks of a layout.  pstride[i] is the plain
// stride of the layout's leg i.  to_blocks = true packs, false unpacks.
inline void plan_pack(double* plain, const long long* pstride, BT& t, bool to_blocks, std::vector<CopyJob>& jobs) {
  const Layout& L = t.L;
  if (L.size > t.capacity) throw Error(2, "plan_pack: capacity");
  L.for_blocks([&](const int* p) {
    long long sb[kMaxRank];
    const long long bb = L.box(p, sb);
    long long pb = 0;
    for (int i = 0; i < L.r; ++i) pb += (p[i] ? L.leg[i].e : 0) * pstride[i];
    CopyJob cj;
    cj.r = L.r;
    for (int i = 0; i < L.r; ++i) cj.dims[i] = L.leg[i].d(p[i]);
    if (to_blocks) {
      cj.in = plain + pb;
      cj.out = t.p + bb;
      for (int i = 0; i < L.r; ++i) {
        cj.istr[i] = pstride[i];
        cj.ostr[i] = sb[i];
      }
    } else {
      cj.in = t.p + bb;
      cj.out = plain + pb;
      for (int i = 0; i < L.r; ++i) {
        cj.istr[i] = sb[i];
        cj.ostr[i] = pstride[i];
      }
    }
    jobs.push_back(cj);
  });
}

}  // namespace hctm
