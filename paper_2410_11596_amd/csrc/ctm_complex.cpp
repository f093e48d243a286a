// Complex iPEPS tensors (Sec. II C): directional CTMRG on a 1 x 1 cell in the
// real representation of the Hermitian structure.
//
// In the eigenbasis of the bra-ket swap the double layer of a complex tensor
// has real blocks of even total parity and imaginary blocks of odd total
// parity, and so has every tensor of the contraction.  Such a tensor
// X = X_re + i X_im is held as two real block tensors, X_re with the layout of
// total parity 0 and X_im (the imaginary parts) with total parity 1, X_im
// right after X_re in one buffer.  A product follows the multiplication rule
// of complex numbers, C_re = A_re B_re - A_im B_im, C_im = A_re B_im +
// A_im B_re: four real block products, each between half-size parity blocks,
// where complex dense products take four full-size real ones.
//
// Truncation: M = H_d H_u is decomposed through the real matrix
// R = D^-1 M D, D = diag(i^p) over the parities p of the cut (M's real blocks
// on the diagonal, its imaginary parts off it, the block (even row, odd
// column) negated): R = U S V^T gives M = (D U) S (D V)^dagger, so the kept
// states are all even and the projectors are
//   P_a = H_u (D V) S^-1/2,  (D V)_re = V on even rows, (D V)_im = V on odd rows,
//   P_b = S^-1/2 (D U)^dagger H_d, (D U)^dagger_re = U_even^T, _im = -U_odd^T.
// R couples the two sectors and is decomposed as one matrix.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ctm.hpp"

namespace hctm {

void Ctm::cmul(const BT& Ar, const BT& Ai, const BT& Br, const BT& Bi, BT& Cr, BT& Ci, const double* cscale,
               const double* rscale) {
  const long long cap = Cr.capacity;
  std::vector<GemmDesc> g;
  plan_contract(Ar, Br, Cr, 1.0, 0.0, g);  // sets Cr.L (total parity 0)
  Ci.p = Cr.p + Cr.L.size;
  Ci.capacity = cap - Cr.L.size;
  plan_contract(Ar, Bi, Ci, 1.0, 0.0, g);  // total parity 1
  for (GemmDesc& d : g) {
    d.cscale = cscale;
    d.rscale = rscale;
  }
  launch_gemms(g);
  plan_contract(Ai, Bi, Cr, -1.0, 1.0, g);
  plan_contract(Ai, Br, Ci, 1.0, 1.0, g);
  for (GemmDesc& d : g) {
    d.cscale = cscale;
    d.rscale = rscale;
  }
  launch_gemms(g);
}

bool Ctm::cmul_permuted(const BT& Ar, const BT& Ai, const BT& Br, const BT& Bi, double* vbuf, long long vcap,
                        BT& outr, BT& outi, const int* perm, int nr_out) {
  const long long cap = outr.capacity;
  std::vector<GemmDesc> g0, g1;
  BT V{Layout(), vbuf, vcap};
  if (!plan_contract_permuted(Ar, Br, V, outr, perm, nr_out, g0)) return false;
  outi.p = outr.p + outr.L.size;
  outi.capacity = cap - outr.L.size;
  if (!plan_contract_permuted(Ar, Bi, V, outi, perm, nr_out, g0)) return false;
  if (!plan_contract_permuted(Ai, Bi, V, outr, perm, nr_out, g1, -1.0, 1.0)) return false;
  if (!plan_contract_permuted(Ai, Br, V, outi, perm, nr_out, g1, 1.0, 1.0)) return false;
  launch_gemms(g0);
  launch_gemms(g1);
  return true;
}

void Ctm::cpermute(const BT& inr, const BT& ini, BT& outr, BT& outi, std::initializer_list<int> perm, int nr_out) {
  const long long cap = outr.capacity;
  permute(inr, outr, perm, nr_out);
  outi.p = outr.p + outr.L.size;
  outi.capacity = cap - outr.L.size;
  permute(ini, outi, perm, nr_out);
}

// both parts lie in one buffer: one norm over both
void Ctm::cnormalise(BT& r, BT& i) {
  if (i.L.size > 0 && i.p != r.p + r.L.size) throw Error(1, "cnormalise: parts not contiguous");
  const size_t n = (size_t)(r.L.size + i.L.size);
  norm2(r.p, n, misc_, part_, st_);
  scale_inv(r.p, n, misc_, st_);
}

// ------------------------------------------------------------- set-up ----
Ctm::Ctm(const double* A_re, const double* A_im, int d, int D, int chi, const Options& o, hipStream_t stream,
         void* workspace, size_t ws_bytes)
    : d_(d), D_(D), chi_(chi), opt_(o) {
  if (!o.cplx || o.form != 0 || o.Lx != 1 || o.Ly != 1 || o.c4v || o.precision != 0)
    throw Error(1, "complex tensors: Z2 form, 1 x 1 cell, directional moves, FP64 only");
  if (2 * d > kMaxPairs) throw Error(1, "complex tensors: d must be at most 8");
  cplx_ = true;
  q_ = D * D;
  cc_ = std::max(chi, q_);
  Lx_ = Ly_ = ns_ = 1;
  const int qo = (D * D - D) / 2;
  lq_ = Leg{q_ - qo, qo};
  if (stream) {
    st_ = stream;
  } else {
    HCTM_HIP(hipStreamCreate(&st_));
    own_stream_ = true;
  }
  const size_t need = workspace_bytes(d, D, chi, o);
  if (workspace) {
    if (ws_bytes < need) throw Error(2, "workspace smaller than ctm_workspace_size");
    mem_ = workspace;
  } else {
    if (hipMalloc(&mem_, need) != hipSuccess) {
      mem_ = nullptr;
      throw Error(2, "hipMalloc of the workspace failed");
    }
    own_mem_ = true;
  }
  ar_.base = reinterpret_cast<char*>(mem_);
  ar_.cap = need;
  plan_memory(false);
  HCTM_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_k_), 64 * sizeof(int), hipHostMallocDefault));
  HCTM_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_d_), (2 * (size_t)cc_ + kHostMisc) * sizeof(double),
                         hipHostMallocDefault));
  setup_complex(A_re, A_im);
}

void Ctm::setup_complex(const double* A_re, const double* A_im) {
  const int q = q_, D = D_, d = d_;
  std::vector<int> ti, tti;
  std::vector<double> tc, ttc;
  basis_table(D, true, ti, tc, tti, ttc);
  HCTM_HIP(hipMemcpy(tab_idx_, ti.data(), sizeof(int) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tab_c_, tc.data(), sizeof(double) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tabT_idx_, tti.data(), sizeof(int) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tabT_c_, ttc.data(), sizeof(double) * 2 * q, hipMemcpyHostToDevice));
  // [A_re; A_im]: physical index s of the real part, d + s of the imaginary part
  const long long nA = (long long)d * D * D * D * D;
  HCTM_HIP(hipMemcpy(A_, A_re, sizeof(double) * nA, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(A_ + nA, A_im, sizeof(double) * nA, hipMemcpyHostToDevice));
  std::vector<double> b(q, 0.0);
  if (opt_.boundary.empty()) {
    for (int k = 0; k < D; ++k) b[k * D + k] = 1.0;
  } else {
    b = opt_.boundary;
  }
  HCTM_HIP(hipMemcpy(b_, b.data(), sizeof(double) * q, hipMemcpyHostToDevice));

  // a = sum_s (A_re + i A_im)[s] (x) (A_re - i A_im)[s]:
  // real part A_re (x) A_re + A_im (x) A_im, imaginary part A_im (x) A_re - A_re (x) A_im
  DLArgs g{};
  g.A = A_;
  g.tab_idx = tab_idx_;
  g.tab_c = tab_c_;
  g.d = 2 * d;
  g.D = D;
  g.npairs = 2 * d;
  for (int s = 0; s < d; ++s) {
    g.ket[2 * s] = s;
    g.bra[2 * s] = s;
    g.w[2 * s] = 1.0;
    g.ket[2 * s + 1] = d + s;
    g.bra[2 * s + 1] = d + s;
    g.w[2 * s + 1] = 1.0;
  }
  g.out = a_plain_[0];
  double_layer_basis(g, st_);
  for (int s = 0; s < d; ++s) {
    g.ket[2 * s] = d + s;
    g.bra[2 * s] = s;
    g.w[2 * s] = 1.0;
    g.ket[2 * s + 1] = s;
    g.bra[2 * s + 1] = d + s;
    g.w[2 * s + 1] = -1.0;
  }
  g.out = a_plain_im_;
  double_layer_basis(g, st_);
  // pack: real part on the even-total blocks, imaginary part on the odd ones
  const long long s0[4] = {(long long)q * q * q, (long long)q * q, (long long)q, 1};
  std::vector<CopyJob> jobs;
  for (int r = 0; r < 4; ++r) {
    BT& tr = a_rot(0, r);
    BT& tI = a_rot_i_[r];
    long long str[4];
    for (int j = 0; j < 4; ++j) str[j] = s0[(j - r + 4) % 4];
    tr.L = Layout({lq_, lq_, lq_, lq_}, 2, 0);
    tI.L = Layout({lq_, lq_, lq_, lq_}, 2, 1);
    tI.p = tr.p + tr.L.size;
    tI.capacity = tr.capacity - tr.L.size;
    plan_pack(a_plain_[0], str, tr, true, jobs);
    plan_pack(a_plain_im_, str, tI, true, jobs);
  }
  launch_copies(jobs);

  // traced boundary (b real and even): C and T of each part
  for (int r = 0; r < 4; ++r) {
    for (int part = 0; part < 2; ++part) {
      init_env(part ? a_plain_im_ : a_plain_[0], q, r, b_, tab_idx_, tab_c_, plain_tmp_, plain_tmp2_, st_);
      BT& Cr = env(0, 2 * r);
      BT& Tr = env(0, 2 * r + 1);
      BT& C = part ? env_i_[2 * r] : Cr;
      BT& T = part ? env_i_[2 * r + 1] : Tr;
      C.L = Layout({lq_, lq_}, 1, part);
      T.L = Layout({lq_, lq_, lq_}, 1, part);
      if (part) {
        C.p = Cr.p + Cr.L.size;
        C.capacity = Cr.capacity - Cr.L.size;
        T.p = Tr.p + Tr.L.size;
        T.capacity = Tr.capacity - Tr.L.size;
      }
      const long long sc[2] = {q, 1};
      const long long stt[3] = {(long long)q * q, q, 1};
      plan_pack(plain_tmp_, sc, C, true, jobs);
      plan_pack(plain_tmp2_, stt, T, true, jobs);
      launch_copies(jobs);
    }
  }
  for (int i = 0; i < 8; ++i) cnormalise(env_[i], env_i_[i]);
  ccorner_spectra();
  sync();
}

// ------------------------------------------------------------ quadrant ----
void Ctm::cquadrant(int j) {
  const int iC = (2 * j) % 8, iT1 = (2 * j + 1) % 8, iT4 = (2 * j + 7) % 8;
  BT Xr{Layout(), mid1_, mid_cap_}, Xi;
  cmul(env_[iC], env_i_[iC], env_[iT1], env_i_[iT1], Xr, Xi);              // [c | u t]
  BT T4r{Layout(), mid2_, mid_cap_}, T4i;
  cpermute(env_[iT4], env_i_[iT4], T4r, T4i, {0, 1, 2}, 2);               // [w l | c]
  // both products written straight into their permuted layouts where
  // possible (the real form's enlarged corner does the same)
  const int pswap[4] = {0, 3, 2, 1}, pq[4] = {0, 2, 1, 3};
  BT Ypr{Layout(), big2_, big_cap_}, Ypi;
  if (!cmul_permuted(T4r, T4i, Xr, Xi, big1_, big_cap_, Ypr, Ypi, pswap, 2)) {
    BT Yr{Layout(), big1_, big_cap_}, Yi;
    cmul(T4r, T4i, Xr, Xi, Yr, Yi);                                        // [w l | u t]
    cpermute(Yr, Yi, Ypr, Ypi, {0, 3, 2, 1}, 2);                           // [w t | u l]
  }
  if (!cmul_permuted(Ypr, Ypi, a_rot(0, j), a_rot_i_[j % 4], big1_, big_cap_, quad(0, j), quad_i_[j % 4], pq, 2)) {
    BT Qr{Layout(), big1_, big_cap_}, Qi;
    cmul(Ypr, Ypi, a_rot(0, j), a_rot_i_[j % 4], Qr, Qi);                  // [w t | d r]
    cpermute(Qr, Qi, quad(0, j), quad_i_[j % 4], {0, 2, 1, 3}, 2);        // [w d | t r]
  }
}

// ---------------------------------------------------------------- move ----
void Ctm::cmove(int r) {
  mark(0);
  for (int i = 0; i < 4; ++i) {
    const int o = (r + i) % 4;
    if (!quad_ok_[o]) {
      cquadrant(o);
      quad_ok_[o] = 1;
    }
  }
  mark(1);
  const int o1 = r % 4, o2 = (r + 1) % 4, o3 = (r + 2) % 4, o4 = (r + 3) % 4;
  BT &Q1 = quad_[o1], &Q2 = quad_[o2], &Q3 = quad_[o3], &Q4 = quad_[o4];
  const int key = (r * kMaxCell + 0) * kMaxCell + 0;
  cmul(Q1, quad_i_[o1], Q2, quad_i_[o2], Hu_, Hu_i_);   // [W | E]
  cmul(Q3, quad_i_[o3], Q4, quad_i_[o4], Hd_, Hd_i_);   // [E | W]
  cmul(Hd_, Hd_i_, Hu_, Hu_i_, M_, M_i_);               // [E | E]
  // R = D^-1 M D: M_re's diagonal blocks, M_im's off-diagonal blocks with the
  // (even row, odd column) one negated; index order of the cut: even, odd
  const int n0 = (int)M_.L.rows[0], n1 = (int)M_.L.rows[1], n = n0 + n1;
  if (M_.L.cols[0] != n0 || M_.L.cols[1] != n1) throw Error(1, "cmove: M is not square per sector");
  R_.L = Layout({Leg{n, 0}, Leg{n, 0}}, 1);
  if (R_.L.size > R_.capacity) throw Error(2, "cmove: R capacity");
  {
    std::vector<CopyJob> jobs;
    auto blk = [&](const double* src, long long ld_src, int rows, int cols, double* dst) {
      if (rows == 0 || cols == 0) return;
      CopyJob j{};
      j.in = src;
      j.out = dst;
      j.r = 2;
      j.dims[0] = rows;
      j.dims[1] = cols;
      j.istr[0] = ld_src;
      j.istr[1] = 1;
      j.ostr[0] = n;
      j.ostr[1] = 1;
      jobs.push_back(j);
    };
    blk(M_.p + M_.L.off[0], M_.L.ld(0), n0, n0, R_.p);
    blk(M_.p + M_.L.off[1], M_.L.ld(1), n1, n1, R_.p + (long long)n0 * n + n0);
    blk(M_i_.p + M_i_.L.off[0], M_i_.L.ld(0), n0, n1, R_.p + n0);
    blk(M_i_.p + M_i_.L.off[1], M_i_.L.ld(1), n1, n0, R_.p + (long long)n0 * n);
    launch_copies(jobs);
    scale_block(R_.p + n0, n0, n1, n, -1.0, st_);
  }
  mark(2);
  truncated_svd(&R_, chi_, key, (uint64_t)records_.size());
  iters_prev_[key] = sec_[0].iters;
  mark(3);

  SvdSector& S = sec_[0];
  const int k = S.k;
  const Leg kn{k, 0};
  const Leg lE0 = Hu_.L.leg[2], lE1 = Hu_.L.leg[3];
  // D V as a structured [E | k] tensor: even rows real, odd rows imaginary
  BT Vr{Layout({lE0, lE1, kn}, 2, 0), const_cast<double*>(S.V), 0};
  BT Vi{Layout({lE0, lE1, kn}, 2, 1), const_cast<double*>(S.V) + (long long)n0 * k, 0};
  Vr.capacity = Vr.L.size;
  Vi.capacity = Vi.L.size;
  if (Vr.L.size != (long long)n0 * k || Vi.L.size != (long long)n1 * k) throw Error(1, "cmove: V layout");
  BT& Pa = Pa_[0];
  BT& Pai = Pa_i_[0];
  Pa.capacity = proj_cap_;
  cmul(Hu_, Hu_i_, Vr, Vi, Pa, Pai, S.isq, nullptr);    // [W | k]
  // (D U)^dagger as [k | E]: U_even^T real, -U_odd^T imaginary
  {
    std::vector<CopyJob> jobs;
    CopyJob a{};
    a.in = S.W;
    a.out = WH_;
    a.r = 2;
    a.dims[0] = k;
    a.dims[1] = n0;
    a.istr[0] = 1;
    a.istr[1] = k;
    a.ostr[0] = n0;
    a.ostr[1] = 1;
    if (n0 > 0 && k > 0) jobs.push_back(a);
    CopyJob b = a;
    b.in = S.W + (long long)n0 * k;
    b.out = WH_ + (long long)k * n0;
    b.dims[1] = n1;
    b.ostr[0] = n1;
    if (n1 > 0 && k > 0) jobs.push_back(b);
    launch_copies(jobs);
    scale_block(WH_ + (long long)k * n0, k, n1, n1, -1.0, st_);
  }
  // its columns are the row indices of M (those of H_d)
  const Leg lR0 = M_.L.leg[0], lR1 = M_.L.leg[1];
  BT Wr{Layout({kn, lR0, lR1}, 1, 0), WH_, (long long)k * n0};
  BT Wi{Layout({kn, lR0, lR1}, 1, 1), WH_ + (long long)k * n0, (long long)k * n1};
  if (Wr.L.size != (long long)k * n0 || Wi.L.size != (long long)k * n1) throw Error(1, "cmove: U layout");
  BT& Pb = Pb_[0];
  BT& Pbi = Pb_i_[0];
  Pb.capacity = proj_cap_;
  cmul(Wr, Wi, Hd_, Hd_i_, Pb, Pbi, nullptr, S.isq);    // [k | W]

  MoveRecord rec;
  rec.k_even = k;
  rec.k_odd = 0;
  rec.frame = r;
  rec.status = svd_status_;
  rec.iters[0] = S.iters;
  rec.sweeps[0] = S.sweeps;
  for (int i = 0; i < k; ++i) rec.spectrum.push_back(hspec(0)[i]);
  std::sort(rec.spectrum.begin(), rec.spectrum.end(), [](double x, double y) { return x > y; });
  const double sm = rec.spectrum.empty() ? 1.0 : rec.spectrum[0];
  for (double& v : rec.spectrum) v /= sm;
  records_.push_back(std::move(rec));

  // renormalisation of the left environment (1 x 1: the same site)
  const int iC1 = (2 * r) % 8, iT1 = (2 * r + 1) % 8, iT3 = (2 * r + 5) % 8, iC4 = (2 * r + 6) % 8,
            iT4 = (2 * r + 7) % 8;
  BT X1r{Layout(), mid1_, mid_cap_}, X1i;
  cmul(env_[iC1], env_i_[iC1], env_[iT1], env_i_[iT1], X1r, X1i);   // [c | u t]
  BT X2r{Layout(), mid2_, mid_cap_}, X2i;
  cpermute(X1r, X1i, X2r, X2i, {0, 1, 2}, 2);                       // [c u | t]
  BT T3r{Layout(), mid1_, mid_cap_}, T3i;
  cpermute(env_[iT3], env_i_[iT3], T3r, T3i, {0, 1, 2}, 2);         // [r u | x]
  BT Zr{Layout(), mid3_, mid_cap_}, Zi;
  cmul(T3r, T3i, env_[iC4], env_i_[iC4], Zr, Zi);                   // [r u | c]
  BT Zpr{Layout(), mid1_, mid_cap_}, Zpi;
  cpermute(Zr, Zi, Zpr, Zpi, {0, 2, 1}, 1);                         // [r | c u]
  BT T4r{Layout(), mid3_, mid_cap_}, T4i;
  cpermute(env_[iT4], env_i_[iT4], T4r, T4i, {0, 1, 2}, 2);         // [w l | c]
  BT Pasr{Layout(), big2_, big_cap_}, Pasi;
  cpermute(Pa, Pai, Pasr, Pasi, {0, 1, 2}, 1);                      // [c | u k]
  // G = T4 P_a [w l | u k] as [w k | u l], then H = G a [w k | e r] as
  // [w e | r k], written by the products where possible (P_a, in big2_, is
  // read while G goes to big1_; G is read while H goes to big2_)
  const int pg[4] = {0, 3, 2, 1}, ph[4] = {0, 2, 3, 1};
  BT Gpr{Layout(), big1_, big_cap_}, Gpi;
  if (!cmul_permuted(T4r, T4i, Pasr, Pasi, big1_, big_cap_, Gpr, Gpi, pg, 2)) {
    Gpr.p = big2_;
    BT Gr{Layout(), big1_, big_cap_}, Gi;
    cmul(T4r, T4i, Pasr, Pasi, Gr, Gi);                              // [w l | u k]
    cpermute(Gr, Gi, Gpr, Gpi, {0, 3, 2, 1}, 2);                    // [w k | u l]
  }
  double* other = Gpr.p == big1_ ? big2_ : big1_;
  BT Hpr{Layout(), other, big_cap_}, Hpi;
  if (!cmul_permuted(Gpr, Gpi, a_rot(0, r), a_rot_i_[r % 4], other, big_cap_, Hpr, Hpi, ph, 2)) {
    Hpr.p = Gpr.p;
    BT Hr{Layout(), other, big_cap_}, Hi;
    cmul(Gpr, Gpi, a_rot(0, r), a_rot_i_[r % 4], Hr, Hi);           // [w k | e r]
    cpermute(Hr, Hi, Hpr, Hpi, {0, 2, 3, 1}, 2);                    // [w e | r k]
  }
  cmul(Pb, Pbi, X2r, X2i, env_[iC1], env_i_[iC1]);                  // [k | t]
  cmul(Zpr, Zpi, Pa, Pai, env_[iC4], env_i_[iC4]);                  // [r | k]
  cmul(Pb, Pbi, Hpr, Hpi, env_[iT4], env_i_[iT4]);                  // [k | r k]
  cnormalise(env_[iC1], env_i_[iC1]);
  cnormalise(env_[iC4], env_i_[iC4]);
  cnormalise(env_[iT4], env_i_[iT4]);
  quad_ok_[r % 4] = 0;
  quad_ok_[(r + 3) % 4] = 0;
  mark(-1);
  eps_site_ = -1;
}

// ------------------------------------------------------ corner spectra ----
// The singular values of a structured corner C are those of the real
// R_C = D^-1 C D (the same block signs as R above).
void Ctm::ccorner_spectra() {
  std::vector<SmallProb> jp;
  SpecArgs a{};
  std::vector<CopyJob> jobs;
  std::vector<std::array<long long, 4>> neg;  // (offset in cmat_, rows, cols, ld) to negate
  for (int c = 0; c < 4; ++c) {
    BT& Cr = env_[2 * c];
    BT& Ci = env_i_[2 * c];
    const int m0 = (int)Cr.L.rows[0], m1 = (int)Cr.L.rows[1], c0 = (int)Cr.L.cols[0], c1 = (int)Cr.L.cols[1];
    const int m = m0 + m1, nn = c0 + c1;
    const long long slot = (long long)(2 * c) * cc_;
    double* mat = cmat_ + (long long)c * cc_ * cc_;
    a.sv[2 * c] = csv_ + slot;
    a.nsv[2 * c] = (m > 0 && nn > 0) ? nn : 0;
    a.sv[2 * c + 1] = csv_ + slot + cc_;
    a.nsv[2 * c + 1] = 0;
    if (m == 0 || nn == 0) continue;
    if ((long long)m * nn > (long long)cc_ * cc_) throw Error(1, "ccorner_spectra: corner too large");
    auto blk = [&](const double* src, long long ld_src, int rows, int cols, double* dst) {
      if (rows == 0 || cols == 0) return;
      CopyJob j{};
      j.in = src;
      j.out = dst;
      j.r = 2;
      j.dims[0] = rows;
      j.dims[1] = cols;
      j.istr[0] = ld_src;
      j.istr[1] = 1;
      j.ostr[0] = nn;
      j.ostr[1] = 1;
      jobs.push_back(j);
    };
    blk(Cr.p + Cr.L.off[0], Cr.L.ld(0), m0, c0, mat);
    blk(Cr.p + Cr.L.off[1], Cr.L.ld(1), m1, c1, mat + (long long)m0 * nn + c0);
    blk(Ci.p + Ci.L.off[0], Ci.L.ld(0), m0, c1, mat + c0);
    blk(Ci.p + Ci.L.off[1], Ci.L.ld(1), m1, c0, mat + (long long)m0 * nn);
    if (m0 > 0 && c1 > 0) neg.push_back({(long long)(mat - cmat_) + c0, m0, c1, nn});
    SmallProb p{};
    p.a = mat;
    p.m = m;
    p.n = nn;
    p.lda = nn;
    p.rel = 1.1e-16 * std::max(m, 8);
    p.max_sweeps = 40;
    p.info = kdev_ + 8;
    p.sv = csv_ + slot;
    p.perm = cperm_ + slot;
    p.work = cwork_ ? cwork_ + (mat - cmat_) : nullptr;
    jp.push_back(p);
  }
  launch_copies(jobs);
  for (const auto& t : neg) scale_block(cmat_ + t[0], (int)t[1], (int)t[2], t[3], -1.0, st_);
  jacobi(jp, st_);
  std::swap(cspec_, cspec_old_);
  a.spec_new = cspec_;
  a.spec_old = cspec_old_;
  a.len = cc_;
  a.have_old = have_old_spec_ ? 1 : 0;
  a.accumulate = 0;
  a.delta = misc_ + 16;
  corner_spectra_delta(a, st_);
  have_old_spec_ = true;
}

// ----------------------------------------------------------- observables ----
void Ctm::ccompute_epsilon() {
  if (eps_site_ == 0) return;
  auto E = [&](int i) -> BT& { return env_[i]; };
  auto Ei = [&](int i) -> BT& { return env_i_[i]; };
  BT TAr{Layout(), mid1_, mid_cap_}, TAi;
  cmul(E(0), Ei(0), E(1), Ei(1), TAr, TAi);                  // [a | U b]
  BT TAsr{Layout(), mid2_, mid_cap_}, TAsi;
  cpermute(TAr, TAi, TAsr, TAsi, {0, 1, 2}, 2);              // [a U | b]
  BT TOPr{Layout(), mid1_, mid_cap_}, TOPi;
  cmul(TAsr, TAsi, E(2), Ei(2), TOPr, TOPi);                 // [a U | c]
  BT TOPpr{Layout(), mid2_, mid_cap_}, TOPpi;
  cpermute(TOPr, TOPi, TOPpr, TOPpi, {1, 2, 0}, 2);          // [U c | a]
  BT T4pr{Layout(), mid3_, mid_cap_}, T4pi;
  cpermute(E(7), Ei(7), T4pr, T4pi, {2, 0, 1}, 1);           // [a | c' L]
  BT LTr{Layout(), big1_, big_cap_}, LTi;
  cmul(TOPpr, TOPpi, T4pr, T4pi, LTr, LTi);                  // [U c | c' L]
  BT LTpr{Layout(), big2_, big_cap_}, LTpi;
  cpermute(LTr, LTi, LTpr, LTpi, {0, 3, 1, 2}, 2);           // [U L | c c']
  BT S1r{Layout(), mid1_, mid_cap_}, S1i;
  cmul(E(4), Ei(4), E(5), Ei(5), S1r, S1i);                  // [e | Dn x]
  BT S1sr{Layout(), mid2_, mid_cap_}, S1si;
  cpermute(S1r, S1i, S1sr, S1si, {0, 1, 2}, 2);              // [e Dn | x]
  BT BOTr{Layout(), mid1_, mid_cap_}, BOTi;
  cmul(S1sr, S1si, E(6), Ei(6), BOTr, BOTi);                 // [e Dn | c']
  BT BOTsr{Layout(), mid2_, mid_cap_}, BOTsi;
  cpermute(BOTr, BOTi, BOTsr, BOTsi, {0, 1, 2}, 1);          // [e | Dn c']
  BT T2sr{Layout(), mid3_, mid_cap_}, T2si;
  cpermute(E(3), Ei(3), T2sr, T2si, {0, 1, 2}, 2);           // [c R | e]
  BT RB0r{Layout(), big1_, big_cap_}, RB0i;
  cmul(T2sr, T2si, BOTsr, BOTsi, RB0r, RB0i);                // [c R | Dn c']
  BT RBr{Layout(), quad_[0].p, quad_[0].capacity}, RBi;      // quadrant memory as scratch
  cpermute(RB0r, RB0i, RBr, RBi, {0, 3, 2, 1}, 2);           // [c c' | Dn R]
  quad_ok_[0] = 0;
  eps_.capacity = (long long)q_ * q_ * q_ * q_;
  cmul(LTpr, LTpi, RBr, RBi, eps_, eps_i_);                  // [U L | Dn R]
  eps_site_ = 0;
}

// The impurity A[s] (x) conj(A[sp]) (rotated, frame-rotated legs) is a
// general complex tensor X + i Y (X = imp_re, Y = imp_im on all blocks); it is
// written as S1 + i S2 with the structured S1 = (X even, Y odd) and
// S2 = (Y even, -X odd).  Both parts go to cimp_ (S1 then S2).
void Ctm::cimpurity(int s, int sp, int frame, BT& s1r, BT& s1i, BT& s2r, BT& s2i) {
  const int d = d_;
  const long long q = q_, q4 = q * q * q * q;
  DLArgs g{};
  g.A = A_;
  g.tab_idx = tab_idx_;
  g.tab_c = tab_c_;
  g.d = 2 * d;
  g.D = D_;
  g.npairs = 2;
  // X = A_re[s] A_re[sp] + A_im[s] A_im[sp] (ket first), into plain_tmp_
  g.ket[0] = s;
  g.bra[0] = sp;
  g.w[0] = 1.0;
  g.ket[1] = d + s;
  g.bra[1] = d + sp;
  g.w[1] = 1.0;
  g.out = plain_tmp_;
  double_layer_basis(g, st_);
  // Y = A_im[s] A_re[sp] - A_re[s] A_im[sp], into plain_tmp2_
  g.ket[0] = d + s;
  g.bra[0] = sp;
  g.w[0] = 1.0;
  g.ket[1] = s;
  g.bra[1] = d + sp;
  g.w[1] = -1.0;
  g.out = plain_tmp2_;
  double_layer_basis(g, st_);
  const long long s0[4] = {q * q * q, q * q, q, 1};
  long long str[4];
  for (int j = 0; j < 4; ++j) str[j] = s0[(j - frame + 4) % 4];
  const Layout L0({lq_, lq_, lq_, lq_}, 2, 0), L1({lq_, lq_, lq_, lq_}, 2, 1);
  s1r = BT{L0, cimp_, L0.size};
  s1i = BT{L1, cimp_ + L0.size, L1.size};
  s2r = BT{L0, cimp_ + q4, L0.size};
  s2i = BT{L1, cimp_ + q4 + L0.size, L1.size};
  std::vector<CopyJob> jobs;
  plan_pack(plain_tmp_, str, s1r, true, jobs);
  plan_pack(plain_tmp2_, str, s1i, true, jobs);
  plan_pack(plain_tmp2_, str, s2r, true, jobs);
  plan_pack(plain_tmp_, str, s2i, true, jobs);
  launch_copies(jobs);
  if (s2i.L.size > 0) {
    fill(misc_ + 30, -1.0, 1, st_);
    scale_inv(s2i.p, (size_t)s2i.L.size, misc_ + 30, st_);
  }
}

void Ctm::rdm1_complex(int x, int y, double* re, double* im) {
  (void)x;
  (void)y;
  ccompute_epsilon();
  const int d = d_;
  int np = 0;
  for (int s = 0; s < d; ++s)
    for (int t = s; t < d; ++t) {
      BT s1r, s1i, s2r, s2i;
      cimpurity(s, t, 0, s1r, s1i, s2r, s2i);
      if (s1r.L.size != eps_.L.size || s1i.L.size != eps_i_.L.size) throw Error(1, "rdm1_complex: layout");
      // rho = <eps, S1> + i <eps, S2>, <X, Y> = X_re.Y_re - X_im.Y_im
      dots({DotJob{eps_.p, s1r.p, eps_.L.size, dots_ + 4 * np},
            DotJob{eps_i_.p, s1i.p, eps_i_.L.size, dots_ + 4 * np + 1},
            DotJob{eps_.p, s2r.p, eps_.L.size, dots_ + 4 * np + 2},
            DotJob{eps_i_.p, s2i.p, eps_i_.L.size, dots_ + 4 * np + 3}},
           dpart_, st_);
      ++np;
    }
  assemble_rho_complex(dots_, d, 0, rho_, rho_ + d * d, st_);
  HCTM_HIP(hipMemcpyAsync(re, rho_, sizeof(double) * d * d, hipMemcpyDeviceToHost, st_));
  HCTM_HIP(hipMemcpyAsync(im, rho_ + d * d, sizeof(double) * d * d, hipMemcpyDeviceToHost, st_));
  sync();
}

}  // namespace hctm

namespace hctm {

// left half of the two-site environment in frame f, closed with a structured
// impurity (as Ctm::left_half); result [y R | z] in a halves slot
void Ctm::cleft_half(int f, const BT& ir, const BT& ii, BT& outr, BT& outi) {
  const int iC1 = (2 * f) % 8, iT1 = (2 * f + 1) % 8, iT3 = (2 * f + 5) % 8, iC4 = (2 * f + 6) % 8,
            iT4 = (2 * f + 7) % 8;
  BT TLr{Layout(), mid1_, mid_cap_}, TLi;
  cmul(env_[iC1], env_i_[iC1], env_[iT1], env_i_[iT1], TLr, TLi);   // [a | U y]
  BT T4r{Layout(), mid2_, mid_cap_}, T4i;
  cpermute(env_[iT4], env_i_[iT4], T4r, T4i, {0, 1, 2}, 2);         // [c' L | a]
  BT W1r{Layout(), big1_, big_cap_}, W1i;
  cmul(T4r, T4i, TLr, TLi, W1r, W1i);                               // [c' L | U y]
  BT W1pr{Layout(), big2_, big_cap_}, W1pi;
  cpermute(W1r, W1i, W1pr, W1pi, {0, 3, 2, 1}, 2);                  // [c' y | U L]
  BT V1r{Layout(), big1_, big_cap_}, V1i;
  cmul(W1pr, W1pi, ir, ii, V1r, V1i);                               // [c' y | Dn R]
  BT V1pr{Layout(), big2_, big_cap_}, V1pi;
  cpermute(V1r, V1i, V1pr, V1pi, {1, 3, 0, 2}, 2);                  // [y R | c' Dn]
  BT T3r{Layout(), mid1_, mid_cap_}, T3i;
  cpermute(env_[iT3], env_i_[iT3], T3r, T3i, {0, 1, 2}, 2);         // [z Dn | x]
  BT Sr{Layout(), mid2_, mid_cap_}, Si;
  cmul(T3r, T3i, env_[iC4], env_i_[iC4], Sr, Si);                   // [z Dn | c']
  BT BLr{Layout(), mid3_, mid_cap_}, BLi;
  cpermute(Sr, Si, BLr, BLi, {2, 1, 0}, 2);                         // [c' Dn | z]
  if (halves_used_ >= halves_max_) throw Error(1, "cleft_half: out of half slots");
  outr = BT{Layout(), halves_ + (long long)halves_used_ * halves_cap_, halves_cap_};
  ++halves_used_;
  cmul(V1pr, V1pi, BLr, BLi, outr, outi);                           // [y R | z]
}

void Ctm::cright_half(int f, const BT& ir, const BT& ii, BT& outr, BT& outi) {
  const int iT1 = (2 * f + 1) % 8, iC2 = (2 * f + 2) % 8, iT2 = (2 * f + 3) % 8, iC3 = (2 * f + 4) % 8,
            iT3 = (2 * f + 5) % 8;
  BT T1r{Layout(), mid1_, mid_cap_}, T1i;
  cpermute(env_[iT1], env_i_[iT1], T1r, T1i, {0, 1, 2}, 2);         // [y U | x]
  BT TRr{Layout(), mid2_, mid_cap_}, TRi;
  cmul(T1r, T1i, env_[iC2], env_i_[iC2], TRr, TRi);                 // [y U | c]
  BT W2r{Layout(), big1_, big_cap_}, W2i;
  cmul(TRr, TRi, env_[iT2], env_i_[iT2], W2r, W2i);                 // [y U | R c'']
  BT W2pr{Layout(), big2_, big_cap_}, W2pi;
  cpermute(W2r, W2i, W2pr, W2pi, {0, 3, 1, 2}, 2);                  // [y c'' | U R]
  BT ipr{Layout(), quad_[1].p, quad_[1].capacity}, ipi;              // quadrant memory as scratch
  quad_ok_[1] = 0;
  cpermute(ir, ii, ipr, ipi, {0, 3, 1, 2}, 2);                      // [u r | l d]
  BT V2r{Layout(), big1_, big_cap_}, V2i;
  cmul(W2pr, W2pi, ipr, ipi, V2r, V2i);                             // [y c'' | L Dn]
  BT V2pr{Layout(), big2_, big_cap_}, V2pi;
  cpermute(V2r, V2i, V2pr, V2pi, {0, 2, 1, 3}, 2);                  // [y L | c'' Dn]
  BT S2r{Layout(), mid1_, mid_cap_}, S2i;
  cmul(env_[iC3], env_i_[iC3], env_[iT3], env_i_[iT3], S2r, S2i);   // [c'' | Dn z]
  BT S2sr{Layout(), mid2_, mid_cap_}, S2si;
  cpermute(S2r, S2i, S2sr, S2si, {0, 1, 2}, 2);                     // [c'' Dn | z]
  if (halves_used_ >= halves_max_) throw Error(1, "cright_half: out of half slots");
  outr = BT{Layout(), halves_ + (long long)halves_used_ * halves_cap_, halves_cap_};
  ++halves_used_;
  cmul(V2pr, V2pi, S2sr, S2si, outr, outi);                         // [y L | z]
}

// rho2 of the pair (0,0)-(1,0) (dir 0) or (0,0)-(0,1) (dir 1) into device
// memory re, im (d^4 each): the halves of every impurity's two structured
// parts, their dots and the Hermitian assembly
void Ctm::rdm2c_dev(int dir, double* re, double* im) {
  const int f = dir == 0 ? 0 : 1;
  const int d = d_, d2 = d * d;
  halves_used_ = 0;
  std::vector<BT> L1r(d2), L1i(d2), L2r(d2), L2i(d2), R1r(d2), R1i(d2), R2r(d2), R2i(d2);
  for (int a = 0; a < d2; ++a) {
    BT s1r, s1i, s2r, s2i;
    cimpurity(a / d, a % d, f, s1r, s1i, s2r, s2i);
    cleft_half(f, s1r, s1i, L1r[a], L1i[a]);
    cleft_half(f, s2r, s2i, L2r[a], L2i[a]);
  }
  for (int b = 0; b < d2; ++b) {
    BT s1r, s1i, s2r, s2i;
    cimpurity(b / d, b % d, f, s1r, s1i, s2r, s2i);
    cright_half(f, s1r, s1i, R1r[b], R1i[b]);
    cright_half(f, s2r, s2i, R2r[b], R2i[b]);
  }
  std::vector<DotJob> jobs;
  for (int a = 0; a < d2; ++a)
    for (int b = 0; b < d2; ++b) {
      if (L1r[a].L.size != R1r[b].L.size || L1i[a].L.size != R1i[b].L.size) throw Error(1, "rdm2c: layout");
      double* o = dots_ + 8 * (a * d2 + b);
      jobs.push_back(DotJob{L1r[a].p, R1r[b].p, L1r[a].L.size, o + 0});
      jobs.push_back(DotJob{L1i[a].p, R1i[b].p, L1i[a].L.size, o + 1});
      jobs.push_back(DotJob{L2r[a].p, R2r[b].p, L2r[a].L.size, o + 2});
      jobs.push_back(DotJob{L2i[a].p, R2i[b].p, L2i[a].L.size, o + 3});
      jobs.push_back(DotJob{L1r[a].p, R2r[b].p, L1r[a].L.size, o + 4});
      jobs.push_back(DotJob{L1i[a].p, R2i[b].p, L1i[a].L.size, o + 5});
      jobs.push_back(DotJob{L2r[a].p, R1r[b].p, L2r[a].L.size, o + 6});
      jobs.push_back(DotJob{L2i[a].p, R1i[b].p, L2i[a].L.size, o + 7});
    }
  dots(jobs, dpart_, st_);
  assemble_rho_complex(dots_, d, 1, re, im, st_);
}

void Ctm::rdm2_complex(int x, int y, int dir, double* re, double* im) {
  (void)x;
  (void)y;
  const long long d4 = (long long)d_ * d_ * d_ * d_;
  rdm2c_dev(dir, rho_, rho_ + d4);
  HCTM_HIP(hipMemcpyAsync(re, rho_, sizeof(double) * d4, hipMemcpyDeviceToHost, st_));
  HCTM_HIP(hipMemcpyAsync(im, rho_ + d4, sizeof(double) * d4, hipMemcpyDeviceToHost, st_));
  sync();
}

// E = Re Tr(rho_h h) + Re Tr(rho_v h) for a real h: the real parts of the
// two Hermitian RDMs traced against h
double Ctm::energy_complex(const double* h_host) {
  const int n = d_ * d_;
  const long long d4 = (long long)n * n;
  rdm2c_dev(0, rho_, rho_ + 2 * d4);
  rdm2c_dev(1, rho_ + d4, rho_ + 3 * d4);
  HCTM_HIP(hipMemcpyAsync(hdev_, h_host, sizeof(double) * d4, hipMemcpyHostToDevice, st_));
  trace_products(rho_, 2, hdev_, n, misc_ + 20, st_);
  HCTM_HIP(hipMemcpyAsync(host_d_, misc_ + 20, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  return host_d_[0];
}

}  // namespace hctm
