// Directional CTMRG on an Lx x Ly unit cell in the eigenbasis of the bra-ket
// swap.
//
// Frames.  Every site (x, y) of the cell (x to the right, y downwards,
// periodic) has eight environment tensors in slots
//   0 C1[d,r]  1 T1[l,d,r]  2 C2[l,d]  3 T2[u,l,d]  4 C3[u,l]  5 T3[r,u,l]
//   6 C4[r,u]  7 T4[d,r,u]
// (legs counter-clockwise; C1 is the corner up-left of the site, T1 the edge
// above it, ...).  Turning the lattice by a quarter turn (old right leg
// becomes the up leg) maps slot i to slot i-2, so a move in any direction is
// the left move of a rotated frame r: its C1 is slot 2r, its T1 slot 2r+1,
// and the double layer is a_r with legs (j - r) mod 4 of a.  In frame r the
// frame's right is the cell direction (3 - r) mod 4 and its down (2 - r) mod 4
// (0 up, 1 left, 2 down, 3 right).  Moves are run in the order left (r=0),
// right (2), top (1), bottom (3).
//
// One left move of frame r sweeps the frame columns X = 0 .. LX-1.  At column
// X, for every frame row Y, the cut between rows Y and Y+1 takes its
// projectors from the 2x2 block of sites with top-left (X, Y); all products
// are block-diagonal GEMMs per parity sector:
//   quadrants  Q1 = C1 T1 T4 a of frame r at (X, Y), Q2 the same of frame r+1
//              at (X+1, Y), Q3 of frame r+2 at (X+1, Y+1), Q4 of frame r+3 at
//              (X, Y+1) (a quadrant is recomputed only after one of its
//              tensors changed);
//   halves     H_u = Q1 Q2, H_d = Q3 Q4, M = H_d H_u;
//   SVD        per sector, truncated to chi over the merged spectrum;
//   projectors P_a(Y) = H_u V S^-1/2, P_b(Y) = S^-1/2 W^T H_d.
// Then the left environment of column X+1 is replaced:
//   C1(X+1,Y) = P_b(Y-1) C1 T1,  T4(X+1,Y) = P_b(Y) T4 a P_a(Y-1),
//   C4(X+1,Y) = T3 C4 P_a(Y)     (C1, T1, T4, a, T3, C4 of site (X, Y)),
// each divided by its Frobenius norm.  With Lx = Ly = 1 this is the one-site
// move.  Tensors are stored as fused-sector block-diagonal matrices
// (blocks.hpp).
#include "ctm.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace hctm {

namespace {
constexpr int kDirectMax = 160;  // sectors up to this size are decomposed directly
constexpr int kWideBlock = 128;  // subspace width reached while a cut converges slowly
constexpr int kCornerSweeps = 24;  // Jacobi sweeps of a corner spectrum with its rotations logged
constexpr int kJacobiSweeps = 40;
// relative residual of the leading columns that ends the subspace iteration
constexpr double kSubspaceTol = 1e-12;
// with the block products in FP32 (BF16x3) the decomposed matrix itself
// carries relative errors of order 1e-7 (1e-5): resolving its subspace
// further buys nothing
constexpr double kSubspaceTolPrec[3] = {kSubspaceTol, 1e-8, 1e-6};
// apply M through the corners when the cut's last truncation took at most
// this many subspace iterations (forming M costs about as much as 8 of them)
constexpr int kImplicitIters = 7;
}

// ------------------------------------------------------------- memory ----
Ctm::Ctm(CountTag, int d, int D, int chi, int Lx, int Ly) : d_(d), D_(D), chi_(chi), Lx_(Lx), Ly_(Ly) {
  q_ = D * D;
  cc_ = std::max(chi, q_);
  ns_ = Lx * Ly;
}

size_t Ctm::workspace_bytes(int d, int D, int chi, const Options& o) {
  Ctm c(CountTag{}, d, D, chi, o.Lx, o.Ly);
  c.cplx_ = o.cplx != 0;
  c.plan_memory(true);
  return c.ar_.used + 256;
}

int Ctm::site(int x, int y) const {
  x = ((x % Lx_) + Lx_) % Lx_;
  y = ((y % Ly_) + Ly_) % Ly_;
  return y * Lx_ + x;
}

// cell offset (x, y) of the frame-r offset (X, Y)
static void to_cell(int r, int X, int Y, int& x, int& y) {
  switch (((r % 4) + 4) % 4) {
    case 0: x = X; y = Y; break;
    case 1: x = -Y; y = X; break;
    case 2: x = -X; y = -Y; break;
    default: x = Y; y = -X; break;
  }
}

int Ctm::site_of(int r, int X, int Y) const {
  int x, y;
  to_cell(r, X, Y, x, y);
  return site(x, y);
}

void Ctm::plan_memory(bool counting) {
  ar_.counting = counting;
  ar_.used = 0;
  const long long q = q_, cc = cc_, ncap = cc * q;
  const long long lcap = std::min<long long>(ncap, std::max<long long>(2LL * chi_ + 64, kDirectMax));
  l_cap_ = (int)lcap;
  const long long q4 = q * q * q * q;
  auto ti = [&](long long n) { return reinterpret_cast<int*>(ar_.take((size_t)((n + 1) / 2))); };
  tab_idx_ = ti(2 * q);
  tab_c_ = ar_.take(2 * q);
  tabT_idx_ = ti(2 * q);
  tabT_c_ = ar_.take(2 * q);
  const int ns = ns_;
  // a complex tensor is held as [A_re; A_im], 2 d physical states
  A_ = ar_.take((size_t)ns * (cplx_ ? 2 : 1) * d_ * D_ * D_ * D_ * D_);
  b_ = ar_.take((size_t)q);
  a_plain_.assign(ns, nullptr);
  for (int s = 0; s < ns; ++s) a_plain_[s] = ar_.take((size_t)q4);
  plain_tmp_ = ar_.take((size_t)q4);
  plain_tmp2_ = ar_.take((size_t)q4);
  a_rot_.assign(4 * ns, BT());
  for (BT& t : a_rot_) {
    t.p = ar_.take((size_t)q4);
    t.capacity = q4;
  }
  env_.assign(8 * ns, BT());
  for (int i = 0; i < 8 * ns; ++i) {
    const long long n = (i % 2 == 0) ? cc * cc : cc * cc * q;
    env_[i].p = ar_.take((size_t)n);
    env_[i].capacity = n;
  }
  quad_.assign(4 * ns, BT());
  quad_ok_.assign(4 * ns, 0);
  for (BT& t : quad_) {
    t.p = ar_.take((size_t)(ncap * ncap));
    t.capacity = ncap * ncap;
  }
  big_cap_ = ncap * ncap;
  big1_ = ar_.take((size_t)big_cap_);
  big2_ = ar_.take((size_t)big_cap_);
  mid_cap_ = cc * cc * q;
  mid1_ = ar_.take((size_t)mid_cap_);
  mid2_ = ar_.take((size_t)mid_cap_);
  mid3_ = ar_.take((size_t)mid_cap_);
  for (BT* t : {&Hu_, &Hd_, &M_}) {
    t->p = ar_.take((size_t)(ncap * ncap));
    t->capacity = ncap * ncap;
  }
  proj_cap_ = ncap * cc;
  const int ncut = std::max(Lx_, Ly_);
  Pa_.assign(ncut, BT());
  Pb_.assign(ncut, BT());
  for (int Y = 0; Y < ncut; ++Y) {
    Pa_[Y].p = ar_.take((size_t)proj_cap_);
    Pa_[Y].capacity = proj_cap_;
    Pb_[Y].p = ar_.take((size_t)proj_cap_);
    Pb_[Y].capacity = proj_cap_;
  }
  kg_.assign(4 * kMaxCell * kMaxCell, std::array<int, 2>{0, 0});
  iters_prev_.assign(4 * kMaxCell * kMaxCell, 0);
  chi_cut_.assign(4 * kMaxCell * kMaxCell, 0);
  // right vectors of the last truncation of every cut (warm starts)
  warm_cap_ = ncap * cc;
  warm_.assign(2 * 4 * kMaxCell * kMaxCell, WarmV());
  for (int r = 0; r < 4; ++r) {
    const int LX = (r % 2 == 0) ? Lx_ : Ly_, LY = (r % 2 == 0) ? Ly_ : Lx_;
    for (int X = 0; X < LX; ++X)
      for (int Y = 0; Y < LY; ++Y)
        for (int P = 0; P < 2; ++P) warm_[((r * kMaxCell + X) * kMaxCell + Y) * 2 + P].V = ar_.take((size_t)warm_cap_);
  }
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    S.Qr = ar_.take((size_t)(ncap * lcap));
    S.Ql = ar_.take((size_t)(ncap * lcap));
    S.Y = ar_.take((size_t)(ncap * lcap));
    S.Tm = ar_.take((size_t)(ncap * lcap));
    S.Qold = ar_.take((size_t)(ncap * lcap));
    S.C1 = ar_.take((size_t)(ncap * lcap));
    S.C2 = ar_.take((size_t)(ncap * lcap));
    S.G = ar_.take((size_t)(lcap * lcap));
    S.Ri = ar_.take((size_t)(lcap * lcap));
    S.B = ar_.take((size_t)(lcap * lcap));
    S.Bj = ar_.take((size_t)(lcap * lcap));
    S.Ub = ar_.take((size_t)(lcap * lcap));
    S.Vb = ar_.take((size_t)(lcap * lcap));
    S.Wbuf = ar_.take((size_t)(ncap * cc));
    S.Vbuf = ar_.take((size_t)(ncap * cc));
    S.sv = ar_.take((size_t)lcap);
    S.isq = ar_.take((size_t)lcap);
    S.isv = ar_.take((size_t)lcap);
    S.perm = ti(lcap);
    S.info = ti(8);
    // rotation log and column-major scratch of the Jacobi SVD (blocks up to
    // 256 x 256 run in LDS or L2)
    const int nj = (int)std::max<long long>(160, std::min<long long>(lcap, 256));
    S.vlog = ar_.take(jacobi_log_doubles(nj, kJacobiSweeps));
    S.jwork = ar_.take((size_t)nj * nj);
  }
  misc_ = ar_.take(64);
  kdev_ = ti(16);
  part_ = ar_.take(2048);
  cspec_ = ar_.take((size_t)(ns * 4 * cc));
  cspec_old_ = ar_.take((size_t)(ns * 4 * cc));
  csv_ = ar_.take((size_t)(ns * 8 * cc));
  cperm_ = ti(ns * 8 * cc);
  cmat_ = ar_.take((size_t)(ns * 8 * cc * cc));
  // column-major scratch that lets corner blocks beyond the LDS Jacobi (up
  // to 256 x 256) run in the L2-resident kernel
  cwork_ = cc <= 256 ? ar_.take((size_t)(ns * 8 * cc * cc)) : nullptr;
  // warm start of those decompositions: per block the right vectors of the
  // last one (two buffers, swapped at each update), the rotations of the new
  // one and their log
  if (cc <= 256) {
    const long long nb = (long long)ns * 8;
    cvec_[0] = ar_.take((size_t)(nb * cc * cc));
    cvec_[1] = ar_.take((size_t)(nb * cc * cc));
    cvj_ = ar_.take((size_t)(nb * cc * cc));
    clog_n_ = (long long)jacobi_log_doubles(cc, kCornerSweeps);
    clog_ = ar_.take((size_t)(nb * clog_n_));
    cinfo_ = ti((int)(2 * nb));  // each block's sweep counts: the replay of its log reads them
    cdims_.assign((size_t)nb, std::array<int, 2>{0, 0});
    ccur_.assign((size_t)nb, 0);
  }
  eps_.p = ar_.take((size_t)q4);
  eps_.capacity = q4;
  halves_cap_ = cc * cc * q;
  halves_max_ = (cplx_ ? 4 : 2) * d_ * d_;
  halves_ = ar_.take((size_t)(halves_max_ * halves_cap_));
  const long long d4 = (long long)d_ * d_ * d_ * d_;
  dots_ = ar_.take((size_t)((cplx_ ? 8 : 2) * d4 + 16));
  dpart_ = ar_.take((size_t)(64 * kMaxDots));
  rho_ = ar_.take((size_t)((cplx_ ? 4 : 2) * ns * d4 + 16));
  hdev_ = ar_.take((size_t)(d4 + 16));
  // split-K partial tiles: a few K slices of the tall n x l products of both
  // sectors, or of the l x l Gram matrices
  gemm_scratch_cap_ = std::max<long long>({1LL << 20, 24LL * lcap * lcap, 16LL * ncap * lcap});
  gemm_scratch_ = ar_.take((size_t)gemm_scratch_cap_);
  if (cplx_) {
    // the imaginary parts share the buffers of the real parts; extra: the
    // plain imaginary double layer, the real matrix R of the truncation, the
    // transposed left vectors and two impurities
    env_i_.assign(env_.size(), BT());
    quad_i_.assign(quad_.size(), BT());
    a_rot_i_.assign(a_rot_.size(), BT());
    Pa_i_.assign(Pa_.size(), BT());
    Pb_i_.assign(Pb_.size(), BT());
    a_plain_im_ = ar_.take((size_t)q4);
    R_.p = ar_.take((size_t)(ncap * ncap));
    R_.capacity = ncap * ncap;
    WH_ = ar_.take((size_t)(ncap * cc));
    cimp_ = ar_.take((size_t)(2 * q4));
  }
}

// ------------------------------------------------------------- set-up ----
Ctm::Ctm(const double* A_host, int d, int D, int chi, const Options& o, hipStream_t stream, void* workspace,
         size_t ws_bytes)
    : d_(d), D_(D), chi_(chi), opt_(o) {
  q_ = D * D;
  cc_ = std::max(chi, q_);
  Lx_ = o.Lx;
  Ly_ = o.Ly;
  ns_ = Lx_ * Ly_;
  const int qo = (D * D - D) / 2;
  lq_ = opt_.form == 0 ? Leg{q_ - qo, qo} : Leg{q_, 0};
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
  // pinned staging: the kept values of both sectors (cc_ each, cc_ >= chi >=
  // any kept count), then kHostMisc slots for scalars read back
  HCTM_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_d_), (2 * (size_t)cc_ + kHostMisc) * sizeof(double),
                         hipHostMallocDefault));
  setup(A_host);
}

Ctm::~Ctm() {
  if (st_) (void)hipStreamSynchronize(st_);
  for (hipEvent_t e : ev_) (void)hipEventDestroy(e);
  for (hipEvent_t e : gev_) (void)hipEventDestroy(e);
  if (host_k_) (void)hipHostFree(host_k_);
  if (host_d_) (void)hipHostFree(host_d_);
  if (own_mem_ && mem_) (void)hipFree(mem_);
  if (own_stream_ && st_) (void)hipStreamDestroy(st_);
}

void Ctm::sync() { HCTM_HIP(hipStreamSynchronize(st_)); }

void Ctm::launch_copies(std::vector<CopyJob>& jobs) {
  copy_jobs(jobs, st_);
  jobs.clear();
}

void Ctm::launch_gemms(std::vector<GemmDesc>& g) {
  if (low_prec_)
    for (GemmDesc& d : g) d.prec = opt_.precision;
  if (!opt_.profile) {
    gemm(g, st_, gemm_scratch_, gemm_scratch_cap_);
    g.clear();
    return;
  }
  obs_.c = this;
  gemm(g, st_, gemm_scratch_, gemm_scratch_cap_, &obs_);
  g.clear();
  if (gev_used_ >= 4096) flush_gemm_stats();
}

// profile mode: an event right before and right after every kernel launch
// of gemm(), so that the GEMM kernel and the split-K reduction are timed
// apart
void Ctm::Observer::mark(int kind, int phase, double flops) {
  if (c->gev_.size() < c->gev_used_ + 1) {
    hipEvent_t e;
    HCTM_HIP(hipEventCreate(&e));
    c->gev_.push_back(e);
  }
  HCTM_HIP(hipEventRecord(c->gev_[c->gev_used_], c->st_));
  ++c->gev_used_;
  if (phase == 1) c->gflops_.push_back(kind == 0 ? flops : -1.0);
}

void Ctm::flush_gemm_stats() {
  if (gev_used_ == 0) return;
  sync();
  for (size_t i = 0; i < gev_used_ / 2; ++i) {
    float ms = 0.f;
    HCTM_HIP(hipEventElapsedTime(&ms, gev_[2 * i], gev_[2 * i + 1]));
    if (gflops_[i] >= 0.0) {
      gemm_stats.seconds += ms * 1e-3;
      gemm_stats.flops += gflops_[i];
      gemm_stats.launches += 1;
    } else {
      gemm_stats.reduce_seconds += ms * 1e-3;
      gemm_stats.reduce_launches += 1;
    }
  }
  gev_used_ = 0;
  gflops_.clear();
}

void Ctm::permute(const BT& in, BT& out, std::initializer_list<int> perm, int nr_out) {
  int pm[kMaxRank];
  int i = 0;
  for (int x : perm) pm[i++] = x;
  if (i != in.L.r) throw Error(1, "permute: rank");
  Layout L;
  L.r = in.L.r;
  L.nr = nr_out;
  L.tp = in.L.tp;
  for (int j = 0; j < L.r; ++j) L.leg[j] = in.L.leg[pm[j]];
  L.finalize();
  out.L = L;
  std::vector<CopyJob> jobs;
  plan_permute(in, out, pm, jobs);
  launch_copies(jobs);
}

void Ctm::contract(const BT& A, const BT& B, BT& C) {
  std::vector<GemmDesc> g;
  plan_contract(A, B, C, 1.0, 0.0, g);
  launch_gemms(g);
}

// (T4 P_a) a of the edge renormalisation as [w e | r k], from T4s [w l | c]
// (in a mid buffer) and P_a as [c | u k] (in big2_): G = T4s P_a [w l | u k]
// is written straight as [w k | u l], then H = G a [w k | e r] straight as
// [w e | r k]; where a product cannot be written permuted it is formed in
// one big buffer and permuted into the other (an input it overwrites is
// consumed by then).
BT Ctm::edge_product(const BT& T4s, const BT& Pas, const BT& a) {
  const int pg[4] = {0, 3, 2, 1}, ph[4] = {0, 2, 3, 1};
  BT G{Layout(), big1_, big_cap_};
  BT Gp{Layout(), big1_, big_cap_};  // P_a (big2_) is read while Gp is written
  if (!contract_permuted(T4s, Pas, G, Gp, pg, 2)) {
    Gp.p = big2_;
    contract(T4s, Pas, G);                   // [w l | u k]
    permute(G, Gp, {0, 3, 2, 1}, 2);         // [w k | u l]
  }
  double* other = Gp.p == big1_ ? big2_ : big1_;
  BT H{Layout(), other, big_cap_};
  BT Hp{Layout(), other, big_cap_};
  if (!contract_permuted(Gp, a, H, Hp, ph, 2)) {
    Hp.p = Gp.p;
    contract(Gp, a, H);                      // [w k | e r]
    permute(H, Hp, {0, 2, 3, 1}, 2);         // [w e | r k]
  }
  return Hp;
}

bool Ctm::contract_permuted(const BT& A, const BT& B, BT& C, BT& out, const int* perm, int nr_out) {
  std::vector<GemmDesc> g;
  if (!plan_contract_permuted(A, B, C, out, perm, nr_out, g)) return false;
  launch_gemms(g);
  return true;
}

void Ctm::normalise(BT& t) {
  norm2(t.p, (size_t)t.L.size, misc_, part_, st_);
  scale_inv(t.p, (size_t)t.L.size, misc_, st_);
}

void Ctm::setup(const double* A_host) {
  const int q = q_, D = D_;
  // basis U (rows) and U^T, at most two entries per row
  std::vector<int> ti, tti;
  std::vector<double> tc, ttc;
  basis_table(D, opt_.form == 0, ti, tc, tti, ttc);
  HCTM_HIP(hipMemcpy(tab_idx_, ti.data(), sizeof(int) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tab_c_, tc.data(), sizeof(double) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tabT_idx_, tti.data(), sizeof(int) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tabT_c_, ttc.data(), sizeof(double) * 2 * q, hipMemcpyHostToDevice));
  const long long nA = (long long)d_ * D * D * D * D;
  HCTM_HIP(hipMemcpy(A_, A_host, sizeof(double) * nA * ns_, hipMemcpyHostToDevice));
  std::vector<double> b(q, 0.0);
  if (opt_.boundary.empty()) {
    for (int k = 0; k < D; ++k) b[k * D + k] = 1.0;
  } else {
    b = opt_.boundary;
  }
  HCTM_HIP(hipMemcpy(b_, b.data(), sizeof(double) * q, hipMemcpyHostToDevice));

  // double layer of every site in the rotated basis, a[U,L,Dn,R] = sum_s A[s] (x) A[s],
  // packed once per frame
  const long long s0[4] = {(long long)q * q * q, (long long)q * q, (long long)q, 1};
  std::vector<CopyJob> jobs;
  for (int st = 0; st < ns_; ++st) {
    DLArgs g;
    g.A = A_ + st * nA;
    g.out = a_plain_[st];
    g.tab_idx = tab_idx_;
    g.tab_c = tab_c_;
    g.d = d_;
    g.D = D;
    g.npairs = d_;
    for (int s = 0; s < d_; ++s) {
      g.ket[s] = s;
      g.bra[s] = s;
      g.w[s] = 1.0;
    }
    double_layer_basis(g, st_);
    for (int r = 0; r < 4; ++r) {
      BT& t = a_rot(st, r);
      t.L = Layout({lq_, lq_, lq_, lq_}, 2);
      long long str[4];
      for (int j = 0; j < 4; ++j) str[j] = s0[(j - r + 4) % 4];
      plan_pack(a_plain_[st], str, t, true, jobs);
    }
    launch_copies(jobs);
  }

  // traced boundary: in frame r, C1 of a site is the double layer at frame
  // offset (-1, -1) with its frame-up and frame-left legs traced, T1 the one
  // at (0, -1) with its frame-up leg traced
  for (int src = 0; src < ns_; ++src) {
    const int sx = src % Lx_, sy = src / Lx_;
    for (int r = 0; r < 4; ++r) {
      init_env(a_plain_[src], q, r, b_, tab_idx_, tab_c_, plain_tmp_, plain_tmp2_, st_);
      // the sites that see src at these offsets
      int cx, cy, ex, ey;
      to_cell(r, -1, -1, cx, cy);
      to_cell(r, 0, -1, ex, ey);
      BT& C = env(site(sx - cx, sy - cy), 2 * r);
      BT& T = env(site(sx - ex, sy - ey), 2 * r + 1);
      C.L = Layout({lq_, lq_}, 1);
      T.L = Layout({lq_, lq_, lq_}, 1);
      const long long sc[2] = {q, 1};
      const long long stt[3] = {(long long)q * q, q, 1};
      plan_pack(plain_tmp_, sc, C, true, jobs);    // init_env wrote C to plain_tmp_
      plan_pack(plain_tmp2_, stt, T, true, jobs);   // and T to plain_tmp2_
      launch_copies(jobs);
    }
  }
  for (BT& t : env_) normalise(t);
  // spectra of the initial corners, so that the first iteration has a delta
  corner_spectra();
  sync();
}

void Ctm::corner_spectrum(int x, int y, int c, double* s) {
  const double* src = cspec_ + ((long long)site(x, y) * 4 + c) * cc_;
  HCTM_HIP(hipMemcpyAsync(host_d_, src, sizeof(double) * cc_, hipMemcpyDeviceToHost, st_));
  sync();
  std::memcpy(s, host_d_, sizeof(double) * cc_);
}

// ------------------------------------------------------------ quadrant ----
// quad(s, o) = C1 T1 T4 a of frame o at site s as a matrix [w d | t r].
void Ctm::quadrant(int s, int j) {
  BT& C = env(s, 2 * j);
  BT& T1 = env(s, 2 * j + 1);
  BT& T4 = env(s, 2 * j + 7);
  BT X{Layout(), mid1_, mid_cap_};
  contract(C, T1, X);                                    // [c | u t]
  BT T4s{Layout(), mid2_, mid_cap_};
  permute(T4, T4s, {0, 1, 2}, 2);                        // [w l | c]
  BT Y{Layout(), big1_, big_cap_};
  BT Yp{Layout(), big2_, big_cap_};
  // [w l | u t] written straight as [w t | u l] (the swap of l and t: each
  // lane's stores are short runs along l that fill whole lines in L2), else
  // formed and permuted
  const int pswap[4] = {0, 3, 2, 1};
  if (!contract_permuted(T4s, X, Y, Yp, pswap, 2)) {
    contract(T4s, X, Y);                                   // [w l | u t]
    permute(Y, Yp, {0, 3, 2, 1}, 2);                       // [w t | u l]
  }
  BT Qp{Layout(), big1_, big_cap_};
  // [w t | d r] written straight as [w d | t r] (one product per box of
  // the permutation), else formed and permuted
  const int perm[4] = {0, 2, 1, 3};
  if (contract_permuted(Yp, a_rot(s, j), Qp, quad(s, j), perm, 2)) return;
  contract(Yp, a_rot(s, j), Qp);                         // [w t | d r]
  permute(Qp, quad(s, j), {0, 2, 1, 3}, 2);              // [w d | t r]
}

// ---------------------------------------------------------------- SVD ----
// Oversampling of the subspace for a kept-state guess kg at a cut: 16 once
// the cut's subspace iteration converges within three iterations; before
// that half the guess (at least 32), and where chi ended the last truncation
// at this cut (the spectrum continues above the cutoff) widened to a block of
// up to 128 columns (at most 64 more than the guess): the tall products M Q
// cost the same for any block width up to 128, and the wider block converges
// faster where the spectrum is flat at the cut.
int Ctm::oversample(int kg, int key) const {
  const int it = iters_prev_[key];
  if (it > 0 && it <= 3) return 16;
  const int p = std::max(32, kg / 2);
  return (chi_cut_[key] && kg + p < kWideBlock) ? std::max(p, std::min(64, kWideBlock - kg)) : p;
}

// CholeskyQR of S->Y into Ql (ql) or Qr with S->passes passes per sector
// (1 inside the subspace iteration, 3 for its final iterate).  Buffer chain
// per sector: pass p reads Y (p = 0) or the previous pass's output and writes
// dst if (passes - 1 - p) is even, else the scratch Tm, so that the last
// pass always ends in dst.
void Ctm::orth(std::vector<SvdSector*>& ss, bool ql) {
  int pmax = 0;
  for (SvdSector* S : ss) {
    if (S->passes < 1 || S->passes > 3) throw Error(1, "orth: passes must be 1, 2 or 3");
    pmax = std::max(pmax, S->passes);
  }
  auto src_of = [&](SvdSector* S, int pass) -> const double* {
    double* dstq = ql ? S->Ql : S->Qr;
    return pass == 0 ? S->Y : (((S->passes - pass) % 2 == 0) ? dstq : S->Tm);
  };
  for (int pass = 0; pass < pmax; ++pass) {
    std::vector<SvdSector*> act;
    for (SvdSector* S : ss)
      if (pass < S->passes) act.push_back(S);
    std::vector<GemmDesc> g;
    for (SvdSector* S : act) {
      const double* src = src_of(S, pass);
      GemmDesc d{};
      d.A = src;
      d.B = src;
      d.C = S->G;
      d.M = S->l;
      d.N = S->l;
      d.K = S->n;
      d.lda = S->l;
      d.ldb = S->l;
      d.ldc = S->l;
      d.ta = 1;
      d.tb = 0;
      d.alpha = 1.0;
      d.beta = 0.0;
      g.push_back(d);
    }
    launch_gemms(g);
    std::vector<SmallProb> sp;
    for (SvdSector* S : act) {
      SmallProb p{};
      p.a = S->G;
      p.b = S->Ri;
      p.m = p.n = S->l;
      p.lda = p.ldb = S->l;
      // unit-diagonal (column-scaled) Gram; a small shift in the first pass
      // keeps the factorisation defined while the columns are nearly parallel
      // (a random start); once the basis is aligned it is lowered so that the
      // residual check below is not limited by it
      p.rel = pass == 0 ? S->rel0 : 0.0;
      p.flags = 1;
      p.sv = S->isv;  // column norms of the pass's input (kept for the check)
      p.info = S->info;
      sp.push_back(p);
    }
    chol_inv(sp, st_);
    for (SvdSector* S : act) {
      double* dstq = ql ? S->Ql : S->Qr;
      double* dst = ((S->passes - 1 - pass) % 2 == 0) ? dstq : S->Tm;
      GemmDesc d{};
      d.A = src_of(S, pass);
      d.B = S->Ri;
      d.C = dst;
      d.M = S->n;
      d.N = S->l;
      d.K = S->l;
      d.lda = S->l;
      d.ldb = S->l;
      d.ldc = S->l;
      d.alpha = 1.0;
      d.beta = 0.0;
      g.push_back(d);
    }
    launch_gemms(g);
  }
}

// Y = M Qr (trans = false) or Y = M^T Ql (trans = true) for every sector of
// ss.  With the matrix formed this is one block product; otherwise M is
// applied as the chain Q3 Q4 Q1 Q2 of the four enlarged corners (transposed
// and reversed for M^T), which costs 8 n^2 l per application instead of the
// 6 n^3 of forming H_u, H_d and M.
void Ctm::apply_M(std::vector<SvdSector*>& ss, bool trans) {
  std::vector<GemmDesc> g;
  if (!implicit_) {
    for (SvdSector* S : ss) {
      GemmDesc d{};
      d.A = S->Mp;
      d.B = trans ? S->Ql : S->Qr;
      d.C = S->Y;
      d.M = S->n;
      d.N = S->l;
      d.K = S->n;
      d.lda = S->n;
      d.ldb = S->l;
      d.ldc = S->l;
      d.ta = trans ? 1 : 0;
      d.alpha = 1.0;
      g.push_back(d);
    }
    launch_gemms(g);
    return;
  }
  static const int order_n[4] = {1, 0, 3, 2};  // Q2, then Q1, Q4, Q3
  static const int order_t[4] = {2, 3, 0, 1};  // Q3^T, then Q4^T, Q1^T, Q2^T
  for (int step = 0; step < 4; ++step) {
    const int qi = trans ? order_t[step] : order_n[step];
    const BT& Q = *impl_q_[qi];
    for (size_t c = 0; c < ss.size(); ++c) {
      SvdSector* S = ss[c];
      const int P = S == &sec_[1] ? 1 : 0;
      const double* src = step == 0 ? (trans ? S->Ql : S->Qr) : ((step % 2 == 1) ? S->C1 : S->C2);
      double* dst = step == 3 ? S->Y : ((step % 2 == 0) ? S->C1 : S->C2);
      const int rows = (int)Q.L.rows[P], cols = (int)Q.L.cols[P];
      GemmDesc d{};
      d.A = Q.p + Q.L.off[P];
      d.B = src;
      d.C = dst;
      d.M = trans ? cols : rows;
      d.N = S->l;
      d.K = trans ? rows : cols;
      d.lda = (int)Q.L.ld(P);
      d.ldb = S->l;
      d.ldc = S->l;
      d.ta = trans ? 1 : 0;
      d.alpha = 1.0;
      g.push_back(d);
    }
    launch_gemms(g);
  }
}

// H_u = Q1 Q2, H_d = Q3 Q4 and M = H_d H_u from the enlarged corners of the
// current cut (impl_q_).
void Ctm::form_M() {
  std::vector<GemmDesc> g;
  plan_contract(*impl_q_[0], *impl_q_[1], Hu_, 1.0, 0.0, g);
  plan_contract(*impl_q_[2], *impl_q_[3], Hd_, 1.0, 0.0, g);
  launch_gemms(g);
  plan_contract(Hd_, Hu_, M_, 1.0, 0.0, g);
  launch_gemms(g);
}

// Truncated SVD of both sector blocks of M (batched): randomized subspace
// iteration, Rayleigh-Ritz and one-sided Jacobi, or Jacobi on the block itself
// when it is small.  key selects the cut: its previous kept count guesses the
// subspace size, and its previous right vectors start the iteration (warm
// start) when the block size is unchanged.  A sector stops iterating once
// M Q_r lies in the span of the left basis to kSubspaceTol (leading columns,
// relative to the largest); its last iterate is re-orthonormalised to
// rounding.  At most the configured number of iterations run.  salt makes the
// random blocks differ between cuts.
void Ctm::truncated_svd(const BT* M, int chi, int key, uint64_t salt) {
  int* kg_io = kg_[key].data();
  implicit_ = M == nullptr;
  for (int attempt = 0; attempt < 4; ++attempt) {
    std::vector<SvdSector*> sub, all;
    bool restart = false;
    for (int P = 0; P < 2; ++P) {
      SvdSector& S = sec_[P];
      // M acts on the east cut: H_d H_u = Q3 Q4 Q1 Q2
      S.n = implicit_ ? (int)impl_q_[1]->L.cols[P] : (int)M->L.rows[P];
      S.Mp = implicit_ ? nullptr : M->p + M->L.off[P];
      S.k = 0;
      S.iters = 0;
      S.sweeps = 0;
      S.warm = false;
      S.fin = false;
      S.done = false;
      S.conv = false;
      if (S.n == 0) {
        S.trusted = 0;
        continue;
      }
      int kg = kg_io[P] > 0 ? kg_io[P] : chi;
      kg = std::min(kg, S.n);
      S.kg = kg;
      const int p = oversample(kg, key);
      S.l = std::min<int>(std::min(S.n, kg + p), l_cap_);
      S.direct = S.n <= kDirectMax || S.l >= S.n;
      if (S.direct && S.n > l_cap_) throw Error(1, "truncated_svd: sector too large for a direct decomposition");
      if (S.direct && implicit_) {
        // a retry's subspace (kept count + 64) reaches the sector size: the
        // block is decomposed directly, which needs M itself; form it from
        // the enlarged corners and restart this attempt on it
        form_M();
        implicit_ = false;
        M = &M_;
        --attempt;
        restart = true;
        break;
      }
      if (S.direct) {
        S.l = S.n;
        S.conv = true;
      }
      // all Ritz columns are decomposed (restricting the Rayleigh-Ritz step
      // to the leading ones gives up the oversampling's accuracy); the
      // trailing p/2 values are not trusted for the truncation
      S.kt = S.direct ? S.n : S.l;
      S.trusted = S.direct ? S.n : S.l - p / 2;
      all.push_back(&S);
      if (!S.direct) sub.push_back(&S);
    }
    if (restart) continue;
    // subspace iteration (both sectors batched)
    if (!sub.empty()) {
      // Start block Q_r.  Warm (the cut's previous right vectors V, k_w of
      // them, orthonormal): [V | R] with the random columns R made
      // orthogonal to V by one block Gram-Schmidt step, R -= V (V^T R); the
      // block only seeds the first product M Q_r, whose orthonormalisation
      // follows.  Cold: random columns orthonormalised by three CholeskyQR
      // passes.
      std::vector<CopyJob> jobs;
      std::vector<SvdSector*> cold;
      std::vector<GemmDesc> proj, rem;
      for (SvdSector* S : sub) {
        const int P = S == &sec_[1] ? 1 : 0;
        const uint64_t seed = opt_.seed * 0x9E3779B97F4A7C15ull + (salt << 4) + P + ((uint64_t)attempt << 2);
        const WarmV& w = warm_[key * 2 + P];
        S->warm = attempt == 0 && w.V && w.n == S->n && w.k > 0;
        random_fill(S->warm ? S->Qr : S->Y, (size_t)S->n * S->l, seed, st_);
        if (!S->warm) {
          S->passes = 3;
          cold.push_back(S);
          continue;
        }
        const int kw = std::min(w.k, S->l), pr = S->l - kw;
        CopyJob j{};
        j.in = w.V;
        j.out = S->Qr;
        j.r = 2;
        j.dims[0] = S->n;
        j.dims[1] = kw;
        j.istr[0] = w.k;
        j.istr[1] = 1;
        j.ostr[0] = S->l;
        j.ostr[1] = 1;
        jobs.push_back(j);
        if (pr == 0) continue;
        GemmDesc d{};  // G = V^T R (kw x pr)
        d.A = S->Qr;
        d.B = S->Qr + kw;
        d.C = S->G;
        d.M = kw;
        d.N = pr;
        d.K = S->n;
        d.lda = S->l;
        d.ldb = S->l;
        d.ldc = pr;
        d.ta = 1;
        d.alpha = 1.0;
        proj.push_back(d);
        GemmDesc e{};  // R -= V G
        e.A = S->Qr;
        e.B = S->G;
        e.C = S->Qr + kw;
        e.M = S->n;
        e.N = pr;
        e.K = kw;
        e.lda = S->l;
        e.ldb = pr;
        e.ldc = S->l;
        e.alpha = -1.0;
        e.beta = 1.0;
        rem.push_back(e);
      }
      launch_copies(jobs);
      launch_gemms(proj);
      launch_gemms(rem);
      for (SvdSector* S : cold) S->rel0 = 1e-10;
      if (!cold.empty()) orth(cold, false);  // Qr
      // Iterate; from the second iteration on, before a sector's new left
      // basis is formed, the residual of the leading columns of Y = M Q_r
      // outside the previous left basis (relative to the largest column)
      // decides whether this iterate is the final one.
      // the C4v scheme decomposes the enlarged corner itself, whose relative
      // spectral gaps are about the square roots of those of H_d H_u: twice
      // the iterations for the same damping of the discarded part
      const int T = std::max(1, opt_.svd_iters) * (opt_.c4v ? 2 : 1);
      std::vector<SvdSector*> act = sub;
      for (int t = 0; t < T && !act.empty(); ++t) {
        apply_M(act, false);  // Y = M Qr
        std::vector<GemmDesc> g;
        for (SvdSector* S : act) S->fin = t == T - 1;
        if (t >= 1) {
          std::vector<SvdSector*> chk = act;
          // C = Ql^T Y[:, :kc] (into G), P = Ql C (into Qold)
          for (SvdSector* S : chk) {
            const int kc = std::min(S->kg, S->l);
            GemmDesc d{};
            d.A = S->Ql;
            d.B = S->Y;
            d.C = S->G;
            d.M = S->l;
            d.N = kc;
            d.K = S->n;
            d.lda = S->l;
            d.ldb = S->l;
            d.ldc = kc;
            d.ta = 1;
            d.alpha = 1.0;
            g.push_back(d);
          }
          launch_gemms(g);
          for (SvdSector* S : chk) {
            const int kc = std::min(S->kg, S->l);
            GemmDesc d{};
            d.A = S->Ql;
            d.B = S->G;
            d.C = S->Qold;
            d.M = S->n;
            d.N = kc;
            d.K = S->l;
            d.lda = S->l;
            d.ldb = kc;
            d.ldc = kc;
            d.alpha = 1.0;
            g.push_back(d);
          }
          launch_gemms(g);
          for (size_t c = 0; c < chk.size(); ++c) {
            SvdSector* S = chk[c];
            const int kc = std::min(S->kg, S->l);
            fill(misc_ + 48 + 2 * c, 0.0, 2, st_);
            col_resid(S->Y, S->l, S->Qold, kc, S->n, kc, misc_ + 48 + 2 * c, st_);
          }
          HCTM_HIP(hipMemcpyAsync(hmisc(), misc_ + 48, sizeof(double) * 2 * chk.size(),
                                  hipMemcpyDeviceToHost, st_));
          sync();
          for (size_t c = 0; c < chk.size(); ++c) {
            const double e = hmisc()[2 * c], ymax = hmisc()[2 * c + 1];
            if (e <= kSubspaceTolPrec[opt_.precision] * ymax) {
              chk[c]->fin = true;
              chk[c]->conv = true;
            }
          }
        }
        for (SvdSector* S : act) {
          S->passes = S->fin ? (S->warm ? 2 : 3) : 1;
          S->rel0 = (S->warm || t >= 3) ? 1e-14 : 1e-10;
        }
        orth(act, true);  // Ql
        apply_M(act, true);  // Y = M^T Ql
        orth(act, false);  // Qr; Y keeps Z = M^T Ql
        std::vector<SvdSector*> next;
        for (SvdSector* S : act) {
          S->iters = t + 1;
          if (!S->fin) next.push_back(S);
        }
        act.swap(next);
      }
      // B = Z^T Qr = Ql^T M Qr
      std::vector<GemmDesc> g;
      for (SvdSector* S : sub) {
        GemmDesc d{};
        d.A = S->Y;
        d.B = S->Qr;
        d.C = S->B;
        d.M = S->l;
        d.N = S->l;
        d.K = S->n;
        d.lda = S->l;
        d.ldb = S->l;
        d.ldc = S->l;
        d.ta = 1;
        d.alpha = 1.0;
        g.push_back(d);
      }
      launch_gemms(g);
      for (SvdSector* S : sub)
        HCTM_HIP(hipMemcpyAsync(S->Bj, S->B, sizeof(double) * S->l * S->l, hipMemcpyDeviceToDevice, st_));
    }
    for (SvdSector* S : all)
      if (S->direct) HCTM_HIP(hipMemcpyAsync(S->Bj, S->Mp, sizeof(double) * S->n * S->n, hipMemcpyDeviceToDevice, st_));
    std::vector<SmallProb> jp;
    for (SvdSector* S : all) {
      SmallProb p{};
      p.a = S->Bj;
      p.b = S->Vb;  // right vectors accumulated with the rotations (kt x kt)
      p.m = S->l;
      p.n = S->kt;
      p.lda = S->l;
      p.rel = 1.1e-16 * S->l;
      p.max_sweeps = kJacobiSweeps;
      // the oversampled trailing columns are the least converged ones
      p.pre = S->direct ? 0 : S->l - S->kg;
      p.vlog = S->vlog;
      p.work = S->jwork;
      p.info = S->info + 1;
      p.sv = S->sv;
      p.perm = S->perm;
      jp.push_back(p);
    }
    jacobi(jp, st_);
    SelectArgs a{};
    a.sv0 = sec_[0].sv;
    a.sv1 = sec_[1].sv;
    a.n0 = sec_[0].n > 0 ? sec_[0].trusted : 0;
    a.n1 = sec_[1].n > 0 ? sec_[1].trusted : 0;
    a.chi = chi;
    a.tau = opt_.tau;
    a.out_k = kdev_;
    a.out_s = misc_ + 8;
    a.isq0 = sec_[0].isq;
    a.isq1 = sec_[1].isq;
    a.isv0 = sec_[0].isv;
    a.isv1 = sec_[1].isv;
    select_states(a, st_);
    HCTM_HIP(hipMemcpyAsync(host_k_, kdev_, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
    HCTM_HIP(hipMemcpyAsync(hmisc() + 8, misc_ + 8, 3 * sizeof(double), hipMemcpyDeviceToHost, st_));
    for (int P = 0; P < 2; ++P) {
      HCTM_HIP(hipMemcpyAsync(host_k_ + 2 + 2 * P, sec_[P].info, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
      // the kept values (at most chi <= cc_ per sector) for the record
      const int nc = std::min(sec_[P].n > 0 ? sec_[P].trusted : 0, chi);
      if (nc > cc_) throw Error(1, "truncated_svd: kept count beyond the staging buffer");
      if (nc > 0)
        HCTM_HIP(hipMemcpyAsync(hspec(P), sec_[P].sv, sizeof(double) * nc, hipMemcpyDeviceToHost, st_));
    }
    sync();
    bool redo = false;
    for (int P = 0; P < 2; ++P) {
      SvdSector& S = sec_[P];
      S.k = host_k_[P];
      S.sweeps = host_k_[3 + 2 * P];
      if (S.n == 0) continue;
      if (host_k_[3 + 2 * P] < 0) throw Error(4, "Jacobi SVD did not converge");
      if (!S.direct && S.k >= S.trusted) {
        kg_io[P] = std::min(S.n, S.k + 64);
        redo = true;
      }
    }
    if (!redo) break;
    if (attempt == 3) throw Error(4, "truncated SVD: subspace too small after retries");
  }
  // health of this truncation: a sector whose subspace iteration ran to the
  // cap without passing the residual test, and a chi cut inside a multiplet
  // (the first discarded value within kSplitGap of the last kept one while
  // it is above the cutoff, so that only chi removed it)
  svd_status_ = 0;
  for (int P = 0; P < 2; ++P)
    if (sec_[P].n > 0 && !sec_[P].conv) svd_status_ |= P == 0 ? kRecUnconvEven : kRecUnconvOdd;
  {
    const double smax = hmisc()[8], nxt = hmisc()[9], last = hmisc()[10];
    if (nxt > opt_.tau * smax && last > 0.0 && last / nxt - 1.0 < kSplitGap) svd_status_ |= kRecSplit;
    // chi, not the cutoff, ended the kept states: the spectrum goes on above
    // the cutoff, so a wider subspace block holds signal, not rounding noise
    chi_cut_[key] = nxt > opt_.tau * smax;
  }
  if (svd_status_ & (kRecUnconvEven | kRecUnconvOdd)) ++svd_unconverged_;
  if (svd_status_ & kRecSplit) ++splits_;
  // vectors of the kept states: U from the orthogonalised columns, V from the
  // accumulated rotations (a consistent pair: B V = U S to rounding)
  std::vector<GemmDesc> g;
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    if (S.k == 0) continue;
    gather_cols(S.Bj, S.l, S.perm, S.sv, S.l, S.k, S.Ub, S.k, st_);
    gather_cols(S.Vb, S.kt, S.perm, nullptr, S.kt, S.k, S.B, S.k, st_);
  }
  for (int P = 0; P < 2; ++P) std::swap(sec_[P].B, sec_[P].Vb);  // Vb <- gathered (kt x k)
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    if (S.k == 0) continue;
    if (S.direct) {
      S.W = nullptr;
      continue;
    }
    GemmDesc d{};
    d.A = S.Ql;
    d.B = S.Ub;
    d.C = S.Wbuf;
    d.M = S.n;
    d.N = S.k;
    d.K = S.l;
    d.lda = S.l;
    d.ldb = S.k;
    d.ldc = S.k;
    d.alpha = 1.0;
    g.push_back(d);
    GemmDesc e = d;
    e.A = S.Qr;  // its first kt columns
    e.B = S.Vb;
    e.C = S.Vbuf;
    e.K = S.kt;
    g.push_back(e);
  }
  launch_gemms(g);
  std::vector<CopyJob> save;
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    kg_io[P] = S.k;
    if (S.direct) {
      S.W = S.Ub;
      S.V = S.Vb;
    } else {
      S.W = S.Wbuf;
      S.V = S.Vbuf;
    }
    // keep the kept right vectors of this cut for the next warm start
    WarmV& w = warm_[key * 2 + P];
    w.n = 0;
    w.k = 0;
    if (w.V && !S.direct && S.k > 0 && (long long)S.n * S.k <= warm_cap_) {
      CopyJob j{};
      j.in = S.V;
      j.out = w.V;
      j.r = 1;
      j.dims[0] = S.n * S.k;
      j.istr[0] = 1;
      j.ostr[0] = 1;
      save.push_back(j);
      w.n = S.n;
      w.k = S.k;
    }
  }
  launch_copies(save);
}

// ---------------------------------------------------------------- move ----
void Ctm::mark(int phase) {
  const size_t i = ev_phase_.size();
  if (ev_.size() <= i) {
    hipEvent_t e;
    HCTM_HIP(hipEventCreate(&e));
    ev_.push_back(e);
  }
  HCTM_HIP(hipEventRecord(ev_[i], st_));
  ev_phase_.push_back(phase);
  // with precision 1 (2) the block products of the corners, halves,
  // projectors and renormalisation run in FP32 (BF16x3); the truncated SVD
  // (phase 2), the normalisations and everything outside the moves stay FP64
  low_prec_ = opt_.precision != 0 && (phase == 0 || phase == 1 || phase == 3);
}

void Ctm::move(int r) {
  const int LX = (r % 2 == 0) ? Lx_ : Ly_;
  const int LY = (r % 2 == 0) ? Ly_ : Lx_;
  for (int X = 0; X < LX; ++X) {
    mark(0);
    for (int Y = 0; Y < LY; ++Y) {
      const int ss[4] = {site_of(r, X, Y), site_of(r, X + 1, Y), site_of(r, X + 1, Y + 1), site_of(r, X, Y + 1)};
      for (int i = 0; i < 4; ++i) {
        const int o = (r + i) % 4;
        if (!quad_ok_[ss[i] * 4 + o]) {
          quadrant(ss[i], o);
          quad_ok_[ss[i] * 4 + o] = 1;
        }
      }
    }
    for (int Y = 0; Y < LY; ++Y) {
      mark(1);
      BT& Q1 = quad(site_of(r, X, Y), r);
      BT& Q2 = quad(site_of(r, X + 1, Y), r + 1);
      BT& Q3 = quad(site_of(r, X + 1, Y + 1), r + 2);
      BT& Q4 = quad(site_of(r, X, Y + 1), r + 3);
      const int key = (r * kMaxCell + X) * kMaxCell + Y;
      // Form H_u, H_d and M only when the subspace iteration is expected to
      // be long (the last truncation at this cut needed many iterations) or
      // a sector is small enough to be decomposed directly; otherwise apply
      // M through the corners.  The first truncation at a cut (bonds still
      // growing, blocks and subspace large) applies it too.
      bool implicit = !opt_.form_m && iters_prev_[key] <= kImplicitIters;
      for (int P = 0; P < 2; ++P) {
        const int n = (int)Q2.L.cols[P];
        if (n == 0) continue;
        const int kg = kg_[key][P] > 0 ? std::min(kg_[key][P], n) : std::min(chi_, n);
        const int l = std::min(std::min(n, kg + oversample(kg, key)), l_cap_);
        if (n <= kDirectMax || l >= n) implicit = false;
      }
      impl_q_[0] = &Q1;
      impl_q_[1] = &Q2;
      impl_q_[2] = &Q3;
      impl_q_[3] = &Q4;
      if (implicit) {
        mark(2);
        truncated_svd(nullptr, chi_, key, (uint64_t)records_.size());
        // a retry with a larger subspace may have needed the matrix itself
        implicit = implicit_;
      } else {
        form_M();
        mark(2);
        truncated_svd(&M_, chi_, key, (uint64_t)records_.size());
      }
      iters_prev_[key] = std::max(sec_[0].iters, sec_[1].iters);
      mark(3);

      // projectors of this cut
      const Leg kn{sec_[0].k, sec_[1].k};
      const Leg lW = Q1.L.leg[0];
      BT& Pa = Pa_[Y];
      BT& Pb = Pb_[Y];
      Pa.L = Layout({lW, lq_, kn}, 2);
      Pb.L = Layout({kn, lW, lq_}, 1);
      if (Pa.L.size > proj_cap_ || Pb.L.size > proj_cap_) throw Error(2, "projector capacity");
      std::vector<GemmDesc> g;
      if (implicit) {
        // P_a = Q1 (Q2 V) S^-1/2, P_b = S^-1/2 (W^T Q3) Q4
        for (int P = 0; P < 2; ++P) {
          SvdSector& S = sec_[P];
          if (S.k == 0) continue;
          GemmDesc d{};
          d.A = Q2.p + Q2.L.off[P];
          d.B = S.V;
          d.C = S.C1;
          d.M = (int)Q2.L.rows[P];
          d.N = S.k;
          d.K = (int)Q2.L.cols[P];
          d.lda = (int)Q2.L.ld(P);
          d.ldb = S.k;
          d.ldc = S.k;
          d.alpha = 1.0;
          g.push_back(d);
          GemmDesc e{};
          e.A = S.W;
          e.B = Q3.p + Q3.L.off[P];
          e.C = S.C2;
          e.M = S.k;
          e.N = (int)Q3.L.cols[P];
          e.K = (int)Q3.L.rows[P];
          e.lda = S.k;
          e.ldb = (int)Q3.L.ld(P);
          e.ldc = (int)Q3.L.cols[P];
          e.ta = 1;
          e.alpha = 1.0;
          g.push_back(e);
        }
        launch_gemms(g);
        for (int P = 0; P < 2; ++P) {
          SvdSector& S = sec_[P];
          if (S.k == 0) continue;
          GemmDesc d{};
          d.A = Q1.p + Q1.L.off[P];
          d.B = S.C1;
          d.C = Pa.p + Pa.L.off[P];
          d.M = (int)Q1.L.rows[P];
          d.N = S.k;
          d.K = (int)Q1.L.cols[P];
          d.lda = (int)Q1.L.ld(P);
          d.ldb = S.k;
          d.ldc = S.k;
          d.alpha = 1.0;
          d.cscale = S.isq;
          g.push_back(d);
          GemmDesc e{};
          e.A = S.C2;
          e.B = Q4.p + Q4.L.off[P];
          e.C = Pb.p + Pb.L.off[P];
          e.M = S.k;
          e.N = (int)Q4.L.cols[P];
          e.K = (int)Q4.L.rows[P];
          e.lda = (int)Q3.L.cols[P];
          e.ldb = (int)Q4.L.ld(P);
          e.ldc = (int)Q4.L.cols[P];
          e.alpha = 1.0;
          e.rscale = S.isq;
          g.push_back(e);
        }
      }
      for (int P = 0; P < 2 && !implicit; ++P) {
        SvdSector& S = sec_[P];
        if (S.k == 0) continue;
        const int nW = (int)Hu_.L.rows[P], nE = (int)Hu_.L.cols[P];
        GemmDesc d{};
        d.A = Hu_.p + Hu_.L.off[P];
        d.B = S.V;
        d.C = Pa.p + Pa.L.off[P];
        d.M = nW;
        d.N = S.k;
        d.K = nE;
        d.lda = nE;
        d.ldb = S.k;
        d.ldc = S.k;
        d.alpha = 1.0;
        d.cscale = S.isq;
        g.push_back(d);
        GemmDesc e{};
        e.A = S.W;
        e.B = Hd_.p + Hd_.L.off[P];
        e.C = Pb.p + Pb.L.off[P];
        e.M = S.k;
        e.N = nW;
        e.K = nE;
        e.lda = S.k;
        e.ldb = nW;
        e.ldc = nW;
        e.ta = 1;
        e.alpha = 1.0;
        e.rscale = S.isq;
        g.push_back(e);
      }
      launch_gemms(g);

      // record: the kept spectra were copied to the host at the truncation sync
      MoveRecord rec;
      rec.k_even = opt_.form == 0 ? kn.e : kn.e + kn.o;
      rec.k_odd = opt_.form == 0 ? kn.o : 0;
      rec.frame = r;
      rec.column = X;
      rec.row = Y;
      rec.implicit = implicit ? 1 : 0;
      rec.status = svd_status_;
      for (int P = 0; P < 2; ++P) {
        rec.iters[P] = sec_[P].iters;
        rec.sweeps[P] = sec_[P].sweeps;
      }
      for (int P = 0; P < 2; ++P)
        for (int i = 0; i < sec_[P].k; ++i) rec.spectrum.push_back(hspec(P)[i]);
      std::sort(rec.spectrum.begin(), rec.spectrum.end(), [](double a, double b) { return a > b; });
      const double s0 = rec.spectrum.empty() ? 1.0 : rec.spectrum[0];
      for (double& v : rec.spectrum) v /= s0;
      records_.push_back(std::move(rec));
    }

    // renormalisation: the left environment of column X+1 from column X.  All
    // sources are read before their own site's tensors are overwritten; for
    // LX > 1 sources and targets are different sites.
    for (int Y = 0; Y < LY; ++Y) {
      const int s = site_of(r, X, Y), t = site_of(r, X + 1, Y);
      BT& Pa_up = Pa_[(Y - 1 + LY) % LY];
      BT& Pb_up = Pb_[(Y - 1 + LY) % LY];
      BT& Pa_dn = Pa_[Y];
      BT& Pb_dn = Pb_[Y];
      BT& C1 = env(s, 2 * r);
      BT& T1 = env(s, 2 * r + 1);
      BT& T3 = env(s, 2 * r + 5);
      BT& C4 = env(s, 2 * r + 6);
      BT& T4 = env(s, 2 * r + 7);
      BT X1{Layout(), mid1_, mid_cap_};
      contract(C1, T1, X1);                      // [c | u t]
      BT X2{Layout(), mid2_, mid_cap_};
      permute(X1, X2, {0, 1, 2}, 2);             // [c u | t]
      BT T3s{Layout(), mid1_, mid_cap_};
      permute(T3, T3s, {0, 1, 2}, 2);            // [r u | x]
      BT Z{Layout(), mid3_, mid_cap_};
      contract(T3s, C4, Z);                      // [r u | c]
      BT Zp{Layout(), mid1_, mid_cap_};
      permute(Z, Zp, {0, 2, 1}, 1);              // [r | c u]
      BT T4s{Layout(), mid3_, mid_cap_};
      permute(T4, T4s, {0, 1, 2}, 2);            // [w l | c]
      BT Pas{Layout(), big2_, big_cap_};
      permute(Pa_up, Pas, {0, 1, 2}, 1);         // [c | u k]
      BT Hp = edge_product(T4s, Pas, a_rot(s, r));  // [w e | r k]
      // the old C1, C4, T4 of site s are no longer read
      BT& C1n = env(t, 2 * r);
      BT& C4n = env(t, 2 * r + 6);
      BT& T4n = env(t, 2 * r + 7);
      contract(Pb_up, X2, C1n);                  // [k | t]
      contract(Zp, Pa_dn, C4n);                  // [r | k]
      contract(Pb_dn, Hp, T4n);                  // [k | r k]
      normalise(C1n);
      normalise(C4n);
      normalise(T4n);
      quad_ok_[t * 4 + r] = 0;
      quad_ok_[t * 4 + (r + 3) % 4] = 0;
    }
    mark(-1);
  }
  eps_site_ = -1;
}

// ------------------------------------------------------------ C4v move ----
// One iteration of the C4v-symmetric scheme (Sec. II A) on a 1 x 1 cell: the
// environment is one corner C and one edge T, the same tensor in every corner
// (edge) slot in that slot's own leg order.  The enlarged corner
// Q = C T T a ([w d | t r], rows and columns over the same fused legs) is
// symmetric, so its right singular vectors V (columns of largest singular
// value = |eigenvalue|) span its dominant eigenvectors and serve as the
// projector from both sides: C' = V^T Q V, T' = V^T (T a) V.
void Ctm::move_c4v() {
  const int s = 0, key = 0;
  mark(0);
  quadrant(s, 0);
  BT& Q = quad(s, 0);
  mark(2);
  truncated_svd(&Q, chi_, key, (uint64_t)records_.size());
  iters_prev_[key] = std::max(sec_[0].iters, sec_[1].iters);
  mark(3);
  const Leg kn{sec_[0].k, sec_[1].k};
  BT& Pa = Pa_[0];
  BT& Pb = Pb_[0];
  Pa.L = Layout({Q.L.leg[0], lq_, kn}, 2);  // V as [w d | k]
  Pb.L = Layout({kn, Q.L.leg[0], lq_}, 1);  // V^T as [k | w d]
  if (Pa.L.size > proj_cap_ || Pb.L.size > proj_cap_) throw Error(2, "projector capacity");
  BT& C = env(s, 0);
  C.L = Layout({kn, kn}, 1);
  std::vector<CopyJob> jobs;
  std::vector<GemmDesc> g;
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    if (S.k == 0) continue;
    if (Q.L.rows[P] != Q.L.cols[P] || Pa.L.rows[P] != S.n) throw Error(1, "C4v move: enlarged corner is not square");
    CopyJob a{};  // Pa = V
    a.in = S.V;
    a.out = Pa.p + Pa.L.off[P];
    a.r = 1;
    a.dims[0] = S.n * S.k;
    a.istr[0] = 1;
    a.ostr[0] = 1;
    jobs.push_back(a);
    CopyJob b{};  // Pb = V^T
    b.in = S.V;
    b.out = Pb.p + Pb.L.off[P];
    b.r = 2;
    b.dims[0] = S.k;
    b.dims[1] = S.n;
    b.istr[0] = 1;
    b.istr[1] = S.k;
    b.ostr[0] = S.n;
    b.ostr[1] = 1;
    jobs.push_back(b);
    GemmDesc d{};  // Q V
    d.A = Q.p + Q.L.off[P];
    d.B = S.V;
    d.C = S.C1;
    d.M = S.n;
    d.N = S.k;
    d.K = S.n;
    d.lda = (int)Q.L.ld(P);
    d.ldb = S.k;
    d.ldc = S.k;
    d.alpha = 1.0;
    g.push_back(d);
  }
  launch_copies(jobs);
  launch_gemms(g);
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    if (S.k == 0) continue;
    GemmDesc e{};  // C' = V^T (Q V)
    e.A = S.V;
    e.B = S.C1;
    e.C = C.p + C.L.off[P];
    e.M = S.k;
    e.N = S.k;
    e.K = S.n;
    e.lda = S.k;
    e.ldb = S.k;
    e.ldc = S.k;
    e.ta = 1;
    e.alpha = 1.0;
    g.push_back(e);
  }
  launch_gemms(g);

  // T' = V^T (T a) V, the edge renormalisation of a move with both
  // projectors taken from the one cut
  BT& T4 = env(s, 7);
  BT T4s{Layout(), mid3_, mid_cap_};
  permute(T4, T4s, {0, 1, 2}, 2);        // [w l | c]
  BT Pas{Layout(), big2_, big_cap_};
  permute(Pa, Pas, {0, 1, 2}, 1);        // [c | u k]
  BT Hp = edge_product(T4s, Pas, a_rot(s, 0));  // [w e | r k]
  contract(Pb, Hp, T4);                  // [k | r k]
  normalise(C);
  normalise(T4);
  // the same corner and edge in every slot
  for (int i = 1; i < 4; ++i) {
    BT& Ci = env(s, 2 * i);
    BT& Ti = env(s, 2 * i + 7);
    Ci.L = C.L;
    Ti.L = T4.L;
    for (int w = 0; w < 2; ++w) {
      CopyJob j{};
      j.in = w == 0 ? C.p : T4.p;
      j.out = w == 0 ? Ci.p : Ti.p;
      j.r = 1;
      j.dims[0] = (int)(w == 0 ? C.L.size : T4.L.size);
      j.istr[0] = 1;
      j.ostr[0] = 1;
      jobs.push_back(j);
    }
  }
  launch_copies(jobs);
  for (int o = 0; o < 4; ++o) quad_ok_[s * 4 + o] = 0;
  mark(-1);

  MoveRecord rec;
  rec.k_even = opt_.form == 0 ? kn.e : kn.e + kn.o;
  rec.k_odd = opt_.form == 0 ? kn.o : 0;
  rec.status = svd_status_;
  for (int P = 0; P < 2; ++P) {
    rec.iters[P] = sec_[P].iters;
    rec.sweeps[P] = sec_[P].sweeps;
  }
  for (int P = 0; P < 2; ++P)
    for (int i = 0; i < sec_[P].k; ++i) rec.spectrum.push_back(hspec(P)[i]);
  std::sort(rec.spectrum.begin(), rec.spectrum.end(), [](double a, double b) { return a > b; });
  const double s0 = rec.spectrum.empty() ? 1.0 : rec.spectrum[0];
  for (double& v : rec.spectrum) v /= s0;
  records_.push_back(std::move(rec));
  eps_site_ = -1;
}

// --------------------------------------------------- corner spectra ----
void Ctm::corner_spectra() {
  std::vector<SmallProb> jp;
  std::vector<SpecArgs> sa(ns_);
  // Warm start (blocks up to 256 x 256): the block C is decomposed as
  // X = C V with V the right vectors of its last decomposition (orthogonal,
  // so X has C's singular values), whose columns are then nearly orthogonal
  // and the one-sided Jacobi needs a few sweeps instead of about eight; the
  // rotations R of this decomposition are logged and give the next V = V R.
  // A block whose shape changed starts from V = identity (X = C).
  std::vector<GemmDesc> warm_x, warm_v;
  std::vector<int> fresh, updated;
  double* mat = cmat_;
  for (int st = 0; st < ns_; ++st) {
    SpecArgs& a = sa[st];
    for (int c = 0; c < 4; ++c) {
      BT& C = env(st, 2 * c);
      for (int P = 0; P < 2; ++P) {
        const int m = (int)C.L.rows[P], n = (int)C.L.cols[P];
        const int b = st * 8 + 2 * c + P;
        const long long slot = (long long)b * cc_;
        a.sv[2 * c + P] = csv_ + slot;
        a.nsv[2 * c + P] = (m > 0 && n > 0) ? n : 0;
        const bool keep = cvj_ != nullptr && m > 0 && n > 0;
        const bool warm = keep && cdims_[b][0] == m && cdims_[b][1] == n;
        if (cvj_) cdims_[b] = {m, n};
        if (m == 0 || n == 0) continue;
        const long long boff = (long long)b * cc_ * cc_;
        if (warm) {
          GemmDesc d{};
          d.A = C.p + C.L.off[P];
          d.B = cvec_[ccur_[b]] + boff;
          d.C = mat;
          d.M = m;
          d.N = n;
          d.K = n;
          d.lda = n;
          d.ldb = n;
          d.ldc = n;
          d.alpha = 1.0;
          warm_x.push_back(d);
          GemmDesc e{};
          e.A = cvec_[ccur_[b]] + boff;
          e.B = cvj_ + boff;
          e.C = cvec_[1 - ccur_[b]] + boff;
          e.M = n;
          e.N = n;
          e.K = n;
          e.lda = n;
          e.ldb = n;
          e.ldc = n;
          e.alpha = 1.0;
          warm_v.push_back(e);
          updated.push_back(b);
        } else {
          HCTM_HIP(hipMemcpyAsync(mat, C.p + C.L.off[P], sizeof(double) * m * n, hipMemcpyDeviceToDevice, st_));
          if (keep) fresh.push_back(b);
        }
        SmallProb p{};
        p.a = mat;
        p.m = m;
        p.n = n;
        p.lda = n;
        p.rel = 1.1e-16 * std::max(m, 8);
        p.max_sweeps = keep ? kCornerSweeps : 40;
        p.info = kdev_ + 8;
        p.sv = csv_ + slot;
        p.perm = cperm_ + slot;
        p.work = cwork_ ? cwork_ + (mat - cmat_) : nullptr;
        if (keep) {
          p.b = cvj_ + boff;
          p.vlog = clog_ + (long long)b * clog_n_;
          p.info = cinfo_ + 2 * b;
        }
        jp.push_back(p);
        mat += (long long)cc_ * cc_;
      }
    }
  }
  launch_gemms(warm_x);
  jacobi(jp, st_);
  launch_gemms(warm_v);
  for (int b : updated) ccur_[b] = 1 - ccur_[b];
  for (int b : fresh) {  // V = R
    const int n = cdims_[b][1];
    const long long boff = (long long)b * cc_ * cc_;
    HCTM_HIP(hipMemcpyAsync(cvec_[ccur_[b]] + boff, cvj_ + boff, sizeof(double) * n * n, hipMemcpyDeviceToDevice,
                            st_));
  }
  std::swap(cspec_, cspec_old_);
  for (int st = 0; st < ns_; ++st) {
    SpecArgs& a = sa[st];
    a.spec_new = cspec_ + (long long)st * 4 * cc_;
    a.spec_old = cspec_old_ + (long long)st * 4 * cc_;
    a.len = cc_;
    a.have_old = have_old_spec_ ? 1 : 0;
    a.accumulate = st > 0 ? 1 : 0;
    a.delta = misc_ + 16;
    corner_spectra_delta(a, st_);
  }
  have_old_spec_ = true;
}

void Ctm::step(int n_iter) {
  ev_phase_.clear();
  static const int order[4] = {0, 2, 1, 3};
  for (int it = 0; it < n_iter; ++it) {
    if (opt_.c4v) {
      move_c4v();
    } else if (cplx_) {
      for (int m = 0; m < 4; ++m) cmove(order[m]);
    } else {
      for (int m = 0; m < 4; ++m) move(order[m]);
    }
    mark(4);
    if (cplx_)
      ccorner_spectra();
    else
      corner_spectra();
    mark(-1);
  }
  HCTM_HIP(hipMemcpyAsync(host_d_, misc_ + 16, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  delta_ = host_d_[0];
  flush_gemm_stats();
  // phase times: quadrants, halves, svd, projectors + renormalisation,
  // corner spectra; the time between two marks counts for the phase of the
  // first
  timing.assign(5, 0.0);
  for (size_t i = 0; i + 1 < ev_phase_.size(); ++i) {
    const int ph = ev_phase_[i];
    if (ph < 0) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev_[i], ev_[i + 1]) == hipSuccess) timing[ph] += ms * 1e-3;
  }
}

Leg Ctm::bond(int x, int y, int side) {
  // the first leg of the edge tensor on that side: T1's left, T2's up, T3's
  // right, T4's down leg
  return env(site(x, y), 2 * (side % 4) + 1).L.leg[0];
}

// ---------------------------------------------------------- observables ----
void Ctm::compute_epsilon_rot(int st) {
  if (eps_site_ == st) return;
  BT& C1 = env(st, 0);
  BT& T1 = env(st, 1);
  BT& C2 = env(st, 2);
  BT& T2 = env(st, 3);
  BT& C3 = env(st, 4);
  BT& T3 = env(st, 5);
  BT& C4 = env(st, 6);
  BT& T4 = env(st, 7);
  BT TA{Layout(), mid1_, mid_cap_};
  contract(C1, T1, TA);                    // [a | U b]
  BT TAs{Layout(), mid2_, mid_cap_};
  permute(TA, TAs, {0, 1, 2}, 2);          // [a U | b]
  BT TOP{Layout(), mid1_, mid_cap_};
  contract(TAs, C2, TOP);                  // [a U | c]
  BT TOPp{Layout(), mid2_, mid_cap_};
  permute(TOP, TOPp, {1, 2, 0}, 2);        // [U c | a]
  BT T4p{Layout(), mid3_, mid_cap_};
  permute(T4, T4p, {2, 0, 1}, 1);          // [a | c' L]
  BT LT{Layout(), big1_, big_cap_};
  contract(TOPp, T4p, LT);                 // [U c | c' L]
  BT LTp{Layout(), big2_, big_cap_};
  permute(LT, LTp, {0, 3, 1, 2}, 2);       // [U L | c c']
  BT S1{Layout(), mid1_, mid_cap_};
  contract(C3, T3, S1);                    // [e | Dn x]
  BT S1s{Layout(), mid2_, mid_cap_};
  permute(S1, S1s, {0, 1, 2}, 2);          // [e Dn | x]
  BT BOT{Layout(), mid1_, mid_cap_};
  contract(S1s, C4, BOT);                  // [e Dn | c']
  BT BOTs{Layout(), mid2_, mid_cap_};
  permute(BOT, BOTs, {0, 1, 2}, 1);        // [e | Dn c']
  BT T2s{Layout(), mid3_, mid_cap_};
  permute(T2, T2s, {0, 1, 2}, 2);          // [c R | e]
  BT RB0{Layout(), big1_, big_cap_};
  contract(T2s, BOTs, RB0);                // [c R | Dn c']
  BT RB{Layout(), quad_[0].p, quad_[0].capacity};  // quadrant memory as scratch
  permute(RB0, RB, {0, 3, 2, 1}, 2);       // [c c' | Dn R]
  quad_ok_[0] = 0;
  contract(LTp, RB, eps_);                 // [U L | Dn R]
  eps_site_ = st;
}

BT Ctm::pack_impurity(int site, int s, int sp, int kind, int frame) {
  DLArgs g{};
  g.A = A_ + (long long)site * d_ * D_ * D_ * D_ * D_;
  g.out = plain_tmp_;
  g.tab_idx = tab_idx_;
  g.tab_c = tab_c_;
  g.d = d_;
  g.D = D_;
  if (kind == 0) {
    g.npairs = 1;
    g.ket[0] = s;
    g.bra[0] = sp;
    g.w[0] = 1.0;
  } else {
    g.npairs = 2;
    g.ket[0] = s;
    g.bra[0] = sp;
    g.w[0] = 0.5;
    g.ket[1] = sp;
    g.bra[1] = s;
    g.w[1] = kind == 1 ? 0.5 : -0.5;
  }
  double_layer_basis(g, st_);
  BT t{Layout({lq_, lq_, lq_, lq_}, 2, kind == 2 ? 1 : 0), plain_tmp2_, (long long)q_ * q_ * q_ * q_};
  const long long q = q_;
  const long long s0[4] = {q * q * q, q * q, q, 1};
  long long st[4];
  for (int j = 0; j < 4; ++j) st[j] = s0[(j - frame + 4) % 4];
  std::vector<CopyJob> jobs;
  plan_pack(plain_tmp_, st, t, true, jobs);
  launch_copies(jobs);
  return t;
}

// left half of the two-site environment in a frame (environment of site st),
// closed with an impurity
BT Ctm::left_half(int f, int st, const BT& imp) {
  BT& C1 = env(st, 2 * f);
  BT& T1 = env(st, 2 * f + 1);
  BT& T3 = env(st, 2 * f + 5);
  BT& C4 = env(st, 2 * f + 6);
  BT& T4 = env(st, 2 * f + 7);
  BT TL{Layout(), mid1_, mid_cap_};
  contract(C1, T1, TL);                    // [a | U y]
  BT T4s{Layout(), mid2_, mid_cap_};
  permute(T4, T4s, {0, 1, 2}, 2);          // [c' L | a]
  BT W1{Layout(), big1_, big_cap_};
  contract(T4s, TL, W1);                   // [c' L | U y]
  BT W1p{Layout(), big2_, big_cap_};
  permute(W1, W1p, {0, 3, 2, 1}, 2);       // [c' y | U L]
  BT V1{Layout(), big1_, big_cap_};
  contract(W1p, imp, V1);                  // [c' y | Dn R]
  BT V1p{Layout(), big2_, big_cap_};
  permute(V1, V1p, {1, 3, 0, 2}, 2);       // [y R | c' Dn]
  BT T3s{Layout(), mid1_, mid_cap_};
  permute(T3, T3s, {0, 1, 2}, 2);          // [z Dn | x]
  BT S{Layout(), mid2_, mid_cap_};
  contract(T3s, C4, S);                    // [z Dn | c']
  BT BL{Layout(), mid3_, mid_cap_};
  permute(S, BL, {2, 1, 0}, 2);            // [c' Dn | z]
  BT out{Layout(), nullptr, halves_cap_};
  out.p = halves_ + (long long)halves_used_ * halves_cap_;
  ++halves_used_;
  contract(V1p, BL, out);                  // [y R | z]
  return out;
}

BT Ctm::right_half(int f, int st, const BT& imp) {
  BT& T1 = env(st, 2 * f + 1);
  BT& C2 = env(st, 2 * f + 2);
  BT& T2 = env(st, 2 * f + 3);
  BT& C3 = env(st, 2 * f + 4);
  BT& T3 = env(st, 2 * f + 5);
  BT T1s{Layout(), mid1_, mid_cap_};
  permute(T1, T1s, {0, 1, 2}, 2);          // [y U | x]
  BT TR{Layout(), mid2_, mid_cap_};
  contract(T1s, C2, TR);                   // [y U | c]
  BT W2{Layout(), big1_, big_cap_};
  contract(TR, T2, W2);                    // [y U | R c'']
  BT W2p{Layout(), big2_, big_cap_};
  permute(W2, W2p, {0, 3, 1, 2}, 2);       // [y c'' | U R]
  BT impp{Layout(), quad_[1].p, quad_[1].capacity};  // quadrant memory as scratch
  quad_ok_[1] = 0;
  permute(imp, impp, {0, 3, 1, 2}, 2);     // [u r | l d]
  BT V2{Layout(), big1_, big_cap_};
  contract(W2p, impp, V2);                 // [y c'' | L Dn]
  BT V2p{Layout(), big2_, big_cap_};
  permute(V2, V2p, {0, 2, 1, 3}, 2);       // [y L | c'' Dn]
  BT S2{Layout(), mid1_, mid_cap_};
  contract(C3, T3, S2);                    // [c'' | Dn z]
  BT S2s{Layout(), mid2_, mid_cap_};
  permute(S2, S2s, {0, 1, 2}, 2);          // [c'' Dn | z]
  BT out{Layout(), nullptr, halves_cap_};
  out.p = halves_ + (long long)halves_used_ * halves_cap_;
  ++halves_used_;
  contract(V2p, S2s, out);                 // [y L | z]
  return out;
}

void Ctm::rdm1(int x, int y, double* rho) {
  const int st = site(x, y);
  compute_epsilon_rot(st);
  const int d = d_;
  int nd = 0;
  for (int s = 0; s < d; ++s)
    for (int t = (opt_.form == 0 ? s : 0); t < d; ++t) {
      BT imp = pack_impurity(st, s, t, opt_.form == 0 ? 1 : 0, 0);
      if (imp.L.size != eps_.L.size) throw Error(1, "rdm1: layout mismatch");
      dots({DotJob{eps_.p, imp.p, eps_.L.size, dots_ + nd}}, dpart_, st_);
      ++nd;
    }
  assemble_rho(dots_, d, opt_.form == 0 ? 1 : 0, rho_, st_);
  HCTM_HIP(hipMemcpyAsync(rho, rho_, sizeof(double) * d * d, hipMemcpyDeviceToHost, st_));
  sync();
}

// rho2 of the pair (x, y)-(x+1, y) (dir 0) or (x, y)-(x, y+1) (dir 1): the
// left half of the first site's environment and the right half of the
// second's, in the frame where the pair is horizontal, each closed with the
// impurities of its site; in the Z2 form only sym x sym and anti x anti pairs
// couple (the environment is even).  Result (d^4) at dst on the device.
void Ctm::rdm2_dev(int x, int y, int dir, double* dst) {
  const int f = dir == 0 ? 0 : 1;
  const int s1 = site(x, y), s2 = dir == 0 ? site(x + 1, y) : site(x, y + 1);
  const int d = d_;
  halves_used_ = 0;
  std::vector<DotJob> jobs;
  int mode;
  if (opt_.form != 0) {
    std::vector<BT> L, R;
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t) L.push_back(left_half(f, s1, pack_impurity(s1, s, t, 0, f)));
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t) R.push_back(right_half(f, s2, pack_impurity(s2, s, t, 0, f)));
    int k = 0;
    for (int a = 0; a < d * d; ++a)
      for (int b = 0; b < d * d; ++b) {
        if (L[a].L.size != R[b].L.size) throw Error(1, "rdm2: layout mismatch");
        jobs.push_back(DotJob{L[a].p, R[b].p, L[a].L.size, dots_ + k++});
      }
    mode = 2;
  } else {
    std::vector<BT> Ls, La, Rs, Ra;
    for (int s = 0; s < d; ++s)
      for (int t = s; t < d; ++t) Ls.push_back(left_half(f, s1, pack_impurity(s1, s, t, 1, f)));
    for (int s = 0; s < d; ++s)
      for (int t = s + 1; t < d; ++t) La.push_back(left_half(f, s1, pack_impurity(s1, s, t, 2, f)));
    for (int s = 0; s < d; ++s)
      for (int t = s; t < d; ++t) Rs.push_back(right_half(f, s2, pack_impurity(s2, s, t, 1, f)));
    for (int s = 0; s < d; ++s)
      for (int t = s + 1; t < d; ++t) Ra.push_back(right_half(f, s2, pack_impurity(s2, s, t, 2, f)));
    int k = 0;
    for (size_t a = 0; a < Ls.size(); ++a)
      for (size_t b = 0; b < Rs.size(); ++b) {
        if (Ls[a].L.size != Rs[b].L.size) throw Error(1, "rdm2: layout mismatch");
        jobs.push_back(DotJob{Ls[a].p, Rs[b].p, Ls[a].L.size, dots_ + k++});
      }
    for (size_t a = 0; a < La.size(); ++a)
      for (size_t b = 0; b < Ra.size(); ++b) {
        if (La[a].L.size != Ra[b].L.size) throw Error(1, "rdm2: layout mismatch");
        jobs.push_back(DotJob{La[a].p, Ra[b].p, La[a].L.size, dots_ + k++});
      }
    mode = 3;
  }
  dots(jobs, dpart_, st_);
  assemble_rho(dots_, d, mode, dst, st_);
}

void Ctm::rdm2(int x, int y, int dir, double* rho) {
  rdm2_dev(x, y, dir, rho_);
  HCTM_HIP(hipMemcpyAsync(rho, rho_, sizeof(double) * d_ * d_ * d_ * d_, hipMemcpyDeviceToHost, st_));
  sync();
}

double Ctm::energy(const double* h_host) {
  // E = (1/ns) sum over sites of Tr(rho_h h) + Tr(rho_v h): all 2 ns RDMs on
  // the device, traced against h / ns
  const int n = d_ * d_;
  const long long d4 = (long long)n * n;
  for (int st = 0; st < ns_; ++st)
    for (int dir = 0; dir < 2; ++dir) rdm2_dev(st % Lx_, st / Lx_, dir, rho_ + (2 * st + dir) * d4);
  std::vector<double> hs(h_host, h_host + d4);
  for (double& v : hs) v /= ns_;
  HCTM_HIP(hipMemcpyAsync(hdev_, hs.data(), sizeof(double) * d4, hipMemcpyHostToDevice, st_));
  trace_products(rho_, 2 * ns_, hdev_, n, misc_ + 20, st_);
  HCTM_HIP(hipMemcpyAsync(host_d_, misc_ + 20, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  return host_d_[0];
}

// eps of site (x, y) in the plain basis (unnormalised) into plain_tmp2_;
// <eps~, a~> into misc_[24]
void Ctm::epsilon_plain(int x, int y, double* eps_host) {
  const int sid = site(x, y);
  compute_epsilon_rot(sid);
  const long long q4 = (long long)q_ * q_ * q_ * q_;
  dots({DotJob{eps_.p, a_rot(sid, 0).p, eps_.L.size, misc_ + 24}}, dpart_, st_);
  fill(plain_tmp_, 0.0, (size_t)q4, st_);
  const long long q = q_;
  const long long str[4] = {q * q * q, q * q, q, 1};
  std::vector<CopyJob> jobs;
  plan_pack(plain_tmp_, str, eps_, false, jobs);
  launch_copies(jobs);
  basis4(plain_tmp_, plain_tmp2_, q_, tabT_idx_, tabT_c_, st_);
  if (eps_host) {
    scale_inv(plain_tmp2_, (size_t)q4, misc_ + 24, st_);
    HCTM_HIP(hipMemcpyAsync(eps_host, plain_tmp2_, sizeof(double) * q4, hipMemcpyDeviceToHost, st_));
    sync();
  }
}

double Ctm::s_err() {
  for (int st = 0; st < ns_; ++st) {
    epsilon_plain(st % Lx_, st / Lx_, nullptr);
    swap_asym(plain_tmp2_, D_, part_, misc_ + 26 + st, st_);
  }
  HCTM_HIP(hipMemcpyAsync(host_d_, misc_ + 26, sizeof(double) * ns_, hipMemcpyDeviceToHost, st_));
  sync();
  double m = 0.0;
  for (int st = 0; st < ns_; ++st) m = std::max(m, host_d_[st]);
  return m;
}

void Ctm::top_bottom(BT& top, BT& bot) {
  BT TA{Layout(), mid1_, mid_cap_};
  contract(env_[0], env_[1], TA);          // [a | U b]
  BT TAs{Layout(), mid2_, mid_cap_};
  permute(TA, TAs, {0, 1, 2}, 2);          // [a U | b]
  contract(TAs, env_[2], top);             // [a U | c]
  BT S1{Layout(), mid1_, mid_cap_};
  contract(env_[4], env_[5], S1);          // [e | Dn x]
  BT S1s{Layout(), mid2_, mid_cap_};
  permute(S1, S1s, {0, 1, 2}, 2);          // [e Dn | x]
  BT B0{Layout(), mid1_, mid_cap_};
  contract(S1s, env_[6], B0);              // [e Dn | c']
  permute(B0, bot, {2, 1, 0}, 2);          // [c' Dn | e]
}

double Ctm::log_kappa() {
  if (ns_ != 1) throw Error(1, "log_kappa: defined for the 1x1 cell only");
  compute_epsilon_rot(0);
  // Z11 = <eps~, a~>
  dots({DotJob{eps_.p, a_rot(0, 0).p, eps_.L.size, misc_ + 40}}, dpart_, st_);
  // Z00 = Tr(C1 C2 C3 C4)
  {
    BT c12{Layout(), big1_, big_cap_}, c123{Layout(), big2_, big_cap_}, c1234{Layout(), big1_, big_cap_};
    contract(env_[0], env_[2], c12);
    contract(c12, env_[4], c123);
    contract(c123, env_[6], c1234);
    const double* p[2];
    int n[2], ld[2], nb = 0;
    for (int P = 0; P < 2; ++P) {
      if (c1234.L.rows[P] == 0) continue;
      p[nb] = c1234.p + c1234.L.off[P];
      n[nb] = (int)c1234.L.rows[P];
      ld[nb] = (int)c1234.L.ld(P);
      ++nb;
    }
    trace_blocks(p, n, ld, nb, misc_ + 41, st_);
  }
  // Z10 = <TOP, BOT>, T1 joined directly to T3
  {
    BT top{Layout(), big1_, big_cap_}, bot{Layout(), big2_, big_cap_};
    top_bottom(top, bot);
    if (top.L.size != bot.L.size) throw Error(1, "log_kappa: layout mismatch");
    dots({DotJob{top.p, bot.p, top.L.size, misc_ + 42}}, dpart_, st_);
  }
  // Z01: C1 C2 T2 C3 C4 with T4 joined directly to T2
  {
    BT u1{Layout(), mid1_, mid_cap_}, u2{Layout(), mid2_, mid_cap_}, u2s{Layout(), mid3_, mid_cap_};
    contract(env_[0], env_[2], u1);        // [a | b]
    contract(u1, env_[3], u2);             // [a | R e]
    permute(u2, u2s, {0, 1, 2}, 2);        // [a R | e]
    BT u3{Layout(), mid1_, mid_cap_}, u4{Layout(), mid2_, mid_cap_}, t4{Layout(), mid3_, mid_cap_};
    contract(u2s, env_[4], u3);            // [a R | y]
    contract(u3, env_[6], u4);             // [a R | c]
    permute(env_[7], t4, {2, 1, 0}, 2);    // T4[c | R a] -> [a R | c]
    if (u4.L.size != t4.L.size) throw Error(1, "log_kappa: layout mismatch");
    dots({DotJob{u4.p, t4.p, u4.L.size, misc_ + 43}}, dpart_, st_);
  }
  log_ratio(misc_ + 40, misc_ + 44, st_);
  HCTM_HIP(hipMemcpyAsync(host_d_, misc_ + 44, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  return host_d_[0];
}

}  // namespace hctm
