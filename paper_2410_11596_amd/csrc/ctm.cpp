// Directional CTMRG on a 1x1 unit cell in the eigenbasis of the bra-ket swap.
//
// Frames.  The eight environment tensors are kept in slots
//   0 C1[d,r]  1 T1[l,d,r]  2 C2[l,d]  3 T2[u,l,d]  4 C3[u,l]  5 T3[r,u,l]
//   6 C4[r,u]  7 T4[d,r,u]
// (legs counter-clockwise).  Turning the lattice by a quarter turn (old right
// leg becomes the up leg) maps slot i to slot i-2, so a move in any direction
// is the left move of a rotated frame r: its C1 is slot 2r, its T1 slot 2r+1,
// and the double layer is a_r with legs (j - r) mod 4 of a.  Moves are run in
// the order left (r=0), right (2), top (1), bottom (3).
//
// One left move (frame r), all products being block-diagonal GEMMs per parity
// sector:
//   quadrants  Q_j[W|N] = C1 T1 T4 a of frame j, for j = r..r+3 (a quadrant
//              is recomputed only after one of its tensors changed);
//   halves     H_u = Q1 Q2, H_d = Q3 Q4, M = H_d H_u;
//   SVD        per sector, truncated to chi over the merged spectrum;
//   projectors P_a = H_u V S^-1/2, P_b = S^-1/2 W^T H_d;
//   renormalise C1' = P_b (C1 T1), T4' = P_b (T4 a P_a), C4' = (T3 C4) P_a,
//              each divided by its Frobenius norm.
// Tensors are stored as fused-sector block-diagonal matrices (blocks.hpp).
#include "ctm.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace hctm {

namespace {
constexpr int kDirectMax = 160;  // sectors up to this size are decomposed directly
constexpr int kJacobiSweeps = 40;
}

// ------------------------------------------------------------- memory ----
Ctm::Ctm(CountTag, int d, int D, int chi) : d_(d), D_(D), chi_(chi) {
  q_ = D * D;
  cc_ = std::max(chi, q_);
}

size_t Ctm::workspace_bytes(int d, int D, int chi, const Options& o) {
  (void)o;
  Ctm c(CountTag{}, d, D, chi);
  c.plan_memory(true);
  return c.ar_.used + 256;
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
  A_ = ar_.take((size_t)d_ * D_ * D_ * D_ * D_);
  b_ = ar_.take((size_t)q);
  a_plain_ = ar_.take((size_t)q4);
  plain_tmp_ = ar_.take((size_t)q4);
  plain_tmp2_ = ar_.take((size_t)q4);
  for (int r = 0; r < 4; ++r) {
    a_rot_[r].p = ar_.take((size_t)q4);
    a_rot_[r].capacity = q4;
  }
  for (int i = 0; i < 8; ++i) {
    const long long n = (i % 2 == 0) ? cc * cc : cc * cc * q;
    env_[i].p = ar_.take((size_t)n);
    env_[i].capacity = n;
  }
  for (int j = 0; j < 4; ++j) {
    quad_[j].p = ar_.take((size_t)(ncap * ncap));
    quad_[j].capacity = ncap * ncap;
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
  Pa_.p = ar_.take((size_t)proj_cap_);
  Pa_.capacity = proj_cap_;
  Pb_.p = ar_.take((size_t)proj_cap_);
  Pb_.capacity = proj_cap_;
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    S.Qr = ar_.take((size_t)(ncap * lcap));
    S.Ql = ar_.take((size_t)(ncap * lcap));
    S.Y = ar_.take((size_t)(ncap * lcap));
    S.Tm = ar_.take((size_t)(ncap * lcap));
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
    S.vlog = ar_.take(jacobi_log_doubles(160, kJacobiSweeps));
  }
  misc_ = ar_.take(64);
  kdev_ = ti(16);
  part_ = ar_.take(2048);
  cspec_ = ar_.take((size_t)(4 * cc));
  cspec_old_ = ar_.take((size_t)(4 * cc));
  csv_ = ar_.take((size_t)(8 * cc));
  cperm_ = ti(8 * cc);
  cmat_ = ar_.take((size_t)(8 * cc * cc));
  eps_.p = ar_.take((size_t)q4);
  eps_.capacity = q4;
  halves_cap_ = cc * cc * q;
  halves_max_ = 2 * d_ * d_;
  halves_ = ar_.take((size_t)(halves_max_ * halves_cap_));
  const long long d4 = (long long)d_ * d_ * d_ * d_;
  dots_ = ar_.take((size_t)(2 * d4 + 16));
  dpart_ = ar_.take((size_t)(64 * kMaxDots));
  rho_ = ar_.take((size_t)(2 * d4 + 16));
  hdev_ = ar_.take((size_t)(d4 + 16));
  gemm_scratch_cap_ = std::max<long long>(1 << 20, 24LL * lcap * lcap);
  gemm_scratch_ = ar_.take((size_t)gemm_scratch_cap_);
}

// ------------------------------------------------------------- set-up ----
Ctm::Ctm(const double* A_host, int d, int D, int chi, const Options& o, hipStream_t stream, void* workspace,
         size_t ws_bytes)
    : d_(d), D_(D), chi_(chi), opt_(o) {
  q_ = D * D;
  cc_ = std::max(chi, q_);
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
  HCTM_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_d_), 4096 * sizeof(double), hipHostMallocDefault));
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
  if (!opt_.profile) {
    gemm(g, st_, gemm_scratch_, gemm_scratch_cap_);
    g.clear();
    return;
  }
  double f = 0.0;
  for (const GemmDesc& d : g)
    if (d.M > 0 && d.N > 0 && d.K > 0) f += 2.0 * d.M * d.N * d.K;
  while (gev_.size() < gev_used_ + 2) {
    hipEvent_t e;
    HCTM_HIP(hipEventCreate(&e));
    gev_.push_back(e);
  }
  HCTM_HIP(hipEventRecord(gev_[gev_used_], st_));
  gemm(g, st_, gemm_scratch_, gemm_scratch_cap_);
  HCTM_HIP(hipEventRecord(gev_[gev_used_ + 1], st_));
  gflops_.push_back(f);
  gev_used_ += 2;
  g.clear();
  if (gev_used_ >= 4096) flush_gemm_stats();
}

void Ctm::flush_gemm_stats() {
  if (gev_used_ == 0) return;
  sync();
  for (size_t i = 0; i < gev_used_ / 2; ++i) {
    float ms = 0.f;
    HCTM_HIP(hipEventElapsedTime(&ms, gev_[2 * i], gev_[2 * i + 1]));
    gemm_stats.seconds += ms * 1e-3;
    gemm_stats.flops += gflops_[i];
    gemm_stats.launches += 1;
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

void Ctm::normalise(BT& t) {
  norm2(t.p, (size_t)t.L.size, misc_, part_, st_);
  scale_inv(t.p, (size_t)t.L.size, misc_, st_);
}

void Ctm::setup(const double* A_host) {
  const int q = q_, D = D_;
  // basis U (rows) and U^T, at most two entries per row
  std::vector<int> ti(2 * q, -1), tti(2 * q, -1);
  std::vector<double> tc(2 * q, 0.0), ttc(2 * q, 0.0);
  if (opt_.form == 0) {
    const double r2 = 1.0 / std::sqrt(2.0);
    int row = 0;
    for (int k = 0; k < D; ++k) {
      ti[2 * row] = k * D + k;
      tc[2 * row] = 1.0;
      ++row;
    }
    for (int sgn = 0; sgn < 2; ++sgn)
      for (int k = 0; k < D; ++k)
        for (int l = k + 1; l < D; ++l) {
          ti[2 * row] = k * D + l;
          tc[2 * row] = r2;
          ti[2 * row + 1] = l * D + k;
          tc[2 * row + 1] = sgn ? -r2 : r2;
          ++row;
        }
  } else {
    for (int a = 0; a < q; ++a) {
      ti[2 * a] = a;
      tc[2 * a] = 1.0;
    }
  }
  std::vector<int> cnt(q, 0);
  for (int a = 0; a < q; ++a)
    for (int w = 0; w < 2; ++w) {
      const int K = ti[2 * a + w];
      if (K < 0) continue;
      tti[2 * K + cnt[K]] = a;
      ttc[2 * K + cnt[K]] = tc[2 * a + w];
      ++cnt[K];
    }
  HCTM_HIP(hipMemcpy(tab_idx_, ti.data(), sizeof(int) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tab_c_, tc.data(), sizeof(double) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tabT_idx_, tti.data(), sizeof(int) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tabT_c_, ttc.data(), sizeof(double) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(A_, A_host, sizeof(double) * d_ * D * D * D * D, hipMemcpyHostToDevice));
  std::vector<double> b(q, 0.0);
  if (opt_.boundary.empty()) {
    for (int k = 0; k < D; ++k) b[k * D + k] = 1.0;
  } else {
    b = opt_.boundary;
  }
  HCTM_HIP(hipMemcpy(b_, b.data(), sizeof(double) * q, hipMemcpyHostToDevice));

  // double layer in the rotated basis, a[U,L,Dn,R] = sum_s A[s] (x) A[s]
  DLArgs g;
  g.A = A_;
  g.out = a_plain_;
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
  const long long s0[4] = {(long long)q * q * q, (long long)q * q, (long long)q, 1};
  std::vector<CopyJob> jobs;
  for (int r = 0; r < 4; ++r) {
    a_rot_[r].L = Layout({lq_, lq_, lq_, lq_}, 2);
    long long st[4];
    for (int j = 0; j < 4; ++j) st[j] = s0[(j - r + 4) % 4];
    plan_pack(a_plain_, st, a_rot_[r], true, jobs);
  }
  launch_copies(jobs);

  // traced boundary: C1, T1 of every frame
  for (int r = 0; r < 4; ++r) {
    init_env(a_plain_, q, r, b_, tab_idx_, tab_c_, plain_tmp_, plain_tmp2_, st_);
    BT& C = env_[2 * r];
    BT& T = env_[2 * r + 1];
    C.L = Layout({lq_, lq_}, 1);
    T.L = Layout({lq_, lq_, lq_}, 1);
    const long long sc[2] = {q, 1};
    const long long stt[3] = {(long long)q * q, q, 1};
    plan_pack(plain_tmp_, sc, C, true, jobs);    // init_env wrote C to plain_tmp_
    plan_pack(plain_tmp2_, stt, T, true, jobs);   // and T to plain_tmp2_
    launch_copies(jobs);
  }
  for (int i = 0; i < 8; ++i) normalise(env_[i]);
  for (int s = 0; s < 4; ++s) side_[s] = lq_;
  sync();
}

// ------------------------------------------------------------ quadrant ----
// quad_[j] = C1 T1 T4 a of frame j as a matrix [w d | t r].
void Ctm::quadrant(int j) {
  BT& C = env_[(2 * j) % 8];
  BT& T1 = env_[(2 * j + 1) % 8];
  BT& T4 = env_[(2 * j + 7) % 8];
  BT X{Layout(), mid1_, mid_cap_};
  contract(C, T1, X);                                    // [c | u t]
  BT T4s{Layout(), mid2_, mid_cap_};
  permute(T4, T4s, {0, 1, 2}, 2);                        // [w l | c]
  BT Y{Layout(), big1_, big_cap_};
  contract(T4s, X, Y);                                   // [w l | u t]
  BT Yp{Layout(), big2_, big_cap_};
  permute(Y, Yp, {0, 3, 2, 1}, 2);                       // [w t | u l]
  BT Qp{Layout(), big1_, big_cap_};
  contract(Yp, a_rot_[j], Qp);                           // [w t | d r]
  permute(Qp, quad_[j], {0, 2, 1, 3}, 2);                // [w d | t r]
}

// ---------------------------------------------------------------- SVD ----
void Ctm::orth(std::vector<SvdSector*>& ss, bool ql, int passes) {
  // src = S.Y, dst = Ql or Qr, scratch Tm; 2 or 3 CholeskyQR passes, the
  // result always ends in dst (pass 0: src->dst, 1: dst->Tm, 2: Tm->dst;
  // with 2 passes the last product writes dst from Tm's predecessor).
  if (passes < 1 || passes > 3) throw Error(1, "orth: passes must be 1, 2 or 3");
  for (int pass = 0; pass < passes; ++pass) {
    std::vector<GemmDesc> g;
    for (SvdSector* S : ss) {
      double* dstq = ql ? S->Ql : S->Qr;
      const double* src = pass == 0 ? S->Y : (((passes - pass) % 2 == 0) ? dstq : S->Tm);
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
    for (SvdSector* S : ss) {
      SmallProb p{};
      p.a = S->G;
      p.b = S->Ri;
      p.m = p.n = S->l;
      p.lda = p.ldb = S->l;
      // unit-diagonal (column-scaled) Gram; a small shift in the first pass
      // keeps the factorisation defined while the columns are nearly parallel.
      // Inner iterations need only a well-conditioned basis (one pass); the
      // last one is orthonormalised to rounding (three passes).
      p.rel = pass == 0 ? 1e-10 : 0.0;
      p.flags = 1;
      p.sv = S->isv;
      p.info = S->info;
      sp.push_back(p);
    }
    chol_inv(sp, st_);
    for (SvdSector* S : ss) {
      // pass p writes dst if (passes - 1 - p) is even, else the scratch Tm
      double* dstq = ql ? S->Ql : S->Qr;
      const double* src = pass == 0 ? S->Y : (((passes - pass) % 2 == 0) ? dstq : S->Tm);
      double* dst = ((passes - 1 - pass) % 2 == 0) ? dstq : S->Tm;
      GemmDesc d{};
      d.A = src;
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

void Ctm::truncated_svd(BT& M, int chi) {
  for (int attempt = 0; attempt < 4; ++attempt) {
    std::vector<SvdSector*> sub, all;
    for (int P = 0; P < 2; ++P) {
      SvdSector& S = sec_[P];
      S.n = (int)M.L.rows[P];
      S.Mp = M.p + M.L.off[P];
      S.k = 0;
      if (S.n == 0) {
        S.trusted = 0;
        continue;
      }
      int kg = S.kg > 0 ? S.kg : chi;
      kg = std::min(kg, S.n);
      const int p = std::max(32, kg / 2);
      S.l = std::min<int>(std::min(S.n, kg + p), l_cap_);
      S.direct = S.n <= kDirectMax || S.l >= S.n;
      if (S.direct && S.n > l_cap_) throw Error(1, "truncated_svd: sector too large for a direct decomposition");
      if (S.direct) S.l = S.n;
      S.trusted = S.direct ? S.n : S.l - p / 2;
      all.push_back(&S);
      if (!S.direct) sub.push_back(&S);
    }
    // subspace iteration (both sectors batched)
    if (!sub.empty()) {
      for (SvdSector* S : sub) {
        const uint64_t seed = opt_.seed * 0x9E3779B97F4A7C15ull + (move_count_ << 4) + (S == &sec_[1] ? 1 : 0) +
                              ((uint64_t)attempt << 2);
        random_fill(S->Y, (size_t)S->n * S->l, seed, st_);
      }
      orth(sub, false, 3);  // Qr
      const int T = std::max(1, opt_.svd_iters);
      for (int t = 0; t < T; ++t) {
        const bool last = t == T - 1;
        std::vector<GemmDesc> g;
        for (SvdSector* S : sub) {
          GemmDesc d{};
          d.A = S->Mp;
          d.B = S->Qr;
          d.C = S->Y;
          d.M = S->n;
          d.N = S->l;
          d.K = S->n;
          d.lda = S->n;
          d.ldb = S->l;
          d.ldc = S->l;
          d.alpha = 1.0;
          g.push_back(d);
        }
        launch_gemms(g);
        orth(sub, true, last ? 3 : 1);  // Ql
        for (SvdSector* S : sub) {
          GemmDesc d{};
          d.A = S->Mp;
          d.B = S->Ql;
          d.C = S->Y;
          d.M = S->n;
          d.N = S->l;
          d.K = S->n;
          d.lda = S->n;
          d.ldb = S->l;
          d.ldc = S->l;
          d.ta = 1;
          d.alpha = 1.0;
          g.push_back(d);
        }
        launch_gemms(g);
        orth(sub, false, last ? 3 : 1);  // Qr; Y keeps Z = M^T Ql
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
      p.b = S->Vb;  // right vectors accumulated with the rotations
      p.m = p.n = S->l;
      p.lda = S->l;
      p.rel = 1.1e-16 * S->l;
      p.max_sweeps = kJacobiSweeps;
      p.vlog = S->vlog;
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
    for (int P = 0; P < 2; ++P) {
      HCTM_HIP(hipMemcpyAsync(host_k_ + 2 + 2 * P, sec_[P].info, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
      const int nc = std::min(sec_[P].n > 0 ? sec_[P].trusted : 0, std::min(chi, 2048));
      if (nc > 0)
        HCTM_HIP(hipMemcpyAsync(host_d_ + 2048 * P, sec_[P].sv, sizeof(double) * nc, hipMemcpyDeviceToHost, st_));
    }
    sync();
    bool redo = false;
    for (int P = 0; P < 2; ++P) {
      SvdSector& S = sec_[P];
      S.k = host_k_[P];
      if (S.n == 0) continue;
      if (host_k_[3 + 2 * P] < 0) throw Error(4, "Jacobi SVD did not converge");
      if (!S.direct && S.k >= S.trusted) {
        S.kg = std::min(S.n, S.k + 64);
        redo = true;
      }
    }
    if (!redo) break;
    if (attempt == 3) throw Error(4, "truncated SVD: subspace too small after retries");
  }
  // vectors of the kept states: U from the orthogonalised columns, V from the
  // accumulated rotations (a consistent pair: B V = U S to rounding)
  std::vector<GemmDesc> g;
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    if (S.k == 0) continue;
    gather_cols(S.Bj, S.l, S.perm, S.sv, S.l, S.k, S.Ub, S.k, st_);
    gather_cols(S.Vb, S.l, S.perm, nullptr, S.l, S.k, S.B, S.k, st_);
  }
  for (int P = 0; P < 2; ++P) std::swap(sec_[P].B, sec_[P].Vb);  // Vb <- gathered (l x k)
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
    e.A = S.Qr;
    e.B = S.Vb;
    e.C = S.Vbuf;
    g.push_back(e);
  }
  launch_gemms(g);
  for (int P = 0; P < 2; ++P) {
    SvdSector& S = sec_[P];
    S.kg = S.k;
    if (S.direct) {
      S.W = S.Ub;
      S.V = S.Vb;
    } else {
      S.W = S.Wbuf;
      S.V = S.Vbuf;
    }
  }
}

// ---------------------------------------------------------------- move ----
void Ctm::move(int r) {
  auto mark = [&](int i) {
    if ((int)ev_.size() <= i) {
      hipEvent_t e;
      HCTM_HIP(hipEventCreate(&e));
      ev_.push_back(e);
    }
    HCTM_HIP(hipEventRecord(ev_[i], st_));
  };
  const int e0 = ev_index_;
  mark(e0);
  for (int i = 0; i < 4; ++i) {
    const int j = (r + i) % 4;
    if (!quad_ok_[j]) {
      quadrant(j);
      quad_ok_[j] = true;
    }
  }
  mark(e0 + 1);
  BT& Q1 = quad_[r];
  BT& Q2 = quad_[(r + 1) % 4];
  BT& Q3 = quad_[(r + 2) % 4];
  BT& Q4 = quad_[(r + 3) % 4];
  {
    std::vector<GemmDesc> g;
    plan_contract(Q1, Q2, Hu_, 1.0, 0.0, g);
    plan_contract(Q3, Q4, Hd_, 1.0, 0.0, g);
    launch_gemms(g);
    plan_contract(Hd_, Hu_, M_, 1.0, 0.0, g);
    launch_gemms(g);
  }
  mark(e0 + 2);
  truncated_svd(M_, chi_);
  mark(e0 + 3);

  // projectors
  const Leg kn{sec_[0].k, sec_[1].k};
  const Leg lW = Q1.L.leg[0];
  Pa_.L = Layout({lW, lq_, kn}, 2);
  Pb_.L = Layout({kn, lW, lq_}, 1);
  if (Pa_.L.size > proj_cap_ || Pb_.L.size > proj_cap_) throw Error(2, "projector capacity");
  {
    std::vector<GemmDesc> g;
    for (int P = 0; P < 2; ++P) {
      SvdSector& S = sec_[P];
      if (S.k == 0) continue;
      const int nW = (int)Hu_.L.rows[P], nE = (int)Hu_.L.cols[P];
      GemmDesc d{};
      d.A = Hu_.p + Hu_.L.off[P];
      d.B = S.V;
      d.C = Pa_.p + Pa_.L.off[P];
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
      e.C = Pb_.p + Pb_.L.off[P];
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
  }

  // renormalisation
  BT& C1 = env_[(2 * r) % 8];
  BT& T1 = env_[(2 * r + 1) % 8];
  BT& T3 = env_[(2 * r + 5) % 8];
  BT& C4 = env_[(2 * r + 6) % 8];
  BT& T4 = env_[(2 * r + 7) % 8];
  BT X{Layout(), mid1_, mid_cap_};
  contract(C1, T1, X);                       // [c | u t]
  BT X2{Layout(), mid2_, mid_cap_};
  permute(X, X2, {0, 1, 2}, 2);              // [c u | t]
  BT T3s{Layout(), mid1_, mid_cap_};
  permute(T3, T3s, {0, 1, 2}, 2);            // [r u | x]
  BT Z{Layout(), mid3_, mid_cap_};
  contract(T3s, C4, Z);                      // [r u | c]
  BT Zp{Layout(), mid1_, mid_cap_};
  permute(Z, Zp, {0, 2, 1}, 1);              // [r | c u]
  BT T4s{Layout(), mid3_, mid_cap_};
  permute(T4, T4s, {0, 1, 2}, 2);            // [w l | c]
  BT Pas{Layout(), big2_, big_cap_};
  permute(Pa_, Pas, {0, 1, 2}, 1);           // [c | u k]
  BT G{Layout(), big1_, big_cap_};
  contract(T4s, Pas, G);                     // [w l | u k]
  BT Gp{Layout(), big2_, big_cap_};
  permute(G, Gp, {0, 3, 2, 1}, 2);           // [w k | u l]
  BT H{Layout(), big1_, big_cap_};
  contract(Gp, a_rot_[r], H);                // [w k | e r]
  BT Hp{Layout(), big2_, big_cap_};
  permute(H, Hp, {0, 2, 3, 1}, 2);           // [w e | r k]
  // the old C1, C4, T4 are no longer read: write the new ones in place
  contract(Pb_, X2, C1);                     // [k | t]
  contract(Zp, Pa_, C4);                     // [r | k]
  contract(Pb_, Hp, T4);                     // [k | r k]
  normalise(C1);
  normalise(C4);
  normalise(T4);
  side_[(3 + r) % 4] = kn;
  quad_ok_[r] = false;
  quad_ok_[(r + 3) % 4] = false;
  mark(e0 + 4);
  ev_index_ += 5;

  // record: the kept spectra were copied to the host at the truncation sync
  MoveRecord rec;
  rec.k_even = opt_.form == 0 ? kn.e : kn.e + kn.o;
  rec.k_odd = opt_.form == 0 ? kn.o : 0;
  for (int P = 0; P < 2; ++P)
    for (int i = 0; i < sec_[P].k; ++i) rec.spectrum.push_back(host_d_[2048 * P + i]);
  std::sort(rec.spectrum.begin(), rec.spectrum.end(), [](double a, double b) { return a > b; });
  const double s0 = rec.spectrum.empty() ? 1.0 : rec.spectrum[0];
  for (double& v : rec.spectrum) v /= s0;
  records_.push_back(std::move(rec));
  ++move_count_;
  eps_ok_ = false;
}

// --------------------------------------------------- corner spectra ----
void Ctm::corner_spectra() {
  std::vector<SmallProb> jp;
  SpecArgs a{};
  const int slots[4] = {0, 2, 4, 6};
  double* mat = cmat_;
  for (int c = 0; c < 4; ++c) {
    BT& C = env_[slots[c]];
    for (int P = 0; P < 2; ++P) {
      const int m = (int)C.L.rows[P], n = (int)C.L.cols[P];
      a.sv[2 * c + P] = csv_ + (2 * c + P) * cc_;
      a.nsv[2 * c + P] = (m > 0 && n > 0) ? n : 0;
      if (m == 0 || n == 0) continue;
      HCTM_HIP(hipMemcpyAsync(mat, C.p + C.L.off[P], sizeof(double) * m * n, hipMemcpyDeviceToDevice, st_));
      SmallProb p{};
      p.a = mat;
      p.m = m;
      p.n = n;
      p.lda = n;
      p.rel = 1.1e-16 * std::max(m, 8);
      p.max_sweeps = 40;
      p.info = kdev_ + 8;
      p.sv = csv_ + (2 * c + P) * cc_;
      p.perm = cperm_ + (2 * c + P) * cc_;
      jp.push_back(p);
      mat += (long long)cc_ * cc_;
    }
  }
  jacobi(jp, st_);
  std::swap(cspec_, cspec_old_);
  a.spec_new = cspec_;
  a.spec_old = cspec_old_;
  a.len = cc_;
  a.have_old = have_old_spec_ ? 1 : 0;
  a.delta = misc_ + 16;
  corner_spectra_delta(a, st_);
  have_old_spec_ = true;
}

void Ctm::step(int n_iter) {
  ev_index_ = 0;
  static const int order[4] = {0, 2, 1, 3};
  for (int it = 0; it < n_iter; ++it) {
    for (int m = 0; m < 4; ++m) move(order[m]);
    corner_spectra();
  }
  HCTM_HIP(hipMemcpyAsync(host_d_, misc_ + 16, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  delta_ = host_d_[0];
  flush_gemm_stats();
  // phase times: quadrants, halves, svd, projectors + renormalisation
  timing.assign(4, 0.0);
  for (int i = 0; i + 4 < ev_index_ + 1 && i < (int)ev_.size(); i += 5) {
    for (int ph = 0; ph < 4; ++ph) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev_[i + ph], ev_[i + ph + 1]) == hipSuccess) timing[ph] += ms * 1e-3;
    }
  }
}

// ---------------------------------------------------------- observables ----
void Ctm::compute_epsilon_rot() {
  if (eps_ok_) return;
  BT& C1 = env_[0];
  BT& T1 = env_[1];
  BT& C2 = env_[2];
  BT& T2 = env_[3];
  BT& C3 = env_[4];
  BT& T3 = env_[5];
  BT& C4 = env_[6];
  BT& T4 = env_[7];
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
  BT RB{Layout(), quad_[0].p, quad_[0].capacity};
  permute(RB0, RB, {0, 3, 2, 1}, 2);       // [c c' | Dn R]
  quad_ok_[0] = false;
  contract(LTp, RB, eps_);                 // [U L | Dn R]
  eps_ok_ = true;
}

BT Ctm::pack_impurity(int s, int sp, int kind, int frame) {
  DLArgs g{};
  g.A = A_;
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

// left half of the two-site environment in a frame, closed with an impurity
BT Ctm::left_half(int f, const BT& imp) {
  BT& C1 = env_[(2 * f) % 8];
  BT& T1 = env_[(2 * f + 1) % 8];
  BT& T3 = env_[(2 * f + 5) % 8];
  BT& C4 = env_[(2 * f + 6) % 8];
  BT& T4 = env_[(2 * f + 7) % 8];
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

BT Ctm::right_half(int f, const BT& imp) {
  BT& T1 = env_[(2 * f + 1) % 8];
  BT& C2 = env_[(2 * f + 2) % 8];
  BT& T2 = env_[(2 * f + 3) % 8];
  BT& C3 = env_[(2 * f + 4) % 8];
  BT& T3 = env_[(2 * f + 5) % 8];
  BT T1s{Layout(), mid1_, mid_cap_};
  permute(T1, T1s, {0, 1, 2}, 2);          // [y U | x]
  BT TR{Layout(), mid2_, mid_cap_};
  contract(T1s, C2, TR);                   // [y U | c]
  BT W2{Layout(), big1_, big_cap_};
  contract(TR, T2, W2);                    // [y U | R c'']
  BT W2p{Layout(), big2_, big_cap_};
  permute(W2, W2p, {0, 3, 1, 2}, 2);       // [y c'' | U R]
  BT impp{Layout(), quad_[1].p, quad_[1].capacity};
  quad_ok_[1] = false;
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

void Ctm::rdm1(double* rho) {
  compute_epsilon_rot();
  const int d = d_;
  int nd = 0;
  for (int s = 0; s < d; ++s)
    for (int t = (opt_.form == 0 ? s : 0); t < d; ++t) {
      BT imp = pack_impurity(s, t, opt_.form == 0 ? 1 : 0, 0);
      if (imp.L.size != eps_.L.size) throw Error(1, "rdm1: layout mismatch");
      dots({DotJob{eps_.p, imp.p, eps_.L.size, dots_ + nd}}, dpart_, st_);
      ++nd;
    }
  assemble_rho(dots_, d, opt_.form == 0 ? 1 : 0, rho_, st_);
  HCTM_HIP(hipMemcpyAsync(rho, rho_, sizeof(double) * d * d, hipMemcpyDeviceToHost, st_));
  sync();
}

// rho2: the left and right halves of the 4 x 3 environment, each closed with
// the impurities of one site; in the Z2 form only sym x sym and anti x anti
// pairs couple (the environment is even).
void Ctm::rdm2(int dir, double* rho) {
  const int f = dir == 0 ? 0 : 1;
  const int d = d_;
  halves_used_ = 0;
  std::vector<DotJob> jobs;
  int mode;
  if (opt_.form != 0) {
    std::vector<BT> L, R;
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t) L.push_back(left_half(f, pack_impurity(s, t, 0, f)));
    for (int s = 0; s < d; ++s)
      for (int t = 0; t < d; ++t) R.push_back(right_half(f, pack_impurity(s, t, 0, f)));
    int k = 0;
    for (int a = 0; a < d * d; ++a)
      for (int b = 0; b < d * d; ++b) jobs.push_back(DotJob{L[a].p, R[b].p, L[a].L.size, dots_ + k++});
    mode = 2;
  } else {
    std::vector<BT> Ls, La, Rs, Ra;
    for (int s = 0; s < d; ++s)
      for (int t = s; t < d; ++t) Ls.push_back(left_half(f, pack_impurity(s, t, 1, f)));
    for (int s = 0; s < d; ++s)
      for (int t = s + 1; t < d; ++t) La.push_back(left_half(f, pack_impurity(s, t, 2, f)));
    for (int s = 0; s < d; ++s)
      for (int t = s; t < d; ++t) Rs.push_back(right_half(f, pack_impurity(s, t, 1, f)));
    for (int s = 0; s < d; ++s)
      for (int t = s + 1; t < d; ++t) Ra.push_back(right_half(f, pack_impurity(s, t, 2, f)));
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
  assemble_rho(dots_, d, mode, rho_, st_);
  HCTM_HIP(hipMemcpyAsync(rho, rho_, sizeof(double) * d * d * d * d, hipMemcpyDeviceToHost, st_));
  sync();
}

double Ctm::energy(const double* h_host) {
  const int d = d_, n = d * d;
  std::vector<double> rh(n * n), rv(n * n);
  // device copies of both RDMs, then E = Tr(rho_h h) + Tr(rho_v h) on the GPU
  rdm2(0, rh.data());
  HCTM_HIP(hipMemcpyAsync(rho_ + n * n, rho_, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st_));
  rdm2(1, rv.data());
  // rho_ now holds [rho_v, rho_h]
  HCTM_HIP(hipMemcpyAsync(hdev_, h_host, sizeof(double) * n * n, hipMemcpyHostToDevice, st_));
  trace_products(rho_, 2, hdev_, n, misc_ + 20, st_);
  HCTM_HIP(hipMemcpyAsync(host_d_, misc_ + 20, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  return host_d_[0];
}

// eps in the plain basis (unnormalised) into plain_tmp2_; <eps~, a~> into misc_[24]
void Ctm::epsilon_plain(double* eps_host) {
  compute_epsilon_rot();
  const long long q4 = (long long)q_ * q_ * q_ * q_;
  dots({DotJob{eps_.p, a_rot_[0].p, eps_.L.size, misc_ + 24}}, dpart_, st_);
  fill(plain_tmp_, 0.0, (size_t)q4, st_);
  const long long q = q_;
  const long long st[4] = {q * q * q, q * q, q, 1};
  std::vector<CopyJob> jobs;
  plan_pack(plain_tmp_, st, eps_, false, jobs);
  launch_copies(jobs);
  basis4(plain_tmp_, plain_tmp2_, q_, tabT_idx_, tabT_c_, st_);
  if (eps_host) {
    scale_inv(plain_tmp2_, (size_t)q4, misc_ + 24, st_);
    HCTM_HIP(hipMemcpyAsync(eps_host, plain_tmp2_, sizeof(double) * q4, hipMemcpyDeviceToHost, st_));
    sync();
  }
}

double Ctm::s_err() {
  epsilon_plain(nullptr);
  swap_asym(plain_tmp2_, D_, part_, misc_ + 26, st_);
  HCTM_HIP(hipMemcpyAsync(host_d_, misc_ + 26, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  return host_d_[0];
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
  compute_epsilon_rot();
  // Z11 = <eps~, a~>
  dots({DotJob{eps_.p, a_rot_[0].p, eps_.L.size, misc_ + 40}}, dpart_, st_);
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
