// HOTRG on the double layer, Z2 (rotated) or plain form (include/hctm_hotrg.h).
//
// Every tensor is a fused-sector block matrix (blocks.hpp), so each
// contraction of a step is one GEMM per parity sector and each leg
// permutation a list of strided block copies; the Gram matrices are block
// diagonal and their sectors go to the batched Jacobi eigensolver together.
// A tensor T[u,l,d,r] is stored as [u l | d r].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "blocks.hpp"
#include "ctm.hpp"
#include "hctm.h"
#include "hctm_hotrg.h"
#include "linalg.hpp"
#include "tensor.hpp"

namespace hctm {
namespace {

constexpr int kSweeps = 40;
constexpr int kEigMax = 4096;   // rows of a Gram sector the eigensolver takes
constexpr int kJacSmall = 141;  // sectors up to this size are decomposed directly (in LDS: n^2 <= 19968)
constexpr int kSubL = 128;      // largest subspace of the iterative eigensolver (max(chi + 32, 2 chi) <= 128)
constexpr int kSubMaxIter = 300;
constexpr double kRitzTol = 1e-12;  // converged: ||G u - lam u|| <= kRitzTol * lam_1 for the leading chi pairs
constexpr double kRitzAccept = 1e-9;

// one Gram sector decomposed by subspace iteration (buffers of a pool slot)
struct EigJob {
  int side = 0, P = 0, n = 0, l = 0, kc = 0, slot = 0;
  const double* G = nullptr;  // n x n, ld n
  double shift = 0.0;         // the iteration runs on G + shift I (rank-deficient G near a fixed point)
  std::vector<double> lam;    // Ritz values of G, descending (host)
};

struct StepRecord {
  std::vector<double> spectrum;
  int k_even = 0, k_odd = 0, side = 0;
  double discarded[2] = {0.0, 0.0};
};

class Hotrg {
 public:
  Hotrg(const double* A, int d, int D, int chi, int form, double tau, int probes, hipStream_t st);
  ~Hotrg();
  void step(int n);
  double log_z();
  void impurity_ratios(double* zb, double* zab);
  void set_bond(const double* h_host);
  double energy();
  void track_rdm1();
  void rdm1(double* rho);
  const std::vector<StepRecord>& records() const { return rec_; }

 private:
  void plan(bool counting);
  void setup(const double* A);
  void permute(const BT& in, BT& out, std::initializer_list<int> perm, int nr_out);
  void contract(const BT& A, const BT& B, BT& C);
  void gram(int side);
  void orth(std::vector<EigJob*>& js, bool from_y);
  void eig_subspace(std::vector<EigJob>& jobs, uint64_t salt);
  void coarse(const BT& upper, const BT& lower, BT& out);
  void impurity(const double* O, int tp, BT& out);
  double trace(const BT& t);
  void sync() { HCTM_HIP(hipStreamSynchronize(st_)); }

  int d_, D_, chi_, form_, q_, C_;
  double tau_;
  int nimp_ = 0;
  hipStream_t st_ = nullptr;
  bool own_stream_ = false;
  void* mem_ = nullptr;
  Arena ar_;
  Leg lq_;
  BT T_, imp_[2], R_, s1_, s2_, s3_, s4_, G_[2], big1_, big2_, U_;
  double* V_[2] = {nullptr, nullptr};
  double* sv_[2] = {nullptr, nullptr};
  int* perm_[2] = {nullptr, nullptr};
  double* vlog_[4] = {nullptr, nullptr, nullptr, nullptr};
  double* jwork_[4] = {nullptr, nullptr, nullptr, nullptr};
  int* jinfo_ = nullptr;
  struct Slot {
    double *Q, *Y, *Uf, *GU, *W, *Ri, *B, *Vb, *Vs, *sv, *isv, *res, *vlog, *work;
    int *perm, *info;
  } slot_[4] = {};
  int* tab_idx_ = nullptr;
  double* tab_c_ = nullptr;
  double* Ad_ = nullptr;
  double* plain_ = nullptr;
  double* plain2_ = nullptr;
  double* misc_ = nullptr;
  double* part_ = nullptr;
  double* gscratch_ = nullptr;
  long long gscratch_cap_ = 0;
  double* host_ = nullptr;  // pinned: spectra, infos, scalars
  std::vector<double> log_norms_;
  std::vector<StepRecord> rec_;
  // bond energy: pairs of impurities (upper, lower), joined in the first step
  struct BondTerm {
    BT up, lo;
  };
  std::vector<BondTerm> bond_;
  void* bond_mem_ = nullptr;
  // one-site RDM: impurities of |s><s'| (Z2: symmetric parts, s <= s')
  std::vector<BT> rdm_;
  std::vector<std::pair<int, int>> rdm_places_;
  void* rdm_mem_ = nullptr;
};

Hotrg::Hotrg(const double* A, int d, int D, int chi, int form, double tau, int probes, hipStream_t st)
    : d_(d), D_(D), chi_(chi), form_(form), tau_(tau) {
  q_ = D * D;
  C_ = std::max(chi, q_);
  nimp_ = probes ? 2 : 0;
  const int qo = (D * D - D) / 2;
  lq_ = form == 0 ? Leg{q_ - qo, qo} : Leg{q_, 0};
  if (st) {
    st_ = st;
  } else {
    HCTM_HIP(hipStreamCreate(&st_));
    own_stream_ = true;
  }
  plan(true);
  const size_t need = ar_.used;
  if (hipMalloc(&mem_, need) != hipSuccess) {
    mem_ = nullptr;
    throw Error(2, "hipMalloc of the HOTRG workspace failed");
  }
  ar_.base = reinterpret_cast<char*>(mem_);
  ar_.cap = need;
  plan(false);
  HCTM_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_), 8192 * sizeof(double), hipHostMallocDefault));
  setup(A);
}

Hotrg::~Hotrg() {
  if (st_) (void)hipStreamSynchronize(st_);
  if (bond_mem_) (void)hipFree(bond_mem_);
  if (rdm_mem_) (void)hipFree(rdm_mem_);
  if (host_) (void)hipHostFree(host_);
  if (mem_) (void)hipFree(mem_);
  if (own_stream_ && st_) (void)hipStreamDestroy(st_);
}

void Hotrg::plan(bool counting) {
  ar_.counting = counting;
  ar_.used = 0;
  const long long C = C_, C2 = C * C, C3 = C2 * C, C4 = C3 * C, C5 = C4 * C, q = q_;
  auto ints = [&](long long n) { return reinterpret_cast<int*>(ar_.take((size_t)((n + 1) / 2))); };
  auto bt = [&](BT& t, long long n) {
    t.p = ar_.take((size_t)n);
    t.capacity = n;
  };
  bt(T_, C4);
  for (int i = 0; i < nimp_; ++i) bt(imp_[i], C4);
  for (BT* t : {&R_, &s1_, &s2_, &s3_, &s4_, &G_[0], &G_[1]}) bt(*t, C4);
  bt(big1_, C5);
  bt(big2_, C5);
  bt(U_, C3);
  for (int s = 0; s < 2; ++s) {
    V_[s] = ar_.take((size_t)C4);
    sv_[s] = ar_.take((size_t)C2);
    perm_[s] = ints(C2);
  }
  for (int i = 0; i < 4; ++i) {
    vlog_[i] = ar_.take(jacobi_log_doubles(kJacSmall, kSweeps));
    jwork_[i] = ar_.take((size_t)kJacSmall * kJacSmall);
  }
  jinfo_ = ints(16);
  for (Slot& z : slot_) {
    const long long nl = (long long)kEigMax * kSubL, ll = (long long)kSubL * kSubL;
    z.Q = ar_.take((size_t)nl);
    z.Y = ar_.take((size_t)nl);
    z.Uf = ar_.take((size_t)nl);
    z.GU = ar_.take((size_t)nl);
    z.W = ar_.take((size_t)ll);
    z.Ri = ar_.take((size_t)ll);
    z.B = ar_.take((size_t)ll);
    z.Vb = ar_.take((size_t)ll);
    z.Vs = ar_.take((size_t)ll);
    z.sv = ar_.take(kSubL);
    z.isv = ar_.take(kSubL);
    z.res = ar_.take(kSubL);
    z.vlog = ar_.take(jacobi_log_doubles(kSubL, kSweeps));
    z.work = ar_.take((size_t)ll);
    z.perm = ints(kSubL);
    z.info = ints(4);
  }
  tab_idx_ = ints(2 * q);
  tab_c_ = ar_.take((size_t)(2 * q));
  Ad_ = ar_.take((size_t)d_ * q * q);
  plain_ = ar_.take((size_t)(q * q * q * q));
  plain2_ = ar_.take((size_t)(q * q * q * q));
  misc_ = ar_.take(64);
  part_ = ar_.take(2048);
  gscratch_cap_ = std::max<long long>(1LL << 22, 4 * C4);
  gscratch_ = ar_.take((size_t)gscratch_cap_);
}

void Hotrg::permute(const BT& in, BT& out, std::initializer_list<int> perm, int nr_out) {
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
  copy_jobs(jobs, st_);
}

void Hotrg::contract(const BT& A, const BT& B, BT& C) {
  std::vector<GemmDesc> g;
  plan_contract(A, B, C, 1.0, 0.0, g);
  gemm(g, st_, gscratch_, gscratch_cap_);
}

void Hotrg::setup(const double* A) {
  const int q = q_;
  std::vector<int> ti, tti;
  std::vector<double> tc, ttc;
  basis_table(D_, form_ == 0, ti, tc, tti, ttc);
  HCTM_HIP(hipMemcpy(tab_idx_, ti.data(), sizeof(int) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(tab_c_, tc.data(), sizeof(double) * 2 * q, hipMemcpyHostToDevice));
  HCTM_HIP(hipMemcpy(Ad_, A, sizeof(double) * d_ * q * q, hipMemcpyHostToDevice));
  DLArgs g;
  g.A = Ad_;
  g.out = plain_;
  g.tab_idx = tab_idx_;
  g.tab_c = tab_c_;
  g.d = d_;
  g.D = D_;
  g.npairs = d_;
  for (int s = 0; s < d_; ++s) {
    g.ket[s] = s;
    g.bra[s] = s;
    g.w[s] = 1.0;
  }
  double_layer_basis(g, st_);
  const long long str[4] = {(long long)q * q * q, (long long)q * q, (long long)q, 1};
  std::vector<CopyJob> jobs;
  T_.L = Layout({lq_, lq_, lq_, lq_}, 2);
  plan_pack(plain_, str, T_, true, jobs);
  copy_jobs(jobs, st_);
  jobs.clear();
  if (nimp_) {
    // the probe b (and |b|) as a D^4 x D^4 matrix between the ket indices
    // (u,l,d,r) and the bra indices, laid out on the joined legs K = k*D + kbar
    const int D = D_;
    const long long n4 = (long long)q * q * q * q;
    for (int w = 0; w < 2; ++w) {
      std::vector<double> b((size_t)n4);
      for (long long e = 0; e < n4; ++e) {
        long long t = e;
        int K[4];
        for (int i = 3; i >= 0; --i) {
          K[i] = (int)(t % q);
          t /= q;
        }
        long long row = 0, col = 0;
        for (int i = 0; i < 4; ++i) {
          row = row * D + K[i] / D;
          col = col * D + K[i] % D;
        }
        const double v = row < col ? 1.0 : (row > col ? -1.0 : 0.0);
        b[(size_t)e] = w == 0 ? v : std::fabs(v);
      }
      sync();  // plain2_ may still be read by the previous rotation
      HCTM_HIP(hipMemcpy(plain2_, b.data(), sizeof(double) * n4, hipMemcpyHostToDevice));
      basis4(plain2_, plain_, q, tab_idx_, tab_c_, st_);
      // b is odd under the bra-ket swap: in the Z2 form only its blocks of
      // odd total parity exist; |b| is even
      imp_[w].L = Layout({lq_, lq_, lq_, lq_}, 2, (form_ == 0 && w == 0) ? 1 : 0);
      plan_pack(plain_, str, imp_[w], true, jobs);
      copy_jobs(jobs, st_);
      jobs.clear();
    }
  }
  norm2(T_.p, (size_t)T_.L.size, misc_, part_, st_);
  scale_inv(T_.p, (size_t)T_.L.size, misc_, st_);
  for (int w = 0; w < nimp_; ++w) scale_inv(imp_[w].p, (size_t)imp_[w].L.size, misc_, st_);
  HCTM_HIP(hipMemcpyAsync(host_, misc_, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  if (!(host_[0] > 0.0) || !std::isfinite(host_[0])) throw Error(4, "HOTRG: the double layer has zero norm");
  log_norms_.assign(1, std::log(host_[0]));
}

// Gram matrix of M[u,l1,l2,d,r1,r2] (the current tensor joined with itself
// along the vertical bond) with rows (l1 l2) (side 0) or (r1 r2) (side 1):
// G = sum_{m m'} A[x1 m x1' m'] B[x2 m x2' m'], A over the upper tensor's
// other legs, B over the lower one's; into G_[side] as [x1 x2 | x1' x2'].
void Hotrg::gram(int side) {
  if (side == 0) {
    permute(T_, s1_, {1, 2, 0, 3}, 2);  // [l m | u r]
    permute(T_, s2_, {0, 3, 1, 2}, 2);  // [u r | l m]
  } else {
    permute(T_, s1_, {3, 2, 0, 1}, 2);  // [r m | u l]
    permute(T_, s2_, {0, 1, 3, 2}, 2);  // [u l | r m]
  }
  contract(s1_, s2_, s3_);  // A [x1 m | x1' m']
  if (side == 0) {
    permute(T_, s1_, {1, 0, 2, 3}, 2);  // [l m | d r]
    permute(T_, s2_, {2, 3, 1, 0}, 2);  // [d r | l m]
  } else {
    permute(T_, s1_, {3, 0, 2, 1}, 2);  // [r m | d l]
    permute(T_, s2_, {2, 1, 3, 0}, 2);  // [d l | r m]
  }
  contract(s1_, s2_, s4_);              // B [x2 m | x2' m']
  permute(s3_, s1_, {0, 2, 1, 3}, 2);   // [x1 x1' | m m']
  permute(s4_, s2_, {1, 3, 0, 2}, 2);   // [m m' | x2 x2']
  contract(s1_, s2_, s3_);              // [x1 x1' | x2 x2']
  permute(s3_, G_[side], {0, 2, 1, 3}, 2);  // [x1 x2 | x1' x2']
}

// Q <- orthonormal basis of Y (from_y) or of Q: two CholeskyQR passes on the
// column-scaled Gram matrix, the first with a small diagonal shift
void Hotrg::orth(std::vector<EigJob*>& js, bool from_y) {
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<GemmDesc> g;
    std::vector<SmallProb> sp;
    for (EigJob* J : js) {
      Slot& z = slot_[J->slot];
      const double* src = pass == 0 ? (from_y ? z.Y : z.Q) : z.GU;
      GemmDesc d{};
      d.A = src;
      d.B = src;
      d.C = z.W;
      d.M = J->l;
      d.N = J->l;
      d.K = J->n;
      d.lda = J->l;
      d.ldb = J->l;
      d.ldc = J->l;
      d.ta = 1;
      d.alpha = 1.0;
      g.push_back(d);
      SmallProb p{};
      p.a = z.W;
      p.b = z.Ri;
      p.m = p.n = J->l;
      p.lda = p.ldb = J->l;
      p.rel = pass == 0 ? 1e-10 : 0.0;
      p.flags = 1;
      p.sv = z.isv;
      p.info = z.info + 2;
      sp.push_back(p);
    }
    gemm(g, st_, gscratch_, gscratch_cap_);
    g.clear();
    chol_inv(sp, st_);
    for (EigJob* J : js) {
      Slot& z = slot_[J->slot];
      GemmDesc d{};
      d.A = pass == 0 ? (from_y ? z.Y : z.Q) : z.GU;
      d.B = z.Ri;
      d.C = pass == 0 ? z.GU : z.Q;
      d.M = J->n;
      d.N = J->l;
      d.K = J->l;
      d.lda = J->l;
      d.ldb = J->l;
      d.ldc = J->l;
      d.alpha = 1.0;
      g.push_back(d);
    }
    gemm(g, st_, gscratch_, gscratch_cap_);
  }
}

// Leading eigenpairs of Gram sectors too large for a direct decomposition:
// subspace iteration Y = (G + shift I) Q, Q = orth(Y), and every third
// iteration a Rayleigh-Ritz step (B = Q^T Y, Jacobi on B, U = Q V) whose
// residuals ||G u - lam u|| over the leading kc pairs decide convergence.
// The shift (1e-14 of the trace) keeps Y of full rank when G is rank
// deficient (near a fixed point), which CholeskyQR needs; it moves no
// eigenvector and is taken off the Ritz values.  The result of job J is in
// its slot: Ritz vectors Uf (n x l, by decreasing value) and J.lam on the
// host.
void Hotrg::eig_subspace(std::vector<EigJob>& jobs, uint64_t salt) {
  if (jobs.empty()) return;
  std::vector<EigJob*> act;
  for (size_t i = 0; i < jobs.size(); ++i) {
    EigJob& J = jobs[i];
    J.slot = (int)i;
    random_fill(slot_[i].Q, (size_t)J.n * J.l, 0x5eed5eedull * (salt + 1) + 7 * i, st_);
    act.push_back(&J);
  }
  orth(act, false);
  for (int t = 0; t < kSubMaxIter && !act.empty(); ++t) {
    std::vector<GemmDesc> g;
    for (EigJob* J : act) {
      Slot& z = slot_[J->slot];
      HCTM_HIP(hipMemcpyAsync(z.Y, z.Q, sizeof(double) * J->n * J->l, hipMemcpyDeviceToDevice, st_));
      GemmDesc d{};  // Y = (G + shift I) Q
      d.A = J->G;
      d.B = z.Q;
      d.C = z.Y;
      d.M = J->n;
      d.N = J->l;
      d.K = J->n;
      d.lda = J->n;
      d.ldb = J->l;
      d.ldc = J->l;
      d.alpha = 1.0;
      d.beta = J->shift;
      g.push_back(d);
    }
    gemm(g, st_, gscratch_, gscratch_cap_);
    g.clear();
    const bool check = t >= 2 && (t % 3 == 2 || t == kSubMaxIter - 1);
    if (check) {
      std::vector<SmallProb> jp;
      for (EigJob* J : act) {
        Slot& z = slot_[J->slot];
        GemmDesc d{};  // B = Q^T Y = Q^T G Q
        d.A = z.Q;
        d.B = z.Y;
        d.C = z.B;
        d.M = J->l;
        d.N = J->l;
        d.K = J->n;
        d.lda = J->l;
        d.ldb = J->l;
        d.ldc = J->l;
        d.ta = 1;
        d.alpha = 1.0;
        g.push_back(d);
        SmallProb p{};
        p.a = z.B;
        p.b = z.Vb;
        p.m = p.n = J->l;
        p.lda = p.ldb = J->l;
        p.rel = 1.1e-16 * J->l;
        p.flags = kJacPairAbs;
        p.max_sweeps = kSweeps;
        p.info = z.info;
        p.sv = z.sv;
        p.perm = z.perm;
        p.vlog = z.vlog;
        p.work = z.work;
        jp.push_back(p);
      }
      gemm(g, st_, gscratch_, gscratch_cap_);
      g.clear();
      jacobi(jp, st_);
      for (EigJob* J : act) {
        Slot& z = slot_[J->slot];
        gather_cols(z.Vb, J->l, z.perm, nullptr, J->l, J->l, z.Vs, J->l, st_);
        for (int w = 0; w < 2; ++w) {
          GemmDesc d{};  // Uf = Q Vs, GU = Y Vs = G Uf
          d.A = w == 0 ? z.Q : z.Y;
          d.B = z.Vs;
          d.C = w == 0 ? z.Uf : z.GU;
          d.M = J->n;
          d.N = J->l;
          d.K = J->l;
          d.lda = J->l;
          d.ldb = J->l;
          d.ldc = J->l;
          d.alpha = 1.0;
          g.push_back(d);
        }
      }
      gemm(g, st_, gscratch_, gscratch_cap_);
      g.clear();
      for (size_t i = 0; i < act.size(); ++i) {
        EigJob* J = act[i];
        Slot& z = slot_[J->slot];
        ritz_resid(z.GU, z.Uf, z.sv, J->n, J->l, J->kc, z.res, st_);
        double* h = host_ + 5000 + 400 * i;
        HCTM_HIP(hipMemcpyAsync(h, z.sv, sizeof(double) * J->l, hipMemcpyDeviceToHost, st_));
        HCTM_HIP(hipMemcpyAsync(h + 200, z.res, sizeof(double) * J->kc, hipMemcpyDeviceToHost, st_));
        HCTM_HIP(hipMemcpyAsync(h + 390, z.info, sizeof(int) * 4, hipMemcpyDeviceToHost, st_));
      }
      sync();
      std::vector<EigJob*> next;
      for (size_t i = 0; i < act.size(); ++i) {
        EigJob* J = act[i];
        const double* h = host_ + 5000 + 400 * i;
        const int* inf = reinterpret_cast<const int*>(h + 390);
        if (inf[0] < 0) throw Error(4, "HOTRG: the Jacobi step of the Rayleigh-Ritz projection did not converge");
        // inf[2] counts the columns that CholeskyQR dropped as numerically
        // dependent, which happens when a Gram sector's rank is below the
        // block (near a product state).  They are zero columns of Q: their
        // Ritz values are zero and fall below the cutoff, as in the CTMRG
        // truncation, so they are not an error.
        double rmax = 0.0;
        for (int c = 0; c < J->kc; ++c) rmax = std::max(rmax, h[200 + c]);
        const double lam1 = h[0];
        const bool last = t == kSubMaxIter - 1;
        if (rmax <= kRitzTol * lam1 || (last && rmax <= kRitzAccept * lam1)) {
          J->lam.assign(h, h + J->l);
          for (double& v : J->lam) v = std::max(0.0, v - J->shift);
        } else if (last) {
          throw Error(4, "HOTRG: the subspace iteration did not converge");
        } else {
          next.push_back(J);
        }
      }
      act.swap(next);
      if (act.empty()) break;
    }
    orth(act, true);
  }
}

// out[u,x,d,y] = sum U[(l1 l2),x] upper[u,l1,m,r1] lower[m,l2,d,r2] U[(r1 r2),y]
// The two products before a permutation are written straight into the
// permuted layout where possible: the product's own layout is only planned
// (in big1_, never written); the first goes to big2_ as the permutation
// would, the second to big1_.
void Hotrg::coarse(const BT& upper, const BT& lower, BT& out) {
  permute(upper, s1_, {0, 2, 3, 1}, 3);  // [u m r1 | l1]
  permute(U_, s2_, {0, 1, 2}, 1);        // [l1 | l2 x]
  const int p1[5] = {0, 2, 4, 1, 3}, p2[5] = {0, 2, 3, 1, 4};
  std::vector<GemmDesc> g;
  if (plan_contract_permuted(s1_, s2_, big1_, big2_, p1, 3, g)) {
    gemm(g, st_, gscratch_, gscratch_cap_);  // [u m r1 | l2 x] as [u r1 x | m l2]
  } else {
    contract(s1_, s2_, big1_);             // [u m r1 | l2 x]
    permute(big1_, big2_, {0, 2, 4, 1, 3}, 3);  // [u r1 x | m l2]
  }
  g.clear();
  BT Y{Layout(), big1_.p, big1_.capacity};
  if (plan_contract_permuted(big2_, lower, big1_, Y, p2, 3, g)) {
    gemm(g, st_, gscratch_, gscratch_cap_);  // [u r1 x | d r2] as [u x d | r1 r2]
    contract(Y, U_, out);                    // [u x d | y]
    return;
  }
  contract(big2_, lower, big1_);         // [u r1 x | d r2]
  permute(big1_, big2_, {0, 2, 3, 1, 4}, 3);  // [u x d | r1 r2]
  contract(big2_, U_, out);              // [u x d | y]
}

void Hotrg::step(int n) {
  for (int it = 0; it < n; ++it) {
    const Leg lh = T_.L.leg[1];
    const long long nsec[2] = {(long long)lh.e * lh.e + (long long)lh.o * lh.o, 2LL * lh.e * lh.o};
    for (int P = 0; P < 2; ++P)
      if (nsec[P] > kEigMax)
        throw Error(1, "HOTRG: a Gram sector of " + std::to_string(nsec[P]) +
                           " rows exceeds the eigensolver's 4096; lower chi");
    gram(0);
    gram(1);
    // eigenpairs of both Gram matrices: sectors up to kJacSmall rows by one
    // batch of direct Jacobi decompositions, larger ones by subspace
    // iteration; the trace of a large sector gives its total weight
    std::vector<SmallProb> jp;
    std::vector<EigJob> sj;
    const long long voff[2] = {0, nsec[0] * nsec[0]}, soff[2] = {0, nsec[0]};
    int big_at[2][2] = {{-1, -1}, {-1, -1}};
    for (int side = 0; side < 2; ++side)
      for (int P = 0; P < 2; ++P) {
        const int nn = (int)nsec[P];
        if (nn == 0) continue;
        if (G_[side].L.rows[P] != nn) throw Error(1, "HOTRG: Gram layout");
        const int idx = side * 2 + P;
        const double* Gp = G_[side].p + G_[side].L.off[P];
        if (nn > kJacSmall) {
          EigJob J;
          J.side = side;
          J.P = P;
          J.n = nn;
          // oversampled to twice the kept count: the Ritz pairs converge at
          // lambda_{l+1} / lambda_chi, slowly on the flat spectra of early steps
          J.l = std::min(nn, std::max(chi_ + 32, 2 * chi_));
          J.kc = std::min(J.l, chi_);
          J.G = Gp;
          big_at[side][P] = (int)sj.size();
          const double* bp[1] = {Gp};
          const int bn[1] = {nn}, bl[1] = {nn};
          trace_blocks(bp, bn, bl, 1, misc_ + 16 + idx, st_);
          sj.push_back(J);
          continue;
        }
        SmallProb p{};
        p.a = G_[side].p + G_[side].L.off[P];
        p.b = V_[side] + voff[P];
        p.m = nn;
        p.n = nn;
        p.lda = nn;
        p.ldb = nn;
        p.rel = 1.1e-16 * nn;
        p.flags = kJacPairAbs;
        p.max_sweeps = kSweeps;
        p.info = jinfo_ + 2 * idx;
        p.sv = sv_[side] + soff[P];
        p.perm = perm_[side] + soff[P];
        p.vlog = vlog_[idx];
        p.work = jwork_[idx];
        jp.push_back(p);
      }
    jacobi(jp, st_);
    if (!sj.empty()) {
      HCTM_HIP(hipMemcpyAsync(host_ + 4100, misc_ + 16, sizeof(double) * 4, hipMemcpyDeviceToHost, st_));
      sync();
      for (EigJob& J : sj) J.shift = 1e-14 * std::max(0.0, host_[4100 + J.side * 2 + J.P]);
    }
    eig_subspace(sj, (uint64_t)rec_.size());
    for (int side = 0; side < 2; ++side)
      for (int P = 0; P < 2; ++P)
        if (nsec[P] > 0 && big_at[side][P] < 0)
          HCTM_HIP(hipMemcpyAsync(host_ + (side * 2 + P) * 1024, sv_[side] + soff[P], sizeof(double) * nsec[P],
                                  hipMemcpyDeviceToHost, st_));
    HCTM_HIP(hipMemcpyAsync(host_ + 4096, jinfo_, sizeof(int) * 8, hipMemcpyDeviceToHost, st_));
    HCTM_HIP(hipMemcpyAsync(host_ + 4100, misc_ + 16, sizeof(double) * 4, hipMemcpyDeviceToHost, st_));
    sync();
    const int* info = reinterpret_cast<const int*>(host_ + 4096);
    // values of sector (side, P): all n of a direct decomposition, or the
    // l Ritz values of a subspace one (the leading chi are converged)
    std::vector<double> lamv[2][2];
    double total[2] = {0.0, 0.0};
    for (int side = 0; side < 2; ++side)
      for (int P = 0; P < 2; ++P) {
        if (nsec[P] == 0) continue;
        const int b = big_at[side][P];
        if (b >= 0) {
          lamv[side][P] = sj[(size_t)b].lam;
          total[side] += host_[4100 + side * 2 + P];
        } else {
          if (info[2 * (side * 2 + P)] < 0) throw Error(4, "HOTRG: the Jacobi eigensolver did not converge");
          const double* h = host_ + (side * 2 + P) * 1024;
          lamv[side][P].assign(h, h + nsec[P]);
          for (double v : lamv[side][P]) total[side] += v;
        }
      }
    // truncation of each side over the merged spectrum (values, then the even
    // sector, then the rank); the side that discards less gives U (the left
    // one on a tie)
    int kc[2][2] = {{0, 0}, {0, 0}};
    double disc[2] = {0.0, 0.0};
    for (int side = 0; side < 2; ++side) {
      struct Ent {
        double v;
        int P, r;
      };
      std::vector<Ent> ent;
      for (int P = 0; P < 2; ++P)
        for (size_t r = 0; r < lamv[side][P].size(); ++r) ent.push_back({lamv[side][P][r], P, (int)r});
      std::stable_sort(ent.begin(), ent.end(), [](const Ent& a, const Ent& b) {
        if (a.v != b.v) return a.v > b.v;
        if (a.P != b.P) return a.P < b.P;
        return a.r < b.r;
      });
      const double smax = ent[0].v;
      long long nkeep = 0;
      for (const Ent& e : ent)
        if (e.v > tau_ * smax) ++nkeep;
      const long long k = std::max<long long>(1, std::min<long long>(chi_, nkeep));
      double kept = 0.0;
      for (long long j = 0; j < k; ++j) {
        kept += ent[(size_t)j].v;
        ++kc[side][ent[(size_t)j].P];
      }
      disc[side] = total[side] - kept;
    }
    // both Gram matrices have the trace ||M||_F^2: weights within 1e-10 of it
    // are a tie
    const int side = disc[1] < disc[0] - 1e-10 * std::max(total[0], total[1]) ? 1 : 0;
    const Leg kn{kc[side][0], kc[side][1]};
    U_.L = Layout({lh, lh, kn}, 2);
    if (U_.L.size > U_.capacity) throw Error(2, "HOTRG: isometry capacity");
    std::vector<CopyJob> ujobs;
    for (int P = 0; P < 2; ++P) {
      const int kP = kn.d(P);
      if (kP == 0) continue;
      const int b = big_at[side][P];
      if (b < 0) {
        gather_cols(V_[side] + voff[P], (int)nsec[P], perm_[side] + soff[P], nullptr, (int)nsec[P], kP,
                    U_.p + U_.L.off[P], kP, st_);
      } else {
        const EigJob& J = sj[(size_t)b];
        if (kP > J.kc) throw Error(1, "HOTRG: kept more states than converged");
        CopyJob c{};
        c.in = slot_[J.slot].Uf;
        c.out = U_.p + U_.L.off[P];
        c.r = 2;
        c.dims[0] = J.n;
        c.dims[1] = kP;
        c.istr[0] = J.l;
        c.istr[1] = 1;
        c.ostr[0] = kP;
        c.ostr[1] = 1;
        ujobs.push_back(c);
      }
    }
    copy_jobs(ujobs, st_);
    StepRecord rec;
    rec.k_even = form_ == 0 ? kn.e : kn.e + kn.o;
    rec.k_odd = form_ == 0 ? kn.o : 0;
    rec.side = side;
    rec.discarded[0] = disc[0];
    rec.discarded[1] = disc[1];
    {
      for (int P = 0; P < 2; ++P)
        for (int i = 0; i < kn.d(P); ++i) rec.spectrum.push_back(lamv[side][P][(size_t)i]);
      std::sort(rec.spectrum.begin(), rec.spectrum.end(), [](double a, double b) { return a > b; });
      const double s0 = rec.spectrum[0];
      for (double& v : rec.spectrum) v /= s0;
    }
    // the pure tensor, then the impurities (above a pure one), all divided
    // by the pure tensor's norm and turned a quarter
    coarse(T_, T_, R_);
    norm2(R_.p, (size_t)R_.L.size, misc_, part_, st_);
    for (int w = 0; w < nimp_; ++w) {
      coarse(imp_[w], T_, s3_);
      scale_inv(s3_.p, (size_t)s3_.L.size, misc_, st_);
      permute(s3_, imp_[w], {3, 0, 1, 2}, 2);
    }
    for (BT& x : rdm_) {
      coarse(x, T_, s3_);
      scale_inv(s3_.p, (size_t)s3_.L.size, misc_, st_);
      permute(s3_, x, {3, 0, 1, 2}, 2);
    }
    // bond terms: the pair joined in the first step, then above a pure tensor
    for (BondTerm& b : bond_) {
      coarse(b.up, rec_.empty() ? b.lo : T_, s3_);
      scale_inv(s3_.p, (size_t)s3_.L.size, misc_, st_);
      permute(s3_, b.up, {3, 0, 1, 2}, 2);
    }
    scale_inv(R_.p, (size_t)R_.L.size, misc_, st_);
    permute(R_, T_, {3, 0, 1, 2}, 2);
    HCTM_HIP(hipMemcpyAsync(host_ + 4200, misc_, sizeof(double), hipMemcpyDeviceToHost, st_));
    sync();
    const double nj = host_[4200];
    if (!(nj > 0.0) || !std::isfinite(nj)) throw Error(4, "HOTRG: the coarse tensor has zero or non-finite norm");
    log_norms_.push_back(std::log(nj));
    rec_.push_back(std::move(rec));
  }
}

// a[O] = sum_{s s'} O[s,s'] A[s] (x) A[s'] (ket s, bra s') in the tensor's
// basis, packed with total parity tp and divided by the initial norm n_0
void Hotrg::impurity(const double* O, int tp, BT& out) {
  const int q = q_;
  DLArgs g;
  g.A = Ad_;
  g.out = plain_;
  g.tab_idx = tab_idx_;
  g.tab_c = tab_c_;
  g.d = d_;
  g.D = D_;
  g.npairs = 0;
  for (int s = 0; s < d_; ++s)
    for (int t = 0; t < d_; ++t)
      if (O[s * d_ + t] != 0.0) {
        if (g.npairs == kMaxPairs) throw Error(1, "HOTRG: too many operator entries");
        g.ket[g.npairs] = s;
        g.bra[g.npairs] = t;
        g.w[g.npairs] = O[s * d_ + t];
        ++g.npairs;
      }
  if (g.npairs == 0) throw Error(1, "HOTRG: empty impurity operator");
  double_layer_basis(g, st_);
  const long long str[4] = {(long long)q * q * q, (long long)q * q, (long long)q, 1};
  out.L = Layout({lq_, lq_, lq_, lq_}, 2, tp);
  std::vector<CopyJob> jobs;
  plan_pack(plain_, str, out, true, jobs);
  copy_jobs(jobs, st_);
  host_[4400] = std::exp(log_norms_[0]);
  HCTM_HIP(hipMemcpyAsync(misc_ + 32, host_ + 4400, sizeof(double), hipMemcpyHostToDevice, st_));
  scale_inv(out.p, (size_t)out.L.size, misc_ + 32, st_);
  sync();  // plain_ and the pinned scalar are reused by the next impurity
}

// h[(s1 s2),(s1' s2')] on a vertical bond, site 1 above site 2:
// h = sum_{a b} E_ab (x) O_ab with E_ab the matrix unit |a><b| and
// O_ab[s2, s2'] = h[(a s2),(b s2')].  In the Z2 form E_ab + E_ba (a <= b) is
// paired with the symmetric part of O_ab + O_ba, E_ab - E_ba (a < b) with
// the antisymmetric part of O_ab - O_ba (mixed parities contribute nothing).
void Hotrg::set_bond(const double* h) {
  if (!rec_.empty()) throw Error(1, "HOTRG: the bond operator must be set before the first step");
  if (d_ > 4) throw Error(1, "HOTRG: the bond energy needs d <= 4");
  const int d = d_;
  auto H = [&](int s1, int s2, int t1, int t2) { return h[(s1 * d + s2) * (d * d) + t1 * d + t2]; };
  struct Term {
    std::vector<double> up, lo;
    int tp;
  };
  std::vector<Term> terms;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      if (form_ == 0 && b < a) continue;
      for (int anti = 0; anti < (form_ == 0 ? 2 : 1); ++anti) {
        if (anti && a == b) continue;
        Term t;
        t.tp = anti;
        t.up.assign((size_t)d * d, 0.0);
        t.lo.assign((size_t)d * d, 0.0);
        bool any = false;
        if (form_ != 0) {
          t.up[(size_t)a * d + b] = 1.0;
          for (int s = 0; s < d; ++s)
            for (int u = 0; u < d; ++u) {
              t.lo[(size_t)s * d + u] = H(a, s, b, u);
              any = any || t.lo[(size_t)s * d + u] != 0.0;
            }
        } else {
          const double sg = anti ? -1.0 : 1.0;
          t.up[(size_t)a * d + b] += 1.0;
          t.up[(size_t)b * d + a] += sg;
          if (a == b) t.up[(size_t)a * d + a] = 1.0;
          // lower: (O_ab + sg O_ba) / 2 (O_aa for a = b), then its
          // (anti)symmetric part
          std::vector<double> o((size_t)d * d);
          for (int s = 0; s < d; ++s)
            for (int u = 0; u < d; ++u) o[(size_t)s * d + u] = 0.5 * (H(a, s, b, u) + sg * H(b, s, a, u));
          for (int s = 0; s < d; ++s)
            for (int u = 0; u < d; ++u) {
              t.lo[(size_t)s * d + u] = 0.5 * (o[(size_t)s * d + u] + sg * o[(size_t)u * d + s]);
              any = any || t.lo[(size_t)s * d + u] != 0.0;
            }
        }
        if (any) terms.push_back(std::move(t));
      }
    }
  if (bond_mem_) {
    HCTM_HIP(hipStreamSynchronize(st_));
    HCTM_HIP(hipFree(bond_mem_));
    bond_mem_ = nullptr;
  }
  bond_.clear();
  if (terms.empty()) return;
  const long long C4 = (long long)C_ * C_ * C_ * C_;
  if (hipMalloc(&bond_mem_, sizeof(double) * C4 * 2 * terms.size()) != hipSuccess) {
    bond_mem_ = nullptr;
    throw Error(2, "hipMalloc of the bond impurities failed");
  }
  double* base = static_cast<double*>(bond_mem_);
  bond_.resize(terms.size());
  for (size_t i = 0; i < terms.size(); ++i) {
    BondTerm& b = bond_[i];
    b.up.p = base + C4 * (2 * i);
    b.up.capacity = C4;
    b.lo.p = base + C4 * (2 * i + 1);
    b.lo.capacity = C4;
    impurity(terms[i].up.data(), terms[i].tp, b.up);
    impurity(terms[i].lo.data(), terms[i].tp, b.lo);
  }
}

void Hotrg::track_rdm1() {
  if (!rec_.empty()) throw Error(1, "HOTRG: the RDM must be requested before the first step");
  if (d_ > 4) throw Error(1, "HOTRG: the RDM needs d <= 4");
  if (!rdm_.empty()) return;
  const int d = d_;
  std::vector<std::pair<int, int>> places;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      if (form_ != 0 || a <= b) places.emplace_back(a, b);
  const long long C4 = (long long)C_ * C_ * C_ * C_;
  if (hipMalloc(&rdm_mem_, sizeof(double) * C4 * places.size()) != hipSuccess) {
    rdm_mem_ = nullptr;
    throw Error(2, "hipMalloc of the RDM impurities failed");
  }
  rdm_.resize(places.size());
  std::vector<double> O((size_t)d * d);
  for (size_t i = 0; i < places.size(); ++i) {
    std::fill(O.begin(), O.end(), 0.0);
    const int a = places[i].first, b = places[i].second;
    if (form_ == 0) {
      O[(size_t)a * d + b] += 0.5;
      O[(size_t)b * d + a] += 0.5;
    } else {
      O[(size_t)a * d + b] = 1.0;
    }
    rdm_[i].p = static_cast<double*>(rdm_mem_) + C4 * i;
    rdm_[i].capacity = C4;
    impurity(O.data(), 0, rdm_[i]);
  }
  rdm_places_ = places;
}

// rho[s,s'] = Z[a(|s><s'|)] / Z, mirrored in the Z2 form, trace one
void Hotrg::rdm1(double* rho) {
  if (rdm_.empty()) throw Error(1, "HOTRG: the RDM was not requested (hotrg_track_rdm1)");
  const int d = d_;
  std::vector<double> r((size_t)d * d, 0.0);
  for (size_t i = 0; i < rdm_.size(); ++i) {
    const int a = rdm_places_[i].first, b = rdm_places_[i].second;
    const double v = trace(rdm_[i]);
    r[(size_t)a * d + b] = v;
    if (form_ == 0) r[(size_t)b * d + a] = v;
  }
  double tr = 0.0;
  for (int s = 0; s < d; ++s) tr += r[(size_t)s * d + s];
  if (!(std::fabs(tr) > 0.0)) throw Error(4, "HOTRG: the RDM has zero trace");
  for (int e = 0; e < d * d; ++e) rho[e] = r[(size_t)e] / tr;
}

double Hotrg::energy() {
  if (bond_.empty()) throw Error(1, "HOTRG: no bond operator (hotrg_set_bond)");
  if (rec_.empty()) throw Error(1, "HOTRG: the bond energy needs at least one step");
  const double tr = trace(T_);
  double e = 0.0;
  for (BondTerm& b : bond_) e += trace(b.up);
  return e / tr;
}

// sum T[u,l,u,l]: the trace of the block matrix [u l | d r]; zero for a
// tensor of odd total parity (no diagonal blocks)
double Hotrg::trace(const BT& t) {
  if (t.L.tp != 0) return 0.0;
  const double* p[2];
  int n[2], ld[2], nb = 0;
  for (int P = 0; P < 2; ++P) {
    if (t.L.rows[P] == 0) continue;
    if (t.L.rows[P] != t.L.cols[P]) throw Error(1, "HOTRG: trace of a non-square block");
    p[nb] = t.p + t.L.off[P];
    n[nb] = (int)t.L.rows[P];
    ld[nb] = (int)t.L.ld(P);
    ++nb;
  }
  trace_blocks(p, n, ld, nb, misc_ + 8, st_);
  HCTM_HIP(hipMemcpyAsync(host_ + 4300, misc_ + 8, sizeof(double), hipMemcpyDeviceToHost, st_));
  sync();
  return host_[4300];
}

double Hotrg::log_z() {
  const double tr = trace(T_);
  if (!(tr > 0.0)) throw Error(4, "HOTRG: the trace of the coarse tensor is not positive");
  double s = 0.0;
  for (size_t j = 0; j < log_norms_.size(); ++j) s += log_norms_[j] / std::ldexp(1.0, (int)j);
  return s + std::log(tr) / std::ldexp(1.0, (int)rec_.size());
}

void Hotrg::impurity_ratios(double* zb, double* zab) {
  if (!nimp_) throw Error(1, "HOTRG: the context carries no probes (hotrg_opts.probes)");
  const double tr = trace(T_);
  *zb = trace(imp_[0]) / tr;
  *zab = trace(imp_[1]) / tr;
}

}  // namespace
}  // namespace hctm

struct hotrg_ctx {
  std::unique_ptr<hctm::Hotrg> h;
  std::string err;
  bool poisoned = false;
};

namespace {

thread_local std::string g_hotrg_err;

template <class F>
int hguarded(hotrg_ctx* c, F f) {
  if (c && c->poisoned) {
    c->err = "context poisoned by an earlier error: " + c->err;
    return CTM_E_STATE;
  }
  try {
    f();
    return CTM_OK;
  } catch (const hctm::Error& e) {
    (c ? c->err : g_hotrg_err) = e.what();
    if (c && (e.code == CTM_E_HIP || e.code == CTM_E_NUMERIC)) c->poisoned = true;
    return e.code;
  } catch (const std::bad_alloc&) {
    (c ? c->err : g_hotrg_err) = "host allocation failed";
    return CTM_E_NOMEM;
  } catch (const std::exception& e) {
    (c ? c->err : g_hotrg_err) = e.what();
    if (c) c->poisoned = true;
    return CTM_E_HIP;
  }
}

}  // namespace

extern "C" {

int hotrg_opts_default(hotrg_opts* o) {
  if (!o) return CTM_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->form = CTM_FORM_Z2;
  o->svd_rel_cutoff = 1e-12;
  return CTM_OK;
}

int hotrg_init(hotrg_ctx** out, const double* A, int d, int D, int chi, const hotrg_opts* o) {
  if (out) *out = nullptr;
  return hguarded(nullptr, [&] {
    if (!out || !A) throw hctm::Error(CTM_E_ARG, "NULL argument");
    hotrg_opts def;
    hotrg_opts_default(&def);
    if (!o) o = &def;
    if (o->form != CTM_FORM_Z2 && o->form != CTM_FORM_DENSE) throw hctm::Error(CTM_E_ARG, "unknown form");
    if (d < 1 || d > 16) throw hctm::Error(CTM_E_ARG, "d must be in [1, 16]");
    if (D < 1 || D > 6) throw hctm::Error(CTM_E_ARG, "D must be in [1, 6]");
    const int cmax = 64;
    if (chi < 1 || std::max(chi, D * D) > cmax)
      throw hctm::Error(CTM_E_ARG, "max(chi, D^2) must be at most " + std::to_string(cmax));
    if (!(o->svd_rel_cutoff >= 0.0) || o->svd_rel_cutoff >= 1.0)
      throw hctm::Error(CTM_E_ARG, "svd_rel_cutoff out of range");
    if (o->probes != 0 && o->probes != 1) throw hctm::Error(CTM_E_ARG, "probes must be 0 or 1");
    const long long n = (long long)d * D * D * D * D;
    for (long long i = 0; i < n; ++i)
      if (!std::isfinite(A[i])) throw hctm::Error(CTM_E_NUMERIC, "A has a non-finite entry");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) throw hctm::Error(CTM_E_HIP, "no HIP device");
    std::unique_ptr<hotrg_ctx> c(new hotrg_ctx);
    c->h.reset(new hctm::Hotrg(A, d, D, chi, o->form == CTM_FORM_Z2 ? 0 : 1, o->svd_rel_cutoff, o->probes,
                               reinterpret_cast<hipStream_t>(o->stream)));
    *out = c.release();
  });
}

int hotrg_step(hotrg_ctx* c, int n) {
  if (!c) return CTM_E_ARG;
  return hguarded(c, [&] {
    if (n < 0) throw hctm::Error(CTM_E_ARG, "n < 0");
    c->h->step(n);
  });
}

int hotrg_log_z(hotrg_ctx* c, double* lnz) {
  if (!c) return CTM_E_ARG;
  return hguarded(c, [&] {
    if (!lnz) throw hctm::Error(CTM_E_ARG, "lnz is NULL");
    *lnz = c->h->log_z();
  });
}

int hotrg_sym_error(hotrg_ctx* c, double* err, double* z_b, double* z_abs) {
  if (!c) return CTM_E_ARG;
  return hguarded(c, [&] {
    double zb = 0.0, zab = 0.0;
    c->h->impurity_ratios(&zb, &zab);
    if (z_b) *z_b = zb;
    if (z_abs) *z_abs = zab;
    if (err) *err = std::fabs(zb) / std::fabs(zab);
  });
}

int hotrg_set_bond(hotrg_ctx* c, const double* h) {
  if (!c) return CTM_E_ARG;
  return hguarded(c, [&] {
    if (!h) throw hctm::Error(CTM_E_ARG, "h is NULL");
    c->h->set_bond(h);
  });
}

int hotrg_energy(hotrg_ctx* c, double* e) {
  if (!c) return CTM_E_ARG;
  return hguarded(c, [&] {
    if (!e) throw hctm::Error(CTM_E_ARG, "e is NULL");
    *e = c->h->energy();
  });
}

int hotrg_track_rdm1(hotrg_ctx* c) {
  if (!c) return CTM_E_ARG;
  return hguarded(c, [&] { c->h->track_rdm1(); });
}

int hotrg_rdm1(hotrg_ctx* c, double* rho) {
  if (!c) return CTM_E_ARG;
  return hguarded(c, [&] {
    if (!rho) throw hctm::Error(CTM_E_ARG, "rho is NULL");
    c->h->rdm1(rho);
  });
}

int hotrg_num_records(hotrg_ctx* c, int* n) {
  if (!c || !n) return CTM_E_ARG;
  *n = (int)c->h->records().size();
  return CTM_OK;
}

int hotrg_record(hotrg_ctx* c, int i, double* spectrum, int cap, int* n, int* k_even, int* k_odd, int* side,
                 double* discarded) {
  if (!c) return CTM_E_ARG;
  const auto& r = c->h->records();
  if (i < 0 || i >= (int)r.size() || cap < 0 || (cap > 0 && !spectrum)) return CTM_E_ARG;
  const hctm::StepRecord& x = r[(size_t)i];
  const int m = (int)x.spectrum.size();
  for (int j = 0; j < std::min(m, cap); ++j) spectrum[j] = x.spectrum[(size_t)j];
  if (n) *n = m;
  if (k_even) *k_even = x.k_even;
  if (k_odd) *k_odd = x.k_odd;
  if (side) *side = x.side;
  if (discarded) {
    discarded[0] = x.discarded[0];
    discarded[1] = x.discarded[1];
  }
  return CTM_OK;
}

const char* hotrg_last_error(const hotrg_ctx* c) { return c ? c->err.c_str() : g_hotrg_err.c_str(); }

void hotrg_free(hotrg_ctx* c) { delete c; }

}  // extern "C"
