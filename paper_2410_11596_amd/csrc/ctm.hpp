// Directional CTMRG engine in the Z2 (Hermitian) basis, Lx x Ly unit cell.
#pragma once
#include <array>
#include <string>
#include <vector>

#include "blocks.hpp"
#include "hctm_internal.hpp"
#include "linalg.hpp"
#include "tensor.hpp"

namespace hctm {

struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool counting = false;
  double* take(size_t n) {
    const size_t b = ((n * sizeof(double)) + 255) & ~size_t(255);
    if (!counting && used + b > cap) throw Error(2, "workspace too small");
    double* p = counting ? nullptr : reinterpret_cast<double*>(base + used);
    used += b;
    return p;
  }
};

// one truncation: the cut between frame rows `row` and `row`+1 left of frame
// column `column` in a move of frame `frame`
struct MoveRecord {
  std::vector<double> spectrum;  // kept values, merged, descending, / largest
  int k_even = 0, k_odd = 0;
  int frame = 0, column = 0, row = 0;
  int iters[2] = {0, 0};   // subspace iterations per sector (0: decomposed directly)
  int sweeps[2] = {0, 0};  // Jacobi sweeps per sector
  int implicit = 0;        // 1: the matrix was applied through the corners
  int status = 0;          // kRec* bits
};

// MoveRecord::status bits
constexpr int kRecUnconvEven = 1;  // even sector: subspace iteration stopped at its cap
constexpr int kRecUnconvOdd = 2;   // odd sector: the same
constexpr int kRecSplit = 4;       // the chi cut fell inside a near-degenerate multiplet
// relative gap s_k / s_{k+1} - 1 below which the last kept and the first
// discarded value count as one multiplet
constexpr double kSplitGap = 1e-10;

constexpr int kMaxCell = 4;  // Lx, Ly <= kMaxCell

struct Options {
  int form = 0;  // 0 Z2, 1 dense
  int Lx = 1, Ly = 1;
  std::vector<double> boundary;
  double tau = 1e-12;
  int svd_iters = 12;
  int form_m = 0;  // 1: always form the decomposed matrix
  int precision = 0;  // 0: FP64 throughout; block products of the moves in 1: FP32, 2: BF16x3
  int c4v = 0;        // 1: one corner and one edge for a C4v-symmetric tensor (1 x 1 cell)
  unsigned long long seed = 0x5eed;
  int profile = 0;  // 1: time every GEMM launch with HIP events
  int cplx = 0;     // 1: complex tensor in the real representation (1 x 1 cell, Z2 form)
};

struct GemmStats {
  double flops = 0.0;    // algorithmic 2*M*N*K summed over problems
  double seconds = 0.0;  // summed durations of the GEMM kernel launches
  long long launches = 0;
  double reduce_seconds = 0.0;  // split-K reductions that follow some of them
  long long reduce_launches = 0;
};

// per-sector state of the truncated SVD
struct SvdSector {
  int n = 0, l = 0, kg = 0, trusted = 0, k = 0, sweeps = 0, iters = 0;
  int kt = 0;            // Ritz columns decomposed (the leading kt of the basis)
  double* jwork = nullptr;  // column-major scratch of the Jacobi SVD
  int passes = 1;        // CholeskyQR passes of the next orthonormalisation
  double rel0 = 1e-10;   // relative diagonal shift of its first pass
  bool direct = false;
  bool warm = false;     // started from the cut's previous right vectors
  bool fin = false;      // the next iterate is the final one
  bool done = false;
  bool conv = false;     // the residual test ended the subspace iteration (or direct)
  const double* Mp = nullptr;  // sector block of M (n x n, ld = n)
  double *Qr = nullptr, *Ql = nullptr, *Y = nullptr, *Tm = nullptr;
  double* Qold = nullptr;  // projection of Y on the previous left basis (check)
  double *C1 = nullptr, *C2 = nullptr;  // intermediates of M applied through the corners
  double *G = nullptr, *Ri = nullptr, *B = nullptr, *Bj = nullptr;
  double *Ub = nullptr, *Vb = nullptr, *Wbuf = nullptr, *Vbuf = nullptr;
  const double *W = nullptr, *V = nullptr;  // kept vectors (n x k) of M_P
  double *sv = nullptr, *isq = nullptr, *isv = nullptr;
  int *perm = nullptr, *info = nullptr;
  double* vlog = nullptr;  // Jacobi rotation log
};

class Ctm {
 public:
  struct CountTag {};
  Ctm(CountTag, int d, int D, int chi, int Lx, int Ly);
  Ctm(const double* A_host, int d, int D, int chi, const Options& o, hipStream_t stream, void* workspace,
      size_t ws_bytes);
  // complex tensor A = A_re + i A_im (o.cplx must be 1)
  Ctm(const double* A_re, const double* A_im, int d, int D, int chi, const Options& o, hipStream_t stream,
      void* workspace, size_t ws_bytes);
  bool is_complex() const { return cplx_; }
  // complex mode: Hermitian RDMs as real and imaginary parts (host arrays)
  void rdm1_complex(int x, int y, double* re, double* im);
  void rdm2_complex(int x, int y, int dir, double* re, double* im);
  ~Ctm();
  static size_t workspace_bytes(int d, int D, int chi, const Options& o);

  void step(int n_iter);
  void set_precision(int p) { opt_.precision = p; }
  int precision() const { return opt_.precision; }
  double delta() const { return delta_; }
  int svd_unconverged() const { return svd_unconverged_; }
  int multiplet_splits() const { return splits_; }
  // current corner spectrum (merged over the sectors, sum-normalised, zero
  // padded) of corner c (0..3) of site (x, y): len() values into s
  void corner_spectrum(int x, int y, int c, double* s);
  int spectrum_len() const { return cc_; }
  void rdm1(int x, int y, double* rho);
  void rdm2(int x, int y, int dir, double* rho);
  void epsilon_plain(int x, int y, double* eps_host);
  double s_err();      // largest over the sites
  double log_kappa();  // 1x1 cell only
  double energy(const double* h_host);  // mean over the sites of E_h + E_v
  const std::vector<MoveRecord>& records() const { return records_; }
  Leg bond(int x, int y, int side);  // side 0 top, 1 right, 2 bottom, 3 left
  int Lx() const { return Lx_; }
  int Ly() const { return Ly_; }
  hipStream_t stream() const { return st_; }
  std::vector<double> timing;  // per-phase seconds of the last step() call
  GemmStats gemm_stats;        // accumulated since the last reset (profile mode)
  void reset_stats() { gemm_stats = GemmStats(); }

 private:
  void plan_memory(bool counting);
  void setup(const double* A_host);
  void launch_copies(std::vector<CopyJob>& jobs);
  void launch_gemms(std::vector<GemmDesc>& g);
  void permute(const BT& in, BT& out, std::initializer_list<int> perm, int nr_out);
  void contract(const BT& A, const BT& B, BT& C);
  // out = (A B) with legs permuted, written by the products themselves (C:
  // the product's layout, never written); false if not possible (nothing
  // launched; the caller forms C and permutes it)
  bool contract_permuted(const BT& A, const BT& B, BT& C, BT& out, const int* perm, int nr_out);
  BT edge_product(const BT& T4s, const BT& Pas, const BT& a);
  // (Ar + i Ai)(Br + i Bi) with legs permuted, written by the products into
  // outr and, right after it, outi (vbuf, vcap: room for the product's
  // layout, never written); false if not possible (nothing launched)
  bool cmul_permuted(const BT& Ar, const BT& Ai, const BT& Br, const BT& Bi, double* vbuf, long long vcap, BT& outr,
                     BT& outi, const int* perm, int nr_out);
  void normalise(BT& t);
  int site(int x, int y) const;             // wrapped site index y*Lx + x
  int site_of(int r, int X, int Y) const;   // site at frame-r coordinates
  BT& env(int s, int i) { return env_[s * 8 + ((i % 8) + 8) % 8]; }
  BT& quad(int s, int o) { return quad_[s * 4 + (o % 4)]; }
  BT& a_rot(int s, int r) { return a_rot_[s * 4 + (r % 4)]; }
  void quadrant(int s, int o);
  void move(int r);
  void move_c4v();
  void mark(int phase);
  void truncated_svd(const BT* M, int chi, int key, uint64_t salt);  // M null: apply via impl_q_
  void form_M();  // H_u, H_d and M of the cut impl_q_
  void apply_M(std::vector<SvdSector*>& ss, bool trans);
  int oversample(int kg, int key) const;
  void orth(std::vector<SvdSector*>& ss, bool ql);
  void corner_spectra();
  void compute_epsilon_rot(int s);  // eps~ of site s into eps_ (layout [U L | Dn R])
  BT left_half(int frame, int s, const BT& imp);
  BT right_half(int frame, int s, const BT& imp);
  BT pack_impurity(int site, int s, int sp, int kind, int frame);  // kind 0 plain, 1 sym, 2 anti
  void rdm2_dev(int x, int y, int dir, double* dst);
  void sync();
  void top_bottom(BT& top, BT& bot);  // TOP[a U | c], BOT[c' Dn | e] (frame 0)

  // ---- complex tensors in the real representation (ctm_complex.cpp) ----
  // A structured complex tensor X = X_re + i X_im is held as two block
  // tensors: X_re with the layout of total parity 0 (its real even-total
  // blocks) and X_im with total parity 1 (the imaginary parts of its odd-total
  // blocks), X_im stored right after X_re in one buffer.
  bool cplx_ = false;
  std::vector<BT> env_i_, quad_i_, a_rot_i_;
  BT Hu_i_, Hd_i_, M_i_, eps_i_;
  std::vector<BT> Pa_i_, Pb_i_;
  BT R_;                      // real n x n matrix decomposed for the truncation
  double* WH_ = nullptr;      // (D U)^dagger of the kept states, k x n
  double* cimp_ = nullptr;    // two impurities, 2 q^4
  double* a_plain_im_ = nullptr;
  void setup_complex(const double* A_re, const double* A_im);
  void cmul(const BT& Ar, const BT& Ai, const BT& Br, const BT& Bi, BT& Cr, BT& Ci, const double* cscale = nullptr,
            const double* rscale = nullptr);
  void cpermute(const BT& inr, const BT& ini, BT& outr, BT& outi, std::initializer_list<int> perm, int nr_out);
  void cnormalise(BT& r, BT& i);
  void cquadrant(int o);
  void cmove(int r);
  void ccorner_spectra();
  void ccompute_epsilon();
  void cimpurity(int s, int sp, int frame, BT& s1r, BT& s1i, BT& s2r, BT& s2i);
  void cleft_half(int f, const BT& ir, const BT& ii, BT& outr, BT& outi);
  void cright_half(int f, const BT& ir, const BT& ii, BT& outr, BT& outi);
  void rdm2c_dev(int dir, double* re, double* im);
 public:
  double energy_complex(const double* h_host);

 private:

  int d_, D_, chi_, q_, cc_;
  int Lx_ = 1, Ly_ = 1, ns_ = 1;
  Leg lq_;
  Options opt_;
  hipStream_t st_ = nullptr;
  bool own_stream_ = false;
  void* mem_ = nullptr;
  bool own_mem_ = false;
  Arena ar_;

  // device tables and inputs
  int* tab_idx_ = nullptr;   // basis U: row -> up to two plain indices
  double* tab_c_ = nullptr;
  int* tabT_idx_ = nullptr;  // U^T
  double* tabT_c_ = nullptr;
  double* A_ = nullptr;       // ns tensors, site s at s * d D^4
  double* b_ = nullptr;
  std::vector<double*> a_plain_;  // per site: q^4, rotated basis, frame 0
  double* plain_tmp_ = nullptr;  // q^4 scratch
  double* plain_tmp2_ = nullptr;
  std::vector<BT> a_rot_;        // site s, frame r at s*4 + r

  std::vector<BT> env_;          // site s, slot i at s*8 + i
  std::vector<BT> quad_;         // site s, frame o at s*4 + o
  std::vector<char> quad_ok_;

  // scratch
  double *big1_ = nullptr, *big2_ = nullptr;
  long long big_cap_ = 0;
  double *mid1_ = nullptr, *mid2_ = nullptr, *mid3_ = nullptr;
  long long mid_cap_ = 0;
  BT Hu_, Hd_, M_;
  std::vector<BT> Pa_, Pb_;      // one pair per cut of the column being swept
  long long proj_cap_ = 0;
  SvdSector sec_[2];
  std::vector<std::array<int, 2>> kg_;  // kept-state guess per (frame, column, row)
  std::vector<int> iters_prev_;           // subspace iterations of the last truncation per cut
  std::vector<char> chi_cut_;             // the last truncation per cut was ended by chi, not the cutoff
  bool low_prec_ = false;  // block products launched now use opt_.precision (set per move phase)
  bool implicit_ = false;                 // M applied through the corners impl_q_
  const BT* impl_q_[4] = {nullptr, nullptr, nullptr, nullptr};
  struct WarmV {
    double* V = nullptr;  // n x k right vectors of the cut's last truncation
    int n = 0, k = 0;
  };
  std::vector<WarmV> warm_;  // (frame, column, row) x sector
  long long warm_cap_ = 0;
  int l_cap_ = 0;
  double* misc_ = nullptr;  // small device scalars
  int* kdev_ = nullptr;
  int* host_k_ = nullptr;   // pinned
  double* host_d_ = nullptr;  // pinned: 2 cc_ kept values, then kHostMisc scalars
  static constexpr int kHostMisc = 64;
  double* hspec(int P) { return host_d_ + (size_t)P * cc_; }
  double* hmisc() { return host_d_ + 2 * (size_t)cc_; }
  int svd_unconverged_ = 0;  // truncations with a sector stopped at the iteration cap
  int splits_ = 0;           // truncations whose chi cut split a multiplet
  int svd_status_ = 0;       // kRec* bits of the last truncation
  double* part_ = nullptr;
  // corner spectra
  double* cspec_ = nullptr;     // sites x 4 corners x chi (current, normalised)
  double* cspec_old_ = nullptr;
  double* csv_ = nullptr;       // scratch singular values
  int* cperm_ = nullptr;
  double* cmat_ = nullptr;      // scratch copies of corner blocks
  double* cwork_ = nullptr;     // Jacobi scratch for them (cc_ <= 256)
  double* cvec_[2] = {nullptr, nullptr};  // right vectors of each corner block's last decomposition
  double* cvj_ = nullptr;       // rotations of the current one
  double* clog_ = nullptr;      // their logs
  long long clog_n_ = 0;        // doubles per log
  int* cinfo_ = nullptr;        // each block's Jacobi sweep counts
  std::vector<std::array<int, 2>> cdims_;  // block shape at the last decomposition
  std::vector<char> ccur_;      // which of cvec_ holds a block's vectors
  bool have_old_spec_ = false;
  double delta_ = 1e300;
  // observables
  BT eps_;
  int eps_site_ = -1;  // site whose eps~ eps_ holds (-1: none)
  std::vector<MoveRecord> records_;
  std::vector<hipEvent_t> ev_;   // phase marks of the current step()
  std::vector<int> ev_phase_;
  double* halves_ = nullptr;
  long long halves_cap_ = 0;
  int halves_used_ = 0;
  int halves_max_ = 0;
  double* gemm_scratch_ = nullptr;  // split-K partial tiles
  long long gemm_scratch_cap_ = 0;
  double* dots_ = nullptr;     // dot-product results
  double* dpart_ = nullptr;    // dot-product partial sums (64 per job)
  double* rho_ = nullptr;      // device RDM outputs (2 ns d^4)
  double* hdev_ = nullptr;     // bond operator (d^4)
  MoveRecord pending_;
  // profile mode: pending event pairs around every GEMM kernel (kind 0) and
  // split-K reduction (kind 1) launch, and the GEMM kernels' flops
  struct Observer : GemmObserver {
    Ctm* c = nullptr;
    void mark(int kind, int phase, double flops) override;
  } obs_;
  std::vector<hipEvent_t> gev_;
  std::vector<double> gflops_;  // flops per pair; < 0: a reduction pair
  size_t gev_used_ = 0;
  void flush_gemm_stats();
};

}  // namespace hctm
