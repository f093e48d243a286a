// C ABI of libhctm.so (declared in include/hctm.h and include/hctm_testing.h).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "ctm.hpp"
#include "hctm.h"
#include "hctm_testing.h"
#include "linalg.hpp"

struct ctm_ctx {
  std::unique_ptr<hctm::Ctm> ctm;
  std::string err;
  bool poisoned = false;
  int d = 0, D = 0, chi = 0, form = 0;
};

namespace {

thread_local std::string g_err;

template <class F>
int guarded(ctm_ctx* c, F f) {
  if (c && c->poisoned) {
    c->err = "context poisoned by an earlier error: " + c->err;
    return CTM_E_STATE;
  }
  try {
    f();
    return CTM_OK;
  } catch (const hctm::Error& e) {
    (c ? c->err : g_err) = e.what();
    if (c && (e.code == CTM_E_HIP || e.code == CTM_E_NUMERIC)) c->poisoned = true;
    return e.code;
  } catch (const std::bad_alloc&) {
    (c ? c->err : g_err) = "host allocation failed";
    return CTM_E_NOMEM;
  } catch (const std::exception& e) {
    (c ? c->err : g_err) = e.what();
    if (c) c->poisoned = true;
    return CTM_E_HIP;
  }
}

hctm::Options to_options(const ctm_opts* o, int D) {
  hctm::Options opt;
  ctm_opts def;
  ctm_opts_default(&def);
  if (!o) o = &def;
  if (o->form != CTM_FORM_Z2 && o->form != CTM_FORM_DENSE) throw hctm::Error(CTM_E_ARG, "unknown form");
  opt.form = o->form == CTM_FORM_Z2 ? 0 : 1;
  if (o->Lx < 1 || o->Lx > hctm::kMaxCell || o->Ly < 1 || o->Ly > hctm::kMaxCell)
    throw hctm::Error(CTM_E_ARG, "Lx and Ly must be in [1, 4]");
  opt.Lx = o->Lx;
  opt.Ly = o->Ly;
  if (!(o->svd_rel_cutoff >= 0.0) || o->svd_rel_cutoff >= 1.0) throw hctm::Error(CTM_E_ARG, "svd_rel_cutoff out of range");
  opt.tau = o->svd_rel_cutoff;
  if (o->svd_iters < 1 || o->svd_iters > 1000) throw hctm::Error(CTM_E_ARG, "svd_iters out of range");
  opt.svd_iters = o->svd_iters;
  if (o->form_m != 0 && o->form_m != 1) throw hctm::Error(CTM_E_ARG, "form_m must be 0 or 1");
  opt.form_m = o->form_m;
  if (o->precision != CTM_PREC_FP64 && o->precision != CTM_PREC_FP32 && o->precision != CTM_PREC_BF16X3)
    throw hctm::Error(CTM_E_ARG, "precision must be CTM_PREC_FP64, CTM_PREC_FP32 or CTM_PREC_BF16X3");
  opt.precision = o->precision;
  if (o->c4v != 0 && o->c4v != 1) throw hctm::Error(CTM_E_ARG, "c4v must be 0 or 1");
  if (o->c4v && (o->Lx != 1 || o->Ly != 1)) throw hctm::Error(CTM_E_ARG, "c4v needs a 1 x 1 cell");
  opt.c4v = o->c4v;
  opt.seed = o->seed;
  opt.profile = o->profile ? 1 : 0;
  if (o->boundary) {
    const int q = D * D;
    opt.boundary.assign(o->boundary, o->boundary + q);
    double mx = 0.0;
    for (double v : opt.boundary) {
      if (!std::isfinite(v)) throw hctm::Error(CTM_E_NUMERIC, "boundary vector is not finite");
      mx = std::max(mx, std::fabs(v));
    }
    if (mx == 0.0) throw hctm::Error(CTM_E_ARG, "boundary vector is zero");
    if (opt.form == 0) {
      for (int k = 0; k < D; ++k)
        for (int l = 0; l < D; ++l)
          if (std::fabs(opt.boundary[k * D + l] - opt.boundary[l * D + k]) > 1e-14 * mx)
            throw hctm::Error(CTM_E_ARG, "boundary vector is not swap symmetric (required in the Z2 form)");
    }
  }
  return opt;
}

// A[s,u,l,d,r] unchanged (to tol relative to its largest entry) by the
// rotation (u,l,d,r) -> (l,d,r,u) and the reflection l <-> r, which generate
// the symmetry group of the square
bool is_c4v(const double* A, int d, int D, double tol) {
  const long long D2 = (long long)D * D, D3 = D2 * D, D4 = D3 * D;
  double mx = 0.0;
  for (long long i = 0; i < d * D4; ++i) mx = std::max(mx, std::fabs(A[i]));
  const double lim = tol * mx;
  for (int s = 0; s < d; ++s)
    for (int u = 0; u < D; ++u)
      for (int l = 0; l < D; ++l)
        for (int dn = 0; dn < D; ++dn)
          for (int r = 0; r < D; ++r) {
            const double* a = A + s * D4;
            const double x = a[u * D3 + l * D2 + dn * D + r];
            if (std::fabs(x - a[l * D3 + dn * D2 + r * D + u]) > lim) return false;
            if (std::fabs(x - a[u * D3 + r * D2 + dn * D + l]) > lim) return false;
          }
  return true;
}

void check_sizes(int d, int D, int chi) {
  if (d < 1 || d > 16) throw hctm::Error(CTM_E_ARG, "d must be in [1, 16]");
  if (D < 1 || D > 8) throw hctm::Error(CTM_E_ARG, "D must be in [1, 8]");
  if (chi < 1 || chi > 4096) throw hctm::Error(CTM_E_ARG, "chi must be in [1, 4096]");
}

}  // namespace

extern "C" {

int ctm_opts_default(ctm_opts* o) {
  if (!o) return CTM_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->form = CTM_FORM_Z2;
  o->Lx = 1;
  o->Ly = 1;
  o->boundary = nullptr;
  o->svd_rel_cutoff = 1e-12;
  o->svd_iters = 12;
  o->form_m = 0;
  o->seed = 0x5eedull;
  return CTM_OK;
}

int ctm_workspace_size(int d, int D, int chi, const ctm_opts* o, size_t* bytes) {
  return guarded(nullptr, [&] {
    if (!bytes) throw hctm::Error(CTM_E_ARG, "bytes is NULL");
    check_sizes(d, D, chi);
    hctm::Options opt = to_options(o, D);
    *bytes = hctm::Ctm::workspace_bytes(d, D, chi, opt);
  });
}

int ctm_init(ctm_ctx** out, const double* A, int d, int D, int chi, const ctm_opts* o) {
  if (out) *out = nullptr;
  return guarded(nullptr, [&] {
    if (!out || !A) throw hctm::Error(CTM_E_ARG, "NULL argument");
    check_sizes(d, D, chi);
    hctm::Options opt = to_options(o, D);
    const long long n = (long long)d * D * D * D * D * opt.Lx * opt.Ly;
    for (long long i = 0; i < n; ++i)
      if (!std::isfinite(A[i])) throw hctm::Error(CTM_E_NUMERIC, "A has a non-finite entry");
    if (opt.c4v && !is_c4v(A, d, D, 1e-12))
      throw hctm::Error(CTM_E_ARG, "c4v: A is not invariant under the rotations and reflections of the square");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) throw hctm::Error(CTM_E_HIP, "no HIP device");
    std::unique_ptr<ctm_ctx> c(new ctm_ctx);
    c->d = d;
    c->D = D;
    c->chi = chi;
    c->form = opt.form;
    void* stream = o ? o->stream : nullptr;
    void* ws = o ? o->workspace : nullptr;
    const size_t wsb = o ? o->workspace_bytes : 0;
    c->ctm.reset(new hctm::Ctm(A, d, D, chi, opt, reinterpret_cast<hipStream_t>(stream), ws, wsb));
    *out = c.release();
  });
}

int ctm_workspace_size_complex(int d, int D, int chi, const ctm_opts* o, size_t* bytes) {
  return guarded(nullptr, [&] {
    if (!bytes) throw hctm::Error(CTM_E_ARG, "bytes is NULL");
    check_sizes(d, D, chi);
    hctm::Options opt = to_options(o, D);
    opt.cplx = 1;
    *bytes = hctm::Ctm::workspace_bytes(d, D, chi, opt);
  });
}

int ctm_init_complex(ctm_ctx** out, const double* A_re, const double* A_im, int d, int D, int chi,
                     const ctm_opts* o) {
  if (out) *out = nullptr;
  return guarded(nullptr, [&] {
    if (!out || !A_re || !A_im) throw hctm::Error(CTM_E_ARG, "NULL argument");
    check_sizes(d, D, chi);
    if (d > 8) throw hctm::Error(CTM_E_ARG, "complex tensors: d must be at most 8");
    hctm::Options opt = to_options(o, D);
    if (opt.form != 0 || opt.Lx != 1 || opt.Ly != 1 || opt.c4v || opt.precision != 0)
      throw hctm::Error(CTM_E_ARG, "complex tensors: Z2 form, 1 x 1 cell, directional moves and FP64 only");
    opt.cplx = 1;
    const long long n = (long long)d * D * D * D * D;
    for (long long i = 0; i < n; ++i)
      if (!std::isfinite(A_re[i]) || !std::isfinite(A_im[i])) throw hctm::Error(CTM_E_NUMERIC, "A has a non-finite entry");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) throw hctm::Error(CTM_E_HIP, "no HIP device");
    std::unique_ptr<ctm_ctx> c(new ctm_ctx);
    c->d = d;
    c->D = D;
    c->chi = chi;
    c->form = 0;
    void* stream = o ? o->stream : nullptr;
    void* ws = o ? o->workspace : nullptr;
    const size_t wsb = o ? o->workspace_bytes : 0;
    c->ctm.reset(new hctm::Ctm(A_re, A_im, d, D, chi, opt, reinterpret_cast<hipStream_t>(stream), ws, wsb));
    *out = c.release();
  });
}

int ctm_rdm_1site_complex(ctm_ctx* c, int x, int y, double* rho_re, double* rho_im) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (!rho_re || !rho_im) throw hctm::Error(CTM_E_ARG, "NULL argument");
    if (!c->ctm->is_complex()) throw hctm::Error(CTM_E_ARG, "not a complex context (use ctm_rdm_1site)");
    if (x != 0 || y != 0) throw hctm::Error(CTM_E_ARG, "site outside the cell");
    c->ctm->rdm1_complex(x, y, rho_re, rho_im);
  });
}

int ctm_rdm_2site_complex(ctm_ctx* c, int x, int y, int dir, double* rho_re, double* rho_im) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (!rho_re || !rho_im) throw hctm::Error(CTM_E_ARG, "NULL argument");
    if (!c->ctm->is_complex()) throw hctm::Error(CTM_E_ARG, "not a complex context (use ctm_rdm_2site)");
    if (dir != 0 && dir != 1) throw hctm::Error(CTM_E_ARG, "dir must be 0 or 1");
    if (x != 0 || y != 0) throw hctm::Error(CTM_E_ARG, "site outside the cell");
    c->ctm->rdm2_complex(x, y, dir, rho_re, rho_im);
  });
}

int ctm_step(ctm_ctx* c, int n_iter) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (n_iter < 0) throw hctm::Error(CTM_E_ARG, "n_iter < 0");
    c->ctm->step(n_iter);
  });
}

int ctm_set_precision(ctm_ctx* c, int precision) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (precision != CTM_PREC_FP64 && precision != CTM_PREC_FP32 && precision != CTM_PREC_BF16X3)
      throw hctm::Error(CTM_E_ARG, "precision must be CTM_PREC_FP64, CTM_PREC_FP32 or CTM_PREC_BF16X3");
    if (c->ctm->is_complex() && precision != CTM_PREC_FP64)
      throw hctm::Error(CTM_E_ARG, "complex tensors run in FP64 only");
    c->ctm->set_precision(precision);
  });
}

int ctm_converged(ctm_ctx* c, double tol, int* converged, double* delta) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    const double dl = c->ctm->delta();
    if (delta) *delta = dl >= 1e299 ? INFINITY : dl;
    if (converged) *converged = dl < tol ? 1 : 0;
  });
}

static void check_site(const ctm_ctx* c, int x, int y) {
  if (x < 0 || y < 0 || x >= c->ctm->Lx() || y >= c->ctm->Ly()) throw hctm::Error(CTM_E_ARG, "site outside the cell");
}

int ctm_rdm_1site(ctm_ctx* c, int x, int y, double* rho) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (!rho) throw hctm::Error(CTM_E_ARG, "rho is NULL");
    if (c->ctm->is_complex()) throw hctm::Error(CTM_E_ARG, "complex context: use ctm_rdm_1site_complex");
    check_site(c, x, y);
    c->ctm->rdm1(x, y, rho);
  });
}

int ctm_rdm_2site(ctm_ctx* c, int x, int y, int dir, double* rho) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (!rho) throw hctm::Error(CTM_E_ARG, "rho is NULL");
    if (dir != 0 && dir != 1) throw hctm::Error(CTM_E_ARG, "dir must be 0 or 1");
    if (c->ctm->is_complex()) throw hctm::Error(CTM_E_ARG, "complex context: use ctm_rdm_2site_complex");
    check_site(c, x, y);
    c->ctm->rdm2(x, y, dir, rho);
  });
}

int ctm_energy(ctm_ctx* c, const double* h, double* e) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (!h || !e) throw hctm::Error(CTM_E_ARG, "NULL argument");
    *e = c->ctm->is_complex() ? c->ctm->energy_complex(h) : c->ctm->energy(h);
  });
}

void ctm_free(ctm_ctx* c) { delete c; }

const char* ctm_last_error(const ctm_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

int ctm_env_epsilon(ctm_ctx* c, int x, int y, double* eps) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (!eps) throw hctm::Error(CTM_E_ARG, "eps is NULL");
    if (c->ctm->is_complex()) throw hctm::Error(CTM_E_ARG, "not available for a complex context");
    check_site(c, x, y);
    c->ctm->epsilon_plain(x, y, eps);
  });
}

int ctm_s_err(ctm_ctx* c, double* s) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (!s) throw hctm::Error(CTM_E_ARG, "NULL argument");
    if (c->ctm->is_complex()) throw hctm::Error(CTM_E_ARG, "not available for a complex context");
    *s = c->ctm->s_err();
  });
}

int ctm_log_kappa(ctm_ctx* c, double* lk) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (!lk) throw hctm::Error(CTM_E_ARG, "NULL argument");
    if (c->ctm->is_complex()) throw hctm::Error(CTM_E_ARG, "not available for a complex context");
    *lk = c->ctm->log_kappa();
  });
}

int ctm_num_records(ctm_ctx* c, int* n) {
  if (!c || !n) return CTM_E_ARG;
  *n = (int)c->ctm->records().size();
  return CTM_OK;
}

int ctm_record(ctm_ctx* c, int m, double* s, int cap, int* n, int* k_even, int* k_odd, int* info) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    const auto& r = c->ctm->records();
    if (m < 0 || m >= (int)r.size()) throw hctm::Error(CTM_E_ARG, "record index out of range");
    const auto& rec = r[m];
    const int ns = (int)rec.spectrum.size();
    if (n) *n = ns;
    if (k_even) *k_even = rec.k_even;
    if (k_odd) *k_odd = rec.k_odd;
    if (info) {
      info[0] = rec.frame;
      info[1] = rec.column;
      info[2] = rec.row;
      info[3] = rec.iters[0];
      info[4] = rec.iters[1];
      info[5] = rec.sweeps[0];
      info[6] = rec.sweeps[1];
      info[7] = rec.implicit;
    }
    if (s)
      for (int i = 0; i < ns && i < cap; ++i) s[i] = rec.spectrum[i];
  });
}

int ctm_record_status(ctm_ctx* c, int m, int* status) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    const auto& r = c->ctm->records();
    if (!status) throw hctm::Error(CTM_E_ARG, "status is NULL");
    if (m < 0 || m >= (int)r.size()) throw hctm::Error(CTM_E_ARG, "record index out of range");
    *status = r[m].status;
  });
}

int ctm_svd_health(ctm_ctx* c, int* unconverged, int* multiplet_splits) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (unconverged) *unconverged = c->ctm->svd_unconverged();
    if (multiplet_splits) *multiplet_splits = c->ctm->multiplet_splits();
  });
}

int ctm_corner_spectrum(ctm_ctx* c, int x, int y, int corner, double* s, int cap, int* n) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (corner < 0 || corner > 3) throw hctm::Error(CTM_E_ARG, "corner must be 0..3");
    check_site(c, x, y);
    const int len = c->ctm->spectrum_len();
    if (n) *n = len;
    if (s) {
      if (cap < len) throw hctm::Error(CTM_E_ARG, "cap is smaller than the spectrum length");
      c->ctm->corner_spectrum(x, y, corner, s);
    }
  });
}

int ctm_sector_dims(ctm_ctx* c, int x, int y, int side, int* chi_even, int* chi_odd) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    if (side < 0 || side > 3) throw hctm::Error(CTM_E_ARG, "side must be 0..3");
    check_site(c, x, y);
    const hctm::Leg l = c->ctm->bond(x, y, side);
    if (chi_even) *chi_even = l.e;
    if (chi_odd) *chi_odd = l.o;
  });
}

int ctm_timing(ctm_ctx* c, double* t, int cap, int* n) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    const auto& tm = c->ctm->timing;
    if (n) *n = (int)tm.size();
    if (t)
      for (int i = 0; i < (int)tm.size() && i < cap; ++i) t[i] = tm[i];
  });
}

int ctm_gemm_reduce_stats(ctm_ctx* c, double* seconds, long long* launches) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    const hctm::GemmStats& g = c->ctm->gemm_stats;
    if (seconds) *seconds = g.reduce_seconds;
    if (launches) *launches = g.reduce_launches;
  });
}

int ctm_gemm_stats(ctm_ctx* c, double* flops, double* seconds, long long* launches, int reset) {
  if (!c) return CTM_E_ARG;
  return guarded(c, [&] {
    const hctm::GemmStats& g = c->ctm->gemm_stats;
    if (flops) *flops = g.flops;
    if (seconds) *seconds = g.seconds;
    if (launches) *launches = g.launches;
    if (reset) c->ctm->reset_stats();
  });
}

// ---------------------------------------------------------- test hooks ----
static int dev_gemm(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb, int ldc, int ta,
                    int tb, double alpha, double beta, const double* cscale, double* scratch, long long scratch_doubles,
                    void* stream, int prec) {
  return guarded(nullptr, [&] {
    if (M < 0 || N < 0 || K < 0) throw hctm::Error(CTM_E_ARG, "negative size");
    hctm::GemmDesc d{};
    d.A = A;
    d.B = B;
    d.C = C;
    d.M = M;
    d.N = N;
    d.K = K;
    d.lda = lda;
    d.ldb = ldb;
    d.ldc = ldc;
    d.ta = ta;
    d.tb = tb;
    d.alpha = alpha;
    d.beta = beta;
    d.cscale = cscale;
    d.rscale = nullptr;
    d.prec = prec;
    hctm::gemm({d}, reinterpret_cast<hipStream_t>(stream), scratch, scratch_doubles);
  });
}

int hctm_dev_gemm(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb, int ldc, int ta,
                  int tb, double alpha, double beta, const double* cscale, double* scratch, long long scratch_doubles,
                  void* stream) {
  return dev_gemm(A, B, C, M, N, K, lda, ldb, ldc, ta, tb, alpha, beta, cscale, scratch, scratch_doubles, stream, 0);
}

int hctm_dev_gemm_f32(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb, int ldc,
                      int ta, int tb, double alpha, double beta, const double* cscale, double* scratch,
                      long long scratch_doubles, void* stream) {
  return dev_gemm(A, B, C, M, N, K, lda, ldb, ldc, ta, tb, alpha, beta, cscale, scratch, scratch_doubles, stream, 1);
}

int hctm_dev_gemm_bf16x3(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb,
                         int ldc, int ta, int tb, double alpha, double beta, const double* cscale, double* scratch,
                         long long scratch_doubles, void* stream) {
  return dev_gemm(A, B, C, M, N, K, lda, ldb, ldc, ta, tb, alpha, beta, cscale, scratch, scratch_doubles, stream, 2);
}

int hctm_dev_gemm_scatter(const double* A, const double* B, double* C, int M, int N, int K, int lda, int ldb,
                          int ta, int tb, double alpha, double beta, int T, int R, const long long* strides,
                          void* stream) {
  return guarded(nullptr, [&] {
    if (M < 1 || N < 1 || K < 1 || T < 1 || R < 1 || M % T != 0 || N % R != 0 || !strides)
      throw hctm::Error(CTM_E_ARG, "sizes must be positive with T dividing M and R dividing N");
    hctm::GemmDesc d{};
    d.A = A;
    d.B = B;
    d.C = C;
    d.M = M;
    d.N = N;
    d.K = K;
    d.lda = lda;
    d.ldb = ldb;
    d.ldc = N;
    d.ta = ta;
    d.tb = tb;
    d.alpha = alpha;
    d.beta = beta;
    d.sc_rn = 2;
    d.sc_cn = 2;
    d.sc_rd[0] = T;
    d.sc_cd[0] = R;
    d.sc_rs[0] = strides[0];
    d.sc_rs[1] = strides[1];
    d.sc_cs[0] = strides[2];
    d.sc_cs[1] = strides[3];
    hctm::gemm({d}, reinterpret_cast<hipStream_t>(stream));
  });
}

int hctm_dev_mfma_probe(double* sink, int blocks, int iters, double* flops, void* stream) {
  return guarded(nullptr, [&] {
    if (blocks < 1 || iters < 1) throw hctm::Error(CTM_E_ARG, "blocks and iters must be positive");
    const double f = hctm::mfma_probe(sink, blocks, iters, reinterpret_cast<hipStream_t>(stream));
    if (flops) *flops = f;
  });
}

int hctm_dev_stream_probe(const double* in, double* out, long long n, void* stream) {
  return guarded(nullptr, [&] {
    if (n < 0) throw hctm::Error(CTM_E_ARG, "negative size");
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15)
      throw hctm::Error(CTM_E_ARG, "stream probe buffers must be 16-byte aligned");
    hctm::stream_probe(in, out, n, reinterpret_cast<hipStream_t>(stream));
  });
}

int hctm_dev_copy(const double* in, double* out, int r, const int* dims, const long long* istr, const long long* ostr,
                  void* stream) {
  return guarded(nullptr, [&] {
    if (r < 1 || r > hctm::kMaxRank) throw hctm::Error(CTM_E_ARG, "rank out of range");
    hctm::CopyJob j{};
    j.in = in;
    j.out = out;
    j.r = r;
    for (int i = 0; i < r; ++i) {
      j.dims[i] = dims[i];
      j.istr[i] = istr[i];
      j.ostr[i] = ostr[i];
    }
    hctm::copy_jobs({j}, reinterpret_cast<hipStream_t>(stream));
  });
}

int hctm_dev_chol_inv(double* G, double* Rinv, int n, double rel, int* info, void* stream) {
  return guarded(nullptr, [&] {
    if (n < 1) throw hctm::Error(CTM_E_ARG, "n < 1");
    hctm::SmallProb p{};
    p.a = G;
    p.b = Rinv;
    p.m = p.n = n;
    p.lda = p.ldb = n;
    p.rel = rel;
    p.info = info;
    hctm::chol_inv({p}, reinterpret_cast<hipStream_t>(stream));
  });
}

int hctm_dev_jacobi(double* X, int m, int n, double tol, int max_sweeps, int pre, double* sv, int* perm,
                    int* sweeps, double* V, double* vlog, double* work, void* stream) {
  return guarded(nullptr, [&] {
    if (m < 1 || n < 1 || n > 1024) throw hctm::Error(CTM_E_ARG, "size out of range");
    hctm::SmallProb p{};
    p.a = X;
    p.m = m;
    p.n = n;
    p.lda = n;
    p.rel = tol;
    p.max_sweeps = max_sweeps;
    p.pre = pre;
    p.info = sweeps;
    p.sv = sv;
    p.perm = perm;
    p.b = V;
    p.vlog = vlog;
    p.work = work;
    if (V && m != n) throw hctm::Error(CTM_E_ARG, "V needs a square X");
    hctm::jacobi({p}, reinterpret_cast<hipStream_t>(stream));
  });
}

long long hctm_dev_jacobi_log_doubles(int n, int max_sweeps) { return (long long)hctm::jacobi_log_doubles(n, max_sweeps); }

}  // extern "C"

// ------------------------------------------------- no-allocation entry ----
// Device scratch of hctm_dev_jacobi_noalloc, for callers that cannot
// allocate: one file-scope array that every device the library runs on holds
// until the process ends.  In host code `scratch` only names the symbol; its
// device address is looked up once per device (with that device current)
// and only that address is ever handed to kernels.
namespace {
constexpr long long kStaticScratchDoubles = 4LL << 20;  // 32 MiB per device
__device__ __align__(256) double scratch[kStaticScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

double* static_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) throw hctm::Error(CTM_E_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) throw hctm::Error(CTM_E_ARG, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw hctm::Error(CTM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int hctm_dev_jacobi_noalloc(double* X, int m, int n, double tol, int max_sweeps, int pre, double* sv,
                                       int* perm, int* sweeps, double* V, void* stream) {
  return guarded(nullptr, [&] {
    if (m < 1 || n < 1 || n > 1024) throw hctm::Error(CTM_E_ARG, "size out of range");
    if (max_sweeps < 1) throw hctm::Error(CTM_E_ARG, "max_sweeps < 1");
    if (V && m != n) throw hctm::Error(CTM_E_ARG, "V needs a square X");
    // rotation log (with V) at the front, then the column-major copy of the
    // L2 kernel (blocks up to 256 x 256), each 256-byte aligned
    const long long log = V ? (((long long)hctm::jacobi_log_doubles(n, max_sweeps) + 31) / 32) * 32 : 0;
    const long long work = (m <= 256 && n <= 256) ? (long long)m * n : 0;
    if (log + work > kStaticScratchDoubles)
      throw hctm::Error(CTM_E_ARG, "hctm_dev_jacobi_noalloc: needs " + std::to_string(log + work) +
                                       " doubles of scratch, the static buffer holds " +
                                       std::to_string(kStaticScratchDoubles) + " (fewer sweeps or columns)");
    double* base = static_scratch();
    hctm::SmallProb p{};
    p.a = X;
    p.m = m;
    p.n = n;
    p.lda = n;
    p.rel = tol;
    p.max_sweeps = max_sweeps;
    p.pre = pre;
    p.info = sweeps;
    p.sv = sv;
    p.perm = perm;
    p.b = V;
    p.vlog = V ? base : nullptr;
    p.work = work ? base + log : nullptr;
    hctm::jacobi({p}, reinterpret_cast<hipStream_t>(stream));
  });
}
