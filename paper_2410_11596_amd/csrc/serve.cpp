// Serving of independent CTMRG solves on one GPU (include/hctm_serve.h).
//
// A fixed pool of max_active worker threads, each with its own HIP stream,
// runs the admitted solves, each on its own context with its workspace
// carved from one device pool, so that the host synchronisations inside a
// solve (the convergence tests of the truncated SVD, the kept counts) never
// hold up the others and their kernels overlap on the device.  Admission is
// first come, first served, by pool space and the cap on concurrent solves;
// an admitted solve waits in a queue for the next free worker.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "hctm.h"
#include "hctm_serve.h"

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct Request {
  long long id = 0;
  std::vector<double> A;
  std::vector<double> Aim;  // imaginary part of a complex tensor (empty: real)
  int d = 0, D = 0, chi = 0, form = 0, max_iter = 0;
  double tol = 0.0;
  size_t ws = 0;   // workspace bytes (ctm_workspace_size)
  size_t off = 0;  // its place in the pool
  bool done = false;
  bool claimed = false;  // a caller waits for it
  ctm_solve_info info{};
  std::vector<double> rho1, rho2h, rho2v;
  std::vector<double> rho1i, rho2hi, rho2vi;  // imaginary parts (complex tensors)
};

// First-fit allocator over the pool: free ranges by offset, merged on return.
class Pool {
 public:
  void reset(size_t n) {
    free_.clear();
    free_[0] = n;
  }
  bool take(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t o = it->first, rest = it->second - n;
      free_.erase(it);
      if (rest) free_[o + n] = rest;
      *off = o;
      return true;
    }
    return false;
  }
  void give(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

void set_message(ctm_solve_info& info, const std::string& m) {
  std::strncpy(info.message, m.c_str(), sizeof(info.message) - 1);
  info.message[sizeof(info.message) - 1] = '\0';
}

}  // namespace

struct ctm_server {
  int device = 0;
  char* pool_base = nullptr;
  size_t pool_bytes = 0;
  int max_active = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> waiting;
  std::map<long long, std::unique_ptr<Request>> all;
  std::deque<Request*> admitted;  // pool space taken, waiting for a worker
  int running = 0;                // admitted and not finished
  long long next_id = 1;
  Pool pool;
  std::vector<std::thread> workers;  // max_active of them, for the server's lifetime
  bool stopping = false;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // Start the oldest waiting solves while they fit (called with mu held).
  void admit_locked() {
    while (!waiting.empty() && running < max_active) {
      Request* r = waiting.front();
      size_t off = 0;
      if (!pool.take(round_up(r->ws), &off)) break;
      waiting.pop_front();
      r->off = off;
      r->info.t_start = now();
      ++running;
      admitted.push_back(r);
      cv.notify_all();
    }
  }

  // Worker: one HIP stream for its lifetime; takes admitted solves in order
  // until the server stops and nothing is left.
  void worker() {
    hipStream_t st = nullptr;
    const bool ok = hipSetDevice(device) == hipSuccess &&
                    hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    if (!ok) st = nullptr;
    for (;;) {
      Request* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [this] { return stopping || !admitted.empty(); });
        if (admitted.empty()) break;  // stopping and drained
        r = admitted.front();
        admitted.pop_front();
      }
      run(r, st);
    }
    if (st) (void)hipStreamDestroy(st);
  }

  void run(Request* r, hipStream_t st) {
    int rc = CTM_OK;
    std::string msg;
    ctm_ctx* c = nullptr;
    int it = 0, conv = 0;
    double delta = INFINITY;
    if (!st) {
      rc = CTM_E_HIP;
      msg = "the worker has no stream";
    }
    try {
      if (rc == CTM_OK) {
        ctm_opts o;
        ctm_opts_default(&o);
        o.form = r->form;
        o.stream = st;
        o.workspace = pool_base + r->off;
        o.workspace_bytes = r->ws;
        rc = r->Aim.empty() ? ctm_init(&c, r->A.data(), r->d, r->D, r->chi, &o)
                            : ctm_init_complex(&c, r->A.data(), r->Aim.data(), r->d, r->D, r->chi, &o);
        if (rc != CTM_OK) msg = ctm_last_error(nullptr);
      }
      while (rc == CTM_OK && it < r->max_iter) {
        rc = ctm_step(c, 1);
        if (rc != CTM_OK) break;
        ++it;
        rc = ctm_converged(c, r->tol, &conv, &delta);
        if (rc != CTM_OK || conv) break;
      }
      if (rc == CTM_OK) {
        const size_t d2 = (size_t)r->d * r->d;
        r->rho1.resize(d2);
        r->rho2h.resize(d2 * d2);
        r->rho2v.resize(d2 * d2);
        r->rho1i.assign(d2, 0.0);
        r->rho2hi.assign(d2 * d2, 0.0);
        r->rho2vi.assign(d2 * d2, 0.0);
        if (r->Aim.empty()) {
          rc = ctm_rdm_1site(c, 0, 0, r->rho1.data());
          if (rc == CTM_OK) rc = ctm_rdm_2site(c, 0, 0, 0, r->rho2h.data());
          if (rc == CTM_OK) rc = ctm_rdm_2site(c, 0, 0, 1, r->rho2v.data());
        } else {
          rc = ctm_rdm_1site_complex(c, 0, 0, r->rho1.data(), r->rho1i.data());
          if (rc == CTM_OK) rc = ctm_rdm_2site_complex(c, 0, 0, 0, r->rho2h.data(), r->rho2hi.data());
          if (rc == CTM_OK) rc = ctm_rdm_2site_complex(c, 0, 0, 1, r->rho2v.data(), r->rho2vi.data());
        }
      }
      if (rc != CTM_OK && c) msg = ctm_last_error(c);
    } catch (const std::exception& e) {
      rc = CTM_E_NOMEM;
      msg = std::string("host allocation failed: ") + e.what();
    }
    ctm_free(c);
    // nothing of this solve may still run when its pool space is reused
    if (st) (void)hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lk(mu);
    pool.give(r->off, round_up(r->ws));
    --running;
    r->info.status = rc;
    r->info.iterations = it;
    r->info.converged = conv;
    r->info.delta = delta;
    r->info.t_end = now();
    if (rc != CTM_OK) set_message(r->info, msg);
    r->done = true;
    admit_locked();
    cv.notify_all();
  }
};

extern "C" {

int ctm_server_create(ctm_server** out, size_t pool_bytes, int max_active) {
  if (!out) return CTM_E_ARG;
  *out = nullptr;
  if (pool_bytes == 0 || max_active < 1 || max_active > 64) return CTM_E_ARG;
  std::unique_ptr<ctm_server> s;
  try {
    s.reset(new ctm_server());
  } catch (const std::bad_alloc&) {
    return CTM_E_NOMEM;
  }
  if (hipGetDevice(&s->device) != hipSuccess) return CTM_E_HIP;
  void* p = nullptr;
  if (hipMalloc(&p, pool_bytes) != hipSuccess) return CTM_E_NOMEM;
  s->pool_base = static_cast<char*>(p);
  s->pool_bytes = pool_bytes;
  s->max_active = max_active;
  s->pool.reset(pool_bytes);
  try {
    for (int i = 0; i < max_active; ++i) s->workers.emplace_back(&ctm_server::worker, s.get());
  } catch (const std::exception&) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stopping = true;
    }
    s->cv.notify_all();
    for (std::thread& t : s->workers) t.join();
    (void)hipFree(s->pool_base);
    return CTM_E_NOMEM;
  }
  *out = s.release();
  return CTM_OK;
}

static int submit(ctm_server* s, const double* A, const double* Aim, int d, int D, int chi, int form, double tol,
                  int max_iter, long long* id) {
  if (!s || !A || !id) return CTM_E_ARG;
  if (form != CTM_FORM_Z2 && form != CTM_FORM_DENSE) return CTM_E_ARG;
  if (Aim && form != CTM_FORM_Z2) return CTM_E_ARG;
  if (Aim && d > 8) return CTM_E_ARG;
  if (!(tol > 0.0) || max_iter < 1) return CTM_E_ARG;
  ctm_opts o;
  ctm_opts_default(&o);
  o.form = form;
  size_t ws = 0;
  // checks d, D, chi
  const int rc = Aim ? ctm_workspace_size_complex(d, D, chi, &o, &ws) : ctm_workspace_size(d, D, chi, &o, &ws);
  if (rc != CTM_OK) return rc;
  if (round_up(ws) > s->pool_bytes) return CTM_E_NOMEM;
  try {
    std::unique_ptr<Request> r(new Request());
    const size_t n = (size_t)d * D * D * D * D;
    r->A.assign(A, A + n);
    for (double x : r->A)
      if (!std::isfinite(x)) return CTM_E_NUMERIC;
    if (Aim) {
      r->Aim.assign(Aim, Aim + n);
      for (double x : r->Aim)
        if (!std::isfinite(x)) return CTM_E_NUMERIC;
    }
    r->d = d;
    r->D = D;
    r->chi = chi;
    r->form = form;
    r->tol = tol;
    r->max_iter = max_iter;
    r->ws = ws;
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    r->info.t_submit = s->now();
    *id = r->id;
    Request* raw = r.get();
    s->all[r->id] = std::move(r);
    s->waiting.push_back(raw);
    s->admit_locked();
  } catch (const std::bad_alloc&) {
    return CTM_E_NOMEM;
  }
  return CTM_OK;
}

int ctm_server_submit(ctm_server* s, const double* A, int d, int D, int chi, int form, double tol, int max_iter,
                      long long* id) {
  return submit(s, A, nullptr, d, D, chi, form, tol, max_iter, id);
}

int ctm_server_submit_complex(ctm_server* s, const double* A_re, const double* A_im, int d, int D, int chi,
                              double tol, int max_iter, long long* id) {
  if (!A_im) return CTM_E_ARG;
  return submit(s, A_re, A_im, d, D, chi, CTM_FORM_Z2, tol, max_iter, id);
}

static int wait_for(ctm_server* s, long long id, double* rho1, double* rho2_h, double* rho2_v, double* rho1_im,
                    double* rho2_h_im, double* rho2_v_im, ctm_solve_info* info) {
  if (!s) return CTM_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return CTM_E_ARG;
  Request* r = it->second.get();
  if (r->claimed) return CTM_E_ARG;  // another caller waits for it
  r->claimed = true;
  s->cv.wait(lk, [r] { return r->done; });
  if (r->info.status == CTM_OK) {
    if (rho1) std::memcpy(rho1, r->rho1.data(), sizeof(double) * r->rho1.size());
    if (rho2_h) std::memcpy(rho2_h, r->rho2h.data(), sizeof(double) * r->rho2h.size());
    if (rho2_v) std::memcpy(rho2_v, r->rho2v.data(), sizeof(double) * r->rho2v.size());
    if (rho1_im) std::memcpy(rho1_im, r->rho1i.data(), sizeof(double) * r->rho1i.size());
    if (rho2_h_im) std::memcpy(rho2_h_im, r->rho2hi.data(), sizeof(double) * r->rho2hi.size());
    if (rho2_v_im) std::memcpy(rho2_v_im, r->rho2vi.data(), sizeof(double) * r->rho2vi.size());
  }
  if (info) *info = r->info;
  s->all.erase(it);
  return CTM_OK;
}

int ctm_server_wait(ctm_server* s, long long id, double* rho1, double* rho2_h, double* rho2_v,
                    ctm_solve_info* info) {
  return wait_for(s, id, rho1, rho2_h, rho2_v, nullptr, nullptr, nullptr, info);
}

int ctm_server_wait_complex(ctm_server* s, long long id, double* rho1_re, double* rho1_im, double* rho2_h_re,
                            double* rho2_h_im, double* rho2_v_re, double* rho2_v_im, ctm_solve_info* info) {
  return wait_for(s, id, rho1_re, rho2_h_re, rho2_v_re, rho1_im, rho2_h_im, rho2_v_im, info);
}

int ctm_server_load(ctm_server* s, int* waiting, int* running) {
  if (!s) return CTM_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (waiting) *waiting = (int)s->waiting.size();
  if (running) *running = s->running;
  return CTM_OK;
}

void ctm_server_destroy(ctm_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [s] { return s->waiting.empty() && s->running == 0; });
    s->stopping = true;
  }
  s->cv.notify_all();
  for (std::thread& t : s->workers)
    if (t.joinable()) t.join();
  if (s->pool_base) (void)hipFree(s->pool_base);
  delete s;
}

}  // extern "C"
