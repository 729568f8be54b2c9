// extern "C" entry points declared in include/mcsvt.h.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <functional>
#include <thread>
#include <utility>
#include <vector>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "solver.hpp"

struct mc_svt {
  std::unique_ptr<mcsvt::Solver> solver;
  std::string err;
};

struct mc_rsvd {
  std::unique_ptr<mcsvt::Solver> solver;
  std::string err;
};

namespace mcsvt {

namespace {
mc_alloc_fn g_alloc = nullptr;
mc_free_fn g_free = nullptr;
void* g_ctx = nullptr;
std::mutex g_alloc_mu;
thread_local std::string t_err;
}  // namespace

[[noreturn]] void throw_hip(hipError_t e, const char* expr, const char* file,
                            int line) {
  char buf[512];
  std::snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s at %s:%d", (int)e,
                hipGetErrorString(e), expr, file, line);
  throw Error(e == hipErrorOutOfMemory ? kENOMEM : kEDEVICE, buf);
}

void* dev_alloc(size_t bytes, hipStream_t stream) {
  mc_alloc_fn fa;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    fa = g_alloc;
    ctx = g_ctx;
  }
  void* p = nullptr;
  if (fa) {
    p = fa(bytes, (void*)stream, ctx);
    if (!p) throw Error(kENOMEM, "allocator hook returned NULL");
    return p;
  }
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(kENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed (" +
                             hipGetErrorString(e) + ")");
  }
  return p;
}

void dev_free(void* p, size_t bytes, hipStream_t stream) {
  mc_free_fn ff;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    ff = g_free;
    ctx = g_ctx;
  }
  if (ff) {
    ff(p, bytes, (void*)stream, ctx);
    return;
  }
  // frees must not race with queued kernels that still read the buffer
  (void)hipStreamSynchronize(stream);
  (void)hipFree(p);
}

}  // namespace mcsvt

void mcsvt_set_thread_error(const char* msg) { mcsvt::t_err = msg ? msg : ""; }

namespace {

// runs f; a failure's message goes to the handle (H has a std::string err),
// or to the calling thread when h is NULL
template <class H, class F>
mc_status guarded_on(H* h, F&& f) {
  try {
    f();
    return MC_OK;
  } catch (const mcsvt::Error& e) {
    (h ? h->err : mcsvt::t_err) = e.what();
    return (mc_status)e.status;
  } catch (const std::bad_alloc&) {
    (h ? h->err : mcsvt::t_err) = "host allocation failed";
    return MC_ENOMEM;
  } catch (const std::exception& e) {
    (h ? h->err : mcsvt::t_err) = e.what();
    return MC_EDEVICE;
  }
}

template <class F>
mc_status guarded(mc_svt_t h, F&& f) {
  return guarded_on(h, std::forward<F>(f));
}

void set_profile(mcsvt::Solver& s, int32_t on) {
  auto& p = s.prof;
  p.collect();
  if (on) p.reset();
  p.on = on != 0;
}

void get_profile(mcsvt::Solver& s, mc_prof_entry* out) {
  auto& p = s.prof;
  p.collect();
  for (int f = 0; f < MC_PROF_FAMILIES; ++f) {
    out[f].launches = p.count[f];
    out[f].ms = p.ms[f];
    out[f].bytes = p.bytes[f];
    out[f].flops = p.flops[f];
  }
}

void fill_info(const mcsvt::StepInfo& s, mc_svt_step_info* o) {
  if (!o) return;
  o->i = s.i;
  o->r = s.r;
  o->k = s.k;
  o->p = s.p;
  o->fresh = s.fresh;
  o->recycled = s.recycled;
  o->rejected = s.rejected;
  o->converged = s.converged;
  o->res = s.res;
  o->sigma_max = s.sigma_max;
}

void fill_result(const mcsvt::Solver& s, mc_svt_result* o) {
  o->iters = s.iters();
  o->rank = s.rank();
  o->converged = s.converged() ? 1 : 0;
  o->fresh = s.fresh_total();
  o->recycled = s.recycled_total();
  o->rejected = s.rejected_total();
  o->res = s.last_res();
  o->c = s.c();
  o->norm2 = s.norm2();
  o->mnorm = s.mnorm();
  o->shifts = s.shifts_seen();
  o->redone = s.redone_total();
}

// COO rows from either COO row ids or a CSR row pointer (host).
std::vector<int64_t> coo_rows(int64_t m, int64_t nnz, const int64_t* rows,
                              int32_t is_csr) {
  std::vector<int64_t> out;
  if (!is_csr) return out;
  MC_REQUIRE(rows[0] == 0 && rows[m] == nnz, mcsvt::kEINVAL,
             "CSR row pointer must start at 0 and end at nnz");
  out.resize(nnz);
  for (int64_t i = 0; i < m; ++i) {
    MC_REQUIRE(rows[i] <= rows[i + 1], mcsvt::kEINVAL,
               "CSR row pointer must be non-decreasing");
    for (int64_t e = rows[i]; e < rows[i + 1]; ++e) out[e] = i;
  }
  return out;
}

void check_sizes(int64_t m, int64_t n, int64_t nnz) {
  MC_REQUIRE(m >= 1 && n >= 1, mcsvt::kEINVAL, "m and n must be >= 1");
  MC_REQUIRE(m < (int64_t)1 << 31 && n < (int64_t)1 << 31, mcsvt::kEINVAL,
             "m and n must be < 2^31");
  MC_REQUIRE(nnz >= 1, mcsvt::kEINVAL, "nnz must be >= 1");
  MC_REQUIRE(nnz < ((int64_t)1 << 31) - 1, mcsvt::kEINVAL, "nnz must be < 2^31 - 1");
  MC_REQUIRE((double)nnz <= (double)m * (double)n, mcsvt::kEDUP,
             "nnz exceeds m*n: cells must repeat");
}

}  // namespace

extern "C" {

int32_t mc_abi_version(void) { return MCSVT_ABI_VERSION; }

mc_status mc_set_allocator(mc_alloc_fn alloc, mc_free_fn release, void* ctx) {
  if ((alloc == nullptr) != (release == nullptr)) {
    mcsvt::t_err = "alloc and release hooks must both be set or both be NULL";
    return MC_EINVAL;
  }
  std::lock_guard<std::mutex> lk(mcsvt::g_alloc_mu);
  mcsvt::g_alloc = alloc;
  mcsvt::g_free = release;
  mcsvt::g_ctx = ctx;
  return MC_OK;
}

void mc_svt_default_params(mc_svt_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tau = 0.0;
  p->delta = 0.0;
  p->eps = 1e-4;
  p->ritz_tol = 1e-4;
  p->c = 0.0;
  p->i_max = 200;
  p->l = 5;
  p->s = 10;
  p->p_init = 3;
  p->p_min = 1;
  p->p_max = 8;
  p->adaptive_p = 1;
  p->i_reuse = 0;
  p->q_reuse = 10;
  p->recycle = 0;
  p->k_max = 0;
  p->precision = MC_FP64;
  p->use_graphs = 1;
  p->seed = 12345;
}

size_t mc_svt_footprint(int64_t m, int64_t n, int64_t nnz, const mc_svt_params* p) {
  mc_svt_params q;
  if (p) q = *p; else mc_svt_default_params(&q);
  if (m < 1 || n < 1 || nnz < 1) return 0;
  return mcsvt::footprint_bytes(m, n, nnz, q);
}

mc_status mc_svt_init(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                      const int32_t* cols, const double* vals, int32_t is_csr,
                      const mc_svt_params* params, void* stream, mc_svt_t* out) {
  if (out) *out = nullptr;
  mc_svt* h = nullptr;
  mc_status st = guarded(nullptr, [&] {
    MC_REQUIRE(out && rows && cols && vals, mcsvt::kEINVAL, "NULL argument");
    check_sizes(m, n, nnz);
    for (int64_t e = 0; e < nnz; ++e)
      MC_REQUIRE(std::isfinite(vals[e]), mcsvt::kEINVAL, "non-finite value in M_Phi");
    mc_svt_params prm;
    if (params) prm = *params; else mc_svt_default_params(&prm);
    std::vector<int64_t> expanded = coo_rows(m, nnz, rows, is_csr);
    const int64_t* r = is_csr ? expanded.data() : rows;
    h = new mc_svt();
    h->solver = mcsvt::make_solver(m, n, nnz, prm, (hipStream_t)stream);
    const int s = h->solver->init(r, cols, vals, true);
    if (s == mcsvt::kERANGE) throw mcsvt::Error(s, "index out of range");
    if (s == mcsvt::kEDUP) throw mcsvt::Error(s, "duplicate cell in Phi");
    if (s != mcsvt::kOK) throw mcsvt::Error(s, "invalid input");
  });
  if (st != MC_OK) {
    delete h;
    return st;
  }
  *out = h;
  return MC_OK;
}

mc_status mc_svt_init_dev(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                          const int32_t* cols, const double* vals, int32_t is_csr,
                          const mc_svt_params* params, void* stream, mc_svt_t* out) {
  if (out) *out = nullptr;
  mc_svt* h = nullptr;
  mc_status st = guarded(nullptr, [&] {
    MC_REQUIRE(out && rows && cols && vals, mcsvt::kEINVAL, "NULL argument");
    check_sizes(m, n, nnz);
    mc_svt_params prm;
    if (params) prm = *params; else mc_svt_default_params(&prm);
    h = new mc_svt();
    h->solver = mcsvt::make_solver(m, n, nnz, prm, (hipStream_t)stream);
    mcsvt::DevBuf<int64_t> expanded;
    const int64_t* r = rows;
    if (is_csr) {
      expanded.reserve(nnz, (hipStream_t)stream);
      if (mcsvt::csr_rows_device(m, nnz, rows, expanded.p, (hipStream_t)stream) != mcsvt::kOK)
        throw mcsvt::Error(mcsvt::kEINVAL,
                           "CSR row pointer must start at 0, end at nnz and not decrease");
      r = expanded.p;
    }
    const int s = h->solver->init(r, cols, vals, true, true);
    if (s == mcsvt::kERANGE) throw mcsvt::Error(s, "index out of range");
    if (s == mcsvt::kEDUP) throw mcsvt::Error(s, "duplicate cell in Phi");
    if (s != mcsvt::kOK) throw mcsvt::Error(s, "invalid input (a non-finite value?)");
  });
  if (st != MC_OK) {
    delete h;
    return st;
  }
  *out = h;
  return MC_OK;
}

mc_status mc_svt_step(mc_svt_t h, mc_svt_step_info* info) {
  if (!h || !h->solver) {
    mcsvt::t_err = "NULL handle";
    return MC_EINVAL;
  }
  return guarded(h, [&] { fill_info(h->solver->step(), info); });
}

namespace {

// Fixed pool of host worker threads for mc_svt_step_many: each handle's step
// (its host control and device round trips) runs on one worker, so a solve
// waiting on its stream never holds back the others.
class StepPool {
 public:
  static StepPool& get() {
    static StepPool pool;
    return pool;
  }
  // run f(0) .. f(n-1) on the workers (and the calling thread); returns when
  // all are done
  void run(int n, const std::function<void(int)>& f) {
    std::unique_lock<std::mutex> lk(m_);
    job_ = &f;
    next_ = 0;
    total_ = n;
    left_ = n;
    ++gen_;
    cv_.notify_all();
    lk.unlock();
    work();
    lk.lock();
    done_cv_.wait(lk, [&] { return left_ == 0; });
    job_ = nullptr;
  }

 private:
  StepPool() {
    const unsigned hw = std::max(2u, std::min(16u, std::thread::hardware_concurrency()));
    for (unsigned t = 0; t + 1 < hw; ++t)
      threads_.emplace_back([this] { loop(); });
  }
  ~StepPool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }
  void work() {
    while (true) {
      int i;
      const std::function<void(int)>* f;
      {
        std::lock_guard<std::mutex> lk(m_);
        if (!job_ || next_ >= total_) return;
        i = next_++;
        f = job_;
      }
      (*f)(i);
      std::lock_guard<std::mutex> lk(m_);
      if (--left_ == 0) done_cv_.notify_all();
    }
  }
  void loop() {
    uint64_t seen = 0;
    while (true) {
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
      }
      work();
    }
  }
  std::mutex m_;
  std::condition_variable cv_, done_cv_;
  std::vector<std::thread> threads_;
  const std::function<void(int)>* job_ = nullptr;
  int next_ = 0, total_ = 0, left_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

}  // namespace

mc_status mc_svt_step_many(mc_svt_t* hs, int32_t count, mc_svt_step_info* info,
                           mc_status* status) {
  if (!hs || count < 0) {
    mcsvt::t_err = "bad handle array";
    return MC_EINVAL;
  }
  std::vector<mc_status> st(count, MC_OK);
  // the device of the calling thread, made current on every worker
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto one = [&](int j) {
    if (!hs[j] || !hs[j]->solver) {
      st[j] = MC_EINVAL;
      return;
    }
    if (hs[j]->solver->converged()) {
      st[j] = MC_EDONE;
      return;
    }
    (void)hipSetDevice(dev);
    st[j] = guarded(hs[j], [&] {
      const mcsvt::StepInfo r = hs[j]->solver->step();
      fill_info(r, info ? &info[j] : nullptr);
    });
  };
  if (count == 1) {
    one(0);
  } else if (count > 1) {
    StepPool::get().run(count, one);
  }
  mc_status worst = MC_OK;
  for (int32_t j = 0; j < count; ++j) {
    if (status) status[j] = st[j];
    if (st[j] != MC_OK && st[j] != MC_EDONE && worst == MC_OK) worst = st[j];
  }
  return worst;
}

mc_status mc_svt_step_group(mc_svt_t* hs, int32_t count, mc_svt_step_info* info,
                            mc_status* status) {
  if (!hs || count < 0) {
    mcsvt::t_err = "bad handle array";
    return MC_EINVAL;
  }
  std::vector<mc_status> st(count, MC_OK);
  std::vector<mcsvt::Solver*> live;
  std::vector<int32_t> at;
  for (int32_t j = 0; j < count; ++j) {
    if (!hs[j] || !hs[j]->solver) {
      st[j] = MC_EINVAL;
    } else if (hs[j]->solver->converged()) {
      st[j] = MC_EDONE;
    } else if (hs[j]->solver->step_busy()) {
      st[j] = MC_EINVAL;
      hs[j]->err = "a step of this solve is in progress";
    } else {
      live.push_back(hs[j]->solver.get());
      at.push_back(j);
    }
  }
  std::vector<int> sst(live.size(), MC_OK);
  std::vector<std::string> serr(live.size());
  const mc_status all = guarded(nullptr, [&] { mcsvt::step_group(live, sst, serr); });
  for (size_t i = 0; i < live.size(); ++i) {
    const int32_t j = at[i];
    if (all != MC_OK) {
      st[j] = all;
      hs[j]->err = mcsvt::t_err;
    } else if (sst[i] != MC_OK) {
      st[j] = (mc_status)sst[i];
      hs[j]->err = serr[i];
    } else {
      fill_info(live[i]->step_result(), info ? &info[j] : nullptr);
    }
  }
  mc_status worst = MC_OK;
  for (int32_t j = 0; j < count; ++j) {
    if (status) status[j] = st[j];
    if (st[j] != MC_OK && st[j] != MC_EDONE && worst == MC_OK) worst = st[j];
  }
  return worst;
}

mc_status mc_svt_solve(mc_svt_t h, mc_svt_result* out) {
  if (!h || !h->solver) {
    mcsvt::t_err = "NULL handle";
    return MC_EINVAL;
  }
  mc_status st = guarded(h, [&] {
    auto& s = *h->solver;
    while (!s.converged() && s.iters() < s.params().i_max) s.step();
  });
  if (st != MC_OK) return st;
  if (out) fill_result(*h->solver, out);
  return h->solver->converged() ? MC_OK : MC_ENOTCONV;
}

mc_status mc_svt_get_result(mc_svt_t h, mc_svt_result* out) {
  if (!h || !h->solver || !out) {
    mcsvt::t_err = "NULL argument";
    return MC_EINVAL;
  }
  fill_result(*h->solver, out);
  return MC_OK;
}

mc_status mc_svt_get_factors(mc_svt_t h, double* U, double* sig, double* V,
                             int64_t ldu, int64_t ldv, int32_t r_cap, int32_t* r) {
  if (!h || !h->solver) {
    mcsvt::t_err = "NULL handle";
    return MC_EINVAL;
  }
  return guarded(h, [&] {
    auto& s = *h->solver;
    const int rk = s.rank();
    if (r) *r = rk;
    MC_REQUIRE(rk <= r_cap, mcsvt::kEINVAL, "r_cap smaller than the rank");
    MC_REQUIRE(ldu >= rk && ldv >= rk, mcsvt::kEINVAL, "leading dimension too small");
    s.get_factors(U, sig, V, ldu, ldv);
  });
}

mc_status mc_svt_get_observed(mc_svt_t h, double* x_phi) {
  if (!h || !h->solver || !x_phi) {
    mcsvt::t_err = "NULL argument";
    return MC_EINVAL;
  }
  return guarded(h, [&] { h->solver->get_observed(x_phi); });
}

mc_status mc_svt_get_y(mc_svt_t h, double* y) {
  if (!h || !h->solver || !y) {
    mcsvt::t_err = "NULL argument";
    return MC_EINVAL;
  }
  return guarded(h, [&] { h->solver->get_y(y); });
}

mc_status mc_svt_get_sigma(mc_svt_t h, double* S, int32_t k_cap, int32_t* k) {
  if (!h || !h->solver) {
    mcsvt::t_err = "NULL handle";
    return MC_EINVAL;
  }
  return guarded(h, [&] {
    const auto& v = h->solver->last_sigma();
    if (k) *k = (int32_t)v.size();
    MC_REQUIRE((int64_t)v.size() <= k_cap, mcsvt::kEINVAL, "k_cap too small");
    for (size_t j = 0; j < v.size(); ++j) S[j] = v[j];
  });
}

mc_status mc_svt_profile(mc_svt_t h, int32_t on) {
  if (!h || !h->solver) {
    mcsvt::t_err = "NULL handle";
    return MC_EINVAL;
  }
  return guarded(h, [&] { set_profile(*h->solver, on); });
}

mc_status mc_svt_get_profile(mc_svt_t h, mc_prof_entry* out, int32_t cap) {
  if (!h || !h->solver || !out || cap < MC_PROF_FAMILIES) {
    mcsvt::t_err = "bad arguments";
    return MC_EINVAL;
  }
  return guarded(h, [&] { get_profile(*h->solver, out); });
}

mc_status mc_svt_destroy(mc_svt_t h) {
  if (!h) return MC_OK;
  mc_status st = guarded(nullptr, [&] { h->solver.reset(); });
  delete h;
  return st;
}

const char* mc_svt_last_error(mc_svt_t h) {
  if (h) return h->err.c_str();
  return mcsvt::t_err.c_str();
}

namespace {

// a solver holding A = (rows, cols, vals) unscaled, for truncated SVDs
std::unique_ptr<mcsvt::Solver> make_rsvd_solver(int64_t m, int64_t n, int64_t nnz,
                                                const int64_t* rows, const int32_t* cols,
                                                const double* vals, int32_t s,
                                                int32_t precision, uint64_t seed,
                                                hipStream_t stream) {
  MC_REQUIRE(rows && cols && vals, mcsvt::kEINVAL, "NULL argument");
  check_sizes(m, n, nnz);
  MC_REQUIRE(s >= 0, mcsvt::kEINVAL, "need s >= 0");
  MC_REQUIRE(precision >= MC_FP64 && precision <= MC_BF16_EIG64, mcsvt::kEINVAL,
             "unknown precision");
  for (int64_t e = 0; e < nnz; ++e)
    MC_REQUIRE(std::isfinite(vals[e]), mcsvt::kEINVAL, "non-finite value");
  mc_svt_params prm;
  mc_svt_default_params(&prm);
  prm.s = s;
  prm.seed = seed;
  prm.precision = (mc_precision)precision;
  auto holder = mcsvt::make_solver(m, n, nnz, prm, stream);
  const int st = holder->init(rows, cols, vals, false);
  if (st == mcsvt::kERANGE) throw mcsvt::Error(st, "index out of range");
  if (st == mcsvt::kEDUP) throw mcsvt::Error(st, "duplicate cell");
  if (st != mcsvt::kOK) throw mcsvt::Error(st, "invalid input");
  return holder;
}

void check_rsvd_shape(int64_t m, int64_t n, int32_t method, int32_t k, int32_t s,
                      int32_t p) {
  MC_REQUIRE(method == MC_RSVD_PI || method == MC_RSVD_BKI, mcsvt::kEINVAL,
             "unknown method (MC_RSVD_PI or MC_RSVD_BKI)");
  MC_REQUIRE(k >= 1 && s >= 0 && p >= 0, mcsvt::kEINVAL, "need k >= 1, s >= 0, p >= 0");
  const int64_t mn = std::min(m, n);
  if (method == MC_RSVD_BKI)
    MC_REQUIRE((int64_t)(p + 1) * (k + s) <= mn, mcsvt::kEINVAL,
               "(p+1)(k+s) must not exceed min(m, n)");
  else
    MC_REQUIRE((int64_t)k + s <= mn, mcsvt::kEINVAL, "k+s must not exceed min(m, n)");
}

void run_rsvd(mcsvt::Solver& solver, int32_t method, int32_t k, int32_t p,
              uint32_t step, uint32_t attempt, double* U, double* S, double* V) {
  if (method == MC_RSVD_PI)
    solver.rsvd_pi(k, p, step, attempt);
  else
    solver.rsvd(k, p, step, attempt);
  solver.get_rsvd(U, S, V);
}

mc_status one_shot(int32_t method, int64_t m, int64_t n, int64_t nnz,
                   const int64_t* rows, const int32_t* cols, const double* vals,
                   int32_t k, int32_t s, int32_t p, uint64_t seed, uint32_t step,
                   uint32_t attempt, int32_t precision, void* stream, double* U,
                   double* S, double* V) {
  return guarded(nullptr, [&] {
    MC_REQUIRE(U && S && V, mcsvt::kEINVAL, "NULL argument");
    check_sizes(m, n, nnz);
    check_rsvd_shape(m, n, method, k, s, p);
    auto solver = make_rsvd_solver(m, n, nnz, rows, cols, vals, s, precision, seed,
                                   (hipStream_t)stream);
    run_rsvd(*solver, method, k, p, step, attempt, U, S, V);
  });
}

}  // namespace

mc_status mc_rsvd_bki(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                      const int32_t* cols, const double* vals, int32_t k,
                      int32_t s, int32_t p, uint64_t seed, uint32_t step,
                      uint32_t attempt, int32_t precision, void* stream,
                      double* U, double* S, double* V) {
  return one_shot(MC_RSVD_BKI, m, n, nnz, rows, cols, vals, k, s, p, seed, step,
                  attempt, precision, stream, U, S, V);
}

mc_status mc_rsvd_pi(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                     const int32_t* cols, const double* vals, int32_t k,
                     int32_t s, int32_t p, uint64_t seed, uint32_t step,
                     uint32_t attempt, int32_t precision, void* stream,
                     double* U, double* S, double* V) {
  return one_shot(MC_RSVD_PI, m, n, nnz, rows, cols, vals, k, s, p, seed, step,
                  attempt, precision, stream, U, S, V);
}

mc_status mc_rsvd_init(int64_t m, int64_t n, int64_t nnz, const int64_t* rows,
                       const int32_t* cols, const double* vals, int32_t s,
                       int32_t precision, uint64_t seed, void* stream,
                       mc_rsvd_t* out) {
  if (!out) {
    mcsvt::t_err = "NULL handle pointer";
    return MC_EINVAL;
  }
  *out = nullptr;
  return guarded(nullptr, [&] {
    auto solver = make_rsvd_solver(m, n, nnz, rows, cols, vals, s, precision, seed,
                                   (hipStream_t)stream);
    auto h = std::make_unique<mc_rsvd>();
    h->solver = std::move(solver);
    *out = h.release();
  });
}

mc_status mc_rsvd_run(mc_rsvd_t h, int32_t method, int32_t k, int32_t p, uint32_t step,
                      uint32_t attempt, double* U, double* S, double* V) {
  if (!h || !h->solver || !S) {
    mcsvt::t_err = "NULL handle or S";
    return MC_EINVAL;
  }
  return guarded_on(h, [&] {
    mcsvt::Solver& solver = *h->solver;
    check_rsvd_shape(solver.m(), solver.n(), method, k, solver.params().s, p);
    run_rsvd(solver, method, k, p, step, attempt, U, S, V);
  });
}

mc_status mc_rsvd_profile(mc_rsvd_t h, int32_t on) {
  if (!h || !h->solver) {
    mcsvt::t_err = "NULL handle";
    return MC_EINVAL;
  }
  return guarded_on(h, [&] { set_profile(*h->solver, on); });
}

mc_status mc_rsvd_get_profile(mc_rsvd_t h, mc_prof_entry* out, int32_t cap) {
  if (!h || !h->solver || !out || cap < MC_PROF_FAMILIES) {
    mcsvt::t_err = "bad arguments";
    return MC_EINVAL;
  }
  return guarded_on(h, [&] { get_profile(*h->solver, out); });
}

mc_status mc_rsvd_destroy(mc_rsvd_t h) {
  if (!h) return MC_OK;
  mc_status st = guarded(nullptr, [&] { h->solver.reset(); });
  delete h;
  return st;
}

const char* mc_rsvd_last_error(mc_rsvd_t h) {
  if (h) return h->err.c_str();
  return mcsvt::t_err.c_str();
}

}  // extern "C"
