// Fast SVT (Alg. 6) control, driven from the host.
//
// One step:
//   k = r + 1; adjust p (Sec. IV.C)
//   repeat
//     fresh rSVD-BKI (Alg. 5) when i < i_reuse, q == q_reuse or there is no
//     usable basis; otherwise recycle the last call's Q (strategy 1) or U
//     (strategy 2) (Sec. IV.B), optionally checked by the Ritz residual (a
//     rejected recycle in step i also makes the rest of step i and the next
//     q_reuse * 2^(s-1) steps fresh, s = rejections since the last accepted
//     recycle)
//   until the k-th singular value <= tau (k += l otherwise)
//   r = #{S_j > tau}; fused SDDMM: residual on Phi and Y += delta P_Phi(M - X)
// The device work of these calls lives in solver_impl.hip.
#include "solver.hpp"

#include <chrono>
#include <cmath>
#include <cstring>

namespace mcsvt {

Profiler::~Profiler() {
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

hipEvent_t Profiler::ev() {
  if (used == pool.size()) {
    hipEvent_t e;
    MC_HIP(hipEventCreate(&e));
    pool.push_back(e);
  }
  return pool[used++];
}

void Profiler::begin(int fam, double b, double f, hipStream_t st) {
  if (!on) return;
  Rec r{fam, b, f, ev(), nullptr};
  MC_HIP(hipEventRecord(r.a, st));
  recs.push_back(r);
}

void Profiler::end(hipStream_t st) {
  if (!on) return;
  Rec& r = recs.back();
  r.b = ev();
  MC_HIP(hipEventRecord(r.b, st));
}

void Profiler::collect() {
  for (Rec& r : recs) {
    MC_HIP(hipEventSynchronize(r.b));
    float t = 0.f;
    MC_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.fam] += t;
    bytes[r.fam] += r.bytes;
    flops[r.fam] += r.flops;
    count[r.fam] += 1;
  }
  recs.clear();
  used = 0;
}

void Profiler::reset() {
  recs.clear();
  used = 0;
  for (int f = 0; f < kProfCount; ++f) ms[f] = bytes[f] = flops[f] = 0, count[f] = 0;
}

void resolve_params(int64_t m, int64_t n, int64_t nnz, mc_svt_params& p) {
  if (!(p.tau > 0)) p.tau = 5.0 * (double)n;
  if (!(p.delta > 0)) p.delta = 1.2 * (double)m * (double)n / (double)nnz;
  MC_REQUIRE(std::isfinite(p.tau) && std::isfinite(p.delta), kEINVAL,
             "tau and delta must be finite");
  MC_REQUIRE(p.eps > 0 && std::isfinite(p.eps), kEINVAL, "eps must be > 0");
  MC_REQUIRE(p.i_max >= 1, kEINVAL, "i_max must be >= 1");
  MC_REQUIRE(p.l >= 1, kEINVAL, "l must be >= 1");
  MC_REQUIRE(p.s >= 0 && p.s <= 4096, kEINVAL, "s out of range");
  MC_REQUIRE(p.p_min >= 0 && p.p_min <= p.p_max && p.p_max <= 64 &&
                 p.p_init >= p.p_min && p.p_init <= p.p_max,
             kEINVAL, "need 0 <= p_min <= p_init <= p_max <= 64");
  MC_REQUIRE(p.recycle >= 0 && p.recycle <= 2, kEINVAL, "recycle must be 0, 1 or 2");
  MC_REQUIRE(p.q_reuse >= 0 && p.i_reuse >= 0, kEINVAL, "i_reuse, q_reuse >= 0");
  MC_REQUIRE(p.k_max >= 0, kEINVAL, "k_max must be >= 0");
  MC_REQUIRE(p.ritz_tol >= 0, kEINVAL, "ritz_tol must be >= 0");
  MC_REQUIRE(p.precision >= 0 && p.precision <= 2, kEINVAL, "bad precision");
}

Solver::Solver(int64_t m, int64_t n, int64_t nnz, const mc_svt_params& prm,
               hipStream_t st)
    : m_(m), n_(n), nnz_(nnz), prm_(prm), st_(st) {
  resolve_params(m, n, nnz, prm_);
  kcap_ = (int)std::min<int64_t>(m, n);
  if (prm_.k_max > 0) kcap_ = std::min(kcap_, prm_.k_max);
  p_ = prm_.p_init;
  solve_dims(m, n, prm_, lim_k_, lim_b_, lim_L_);
}

Solver::~Solver() {
  if (done_ev_) (void)hipEventDestroy(done_ev_);
}

void Solver::widths(int k, int p, int& b, int& p_eff) const {
  const int64_t mn = std::min(m_, n_);
  b = (int)std::min<int64_t>((int64_t)k + prm_.s, mn);
  // rSVD-BKI stacks p + 1 blocks and needs (p + 1) b <= min(m, n); rSVD-PI
  // keeps one block whatever p is
  p_eff = power_ ? std::max(0, p)
                 : (int)std::max<int64_t>(0, std::min<int64_t>(p, mn / b - 1));
}

void Solver::mark() {
  if (!done_ev_) MC_HIP(hipEventCreateWithFlags(&done_ev_, hipEventDisableTiming));
  MC_HIP(hipEventRecord(done_ev_, st_));
}

// Short waits (a step's read-backs, tens to hundreds of microseconds) poll
// the event; a blocked wait can add the wake-up latency of the host thread
// to every step.  Waits longer than 0.5 ms block.
void Solver::wait() {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t e = hipEventQuery(done_ev_);
    if (e == hipSuccess) return;
    if (e != hipErrorNotReady) MC_HIP(e);
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(500)) break;
  }
  MC_HIP(hipEventSynchronize(done_ev_));
}

void Solver::fresh_svd(int k, int p, uint32_t step_id, uint32_t attempt) {
  fresh_launch(k, p, step_id, attempt, false);
  mark();
  wait();
  if (!fresh_finish(k)) {
    ++redone_total_;
    fresh_launch(k, p, step_id, attempt, true);
    mark();
    wait();
    fresh_finish(k);
  }
}

double Solver::sddmm(int r) {
  sddmm_launch(r);
  mark();
  wait();
  return sddmm_finish();
}

// Enqueue the next SVD call of the rank search: recycled when the gate of
// Alg. 6 allows it (Sec. IV.B), fresh otherwise.
void Solver::launch_svd(bool force_fresh) {
  const int k = k_cur_;
  // after a rejected recycle: the rest of that step and a pause that doubles
  // with each further rejection before a recycled result is accepted
  const int64_t pause = rej_run_ > 0 ? (int64_t)prm_.q_reuse << std::min(rej_run_ - 1, 20) : 0;
  const bool suspended = rej_i_ > 0 && i_ >= rej_i_ && i_ <= rej_i_ + pause;
  const bool fresh = force_fresh || prm_.recycle == 0 || i_ < prm_.i_reuse ||
                     q_ == prm_.q_reuse || basis_cols_ == 0 || k > basis_cols_ ||
                     suspended;
  if (fresh) {
    last_attempt_ = attempt_++;
    ++cur_.fresh;
  } else {
    ++q_;
    ++cur_.recycled;
  }
  cur_recycled_ = !fresh;
  if (defer_) {
    defer_svd(fresh, k, p_, (uint32_t)i_, last_attempt_, false);
    return;
  }
  if (fresh)
    fresh_launch(k, p_, (uint32_t)i_, last_attempt_, false);
  else
    recycled_launch(k);
  mark();
  phase_ = kSvd;
}

void Solver::defer_svd(bool fresh, int k, int p, uint32_t step, uint32_t attempt,
                       bool guarded) {
  pend_.fresh = fresh;
  pend_.guarded = guarded;
  pend_.k = k;
  pend_.p = p;
  pend_.step = step;
  pend_.attempt = attempt;
  phase_ = kSvdPending;
}

void Solver::launch_pending() {
  MC_REQUIRE(phase_ == kSvdPending, kEINVAL, "no pending SVD call");
  if (pend_.fresh)
    fresh_launch(pend_.k, pend_.p, pend_.step, pend_.attempt, pend_.guarded);
  else
    recycled_launch(pend_.k);
  mark();
  phase_ = kSvd;
}

void Solver::fresh_group_begin() {
  MC_REQUIRE(phase_ == kSvdPending && pend_.fresh, kEINVAL, "no pending fresh call");
  fresh_begin(pend_.k, pend_.p, pend_.step, pend_.attempt, pend_.guarded);
}

void Solver::fresh_group_end() {
  fresh_end();
  mark();
  phase_ = kSvd;
}

void Solver::step_begin() {
  MC_REQUIRE(!converged_, kEDONE, "the solve has already converged");
  MC_REQUIRE(phase_ == kIdle, kEINVAL, "a step of this solve is in progress");
  cur_ = StepInfo();
  ++i_;
  k_cur_ = std::min(r_ + 1, kcap_);
  if (prm_.adaptive_p && err_hist_.size() >= 2) {           // Sec. IV.C
    const size_t h = err_hist_.size();
    if (err_hist_[h - 1] > err_hist_[h - 2]) {
      ++p_;
      streak_ = 0;
    } else if (++streak_ == 10) {
      --p_;
      streak_ = 0;
    }
    p_ = std::min(std::max(p_, prm_.p_min), prm_.p_max);
  }
  attempt_ = 0;
  try {
    launch_svd(false);
  } catch (...) {
    phase_ = kIdle;
    throw;
  }
}

bool Solver::step_poll(bool block) {
  if (phase_ == kIdle) return true;
  if (phase_ == kSvdPending) return false;           // waits for its driver
  if (block) {
    wait();
  } else {
    const hipError_t e = hipEventQuery(done_ev_);
    if (e == hipErrorNotReady) return false;
    MC_HIP(e);
  }
  try {
    if (phase_ == kSvd) {
      if (cur_recycled_) {
        const double ratio = recycled_finish(k_cur_);
        if (prm_.ritz_tol > 0 && ratio > prm_.ritz_tol) {    // guard: redo fresh
          ++cur_.rejected;
          rej_i_ = i_;
          ++rej_run_;
          launch_svd(true);
          return false;
        }
        rej_run_ = 0;
      } else if (!fresh_finish(k_cur_)) {
        // a shifted Cholesky factorisation in the unguarded call: redo it
        // guarded (same attempt, same test matrix)
        ++redone_total_;
        if (defer_) {
          defer_svd(true, k_cur_, p_, (uint32_t)i_, last_attempt_, true);
          return false;
        }
        fresh_launch(k_cur_, p_, (uint32_t)i_, last_attempt_, true);
        mark();
        return false;
      }
      if (lastS_[k_cur_ - 1] > prm_.tau && k_cur_ < kcap_) {  // rank search
        k_cur_ = std::min(k_cur_ + prm_.l, kcap_);
        launch_svd(false);
        return false;
      }
      int r = 0;
      while (r < k_cur_ && lastS_[r] > prm_.tau) ++r;
      r_ = r;
      sig_host_.assign(r, 0.0);
      for (int j = 0; j < r; ++j) sig_host_[j] = lastS_[j] - prm_.tau;
      sddmm_launch(r);
      mark();
      phase_ = kSddmm;
      return false;
    }
    const double res = std::sqrt(sddmm_finish()) / mnorm_;
    MC_REQUIRE(std::isfinite(res), kENUMERIC, "non-finite residual");
    err_hist_.push_back(res);
    fresh_total_ += cur_.fresh;
    recycled_total_ += cur_.recycled;
    rejected_total_ += cur_.rejected;
    converged_ = res < prm_.eps;
    cur_.i = i_;
    cur_.r = r_;
    cur_.k = k_cur_;
    cur_.p = p_;
    cur_.res = res;
    cur_.converged = converged_ ? 1 : 0;
    cur_.sigma_max = lastS_.empty() ? 0.0 : lastS_[0];
    phase_ = kIdle;
    return true;
  } catch (...) {
    phase_ = kIdle;
    throw;
  }
}

StepInfo Solver::step() {
  step_begin();
  while (!step_poll(true)) {
  }
  return cur_;
}

void solve_dims(int64_t m, int64_t n, const mc_svt_params& p, int64_t& k, int64_t& b,
                int64_t& L) {
  const int64_t mn = std::min(m, n);
  k = p.k_max > 0 ? std::min<int64_t>(p.k_max, mn) : mn;
  // widths(): b = min(k + s, min(m, n)); the set-up run has b = 11, p = 10
  b = std::max(std::min<int64_t>(k + std::max(p.s, 0), mn), std::min<int64_t>(11, mn));
  L = std::max(std::min<int64_t>((int64_t)(std::max(p.p_max, 0) + 1) * b, mn),
               std::min<int64_t>(121, mn));
}

size_t footprint_bytes(int64_t m, int64_t n, int64_t nnz, const mc_svt_params& p) {
  int64_t k, b, L;
  solve_dims(m, n, p, k, b, L);
  const int64_t Lp = round_up(L, 32);
  const int64_t mx = std::max(m, n);
  size_t bytes = 0;
  bytes += (size_t)nnz * (8 * 3 + 4 * 6);                 // values + layout
  // pointers; work schedules of both directions: plain segments and fix-ups
  // (at most rows + slots each), and where a banded form is built its
  // segments with their padding (at most kBands times the live ones)
  const int64_t slots = spmm_slot_bound(nnz);
  bytes += (size_t)(m + n + 2) * 4 + (size_t)16 * (2 * (m + n) + 4 * slots);
  for (int64_t g : {n, m})
    if (g >= kBandMinRows)
      bytes += (size_t)16 * (kBands * (mx + slots) + mx + slots);
  bytes += (size_t)8 * (n * b + 2 * m * L + m * std::max(b, k) + m * b + n * b +
                        n * L + L * L + L * b + 2 * b * b + m * k + n * k +
                        L * k + 4 * L);
  bytes += (size_t)8 * (gram_splits(mx, (int)L, (int)L, 1) * L * L);
  bytes += (size_t)8 * (3 * Lp * Lp);
  // tridiagonal eigensolver: reflector rows, and for the multi-launch path a
  // copy of G, reflectors, vectors and small factors (k <= 140)
  const int64_t Lb = std::min<int64_t>(L, 1024), kb = std::min<int64_t>(Lb, 140);
  bytes += (size_t)8 * (L * L);
  bytes += (size_t)8 * TriBigWork::doubles((int)Lb, (int)kb);
  // SpMM partial rows (slots x the widest panel), SDDMM partials (one per
  // workgroup of row segments, plain or banded, or per 256 entries), P_Phi(X)
  bytes += (size_t)8 * (slots * std::max({b, L, k}) +
                        std::max(ceil_div(nnz, 256),
                                 ceil_div((int64_t)kBands * (mx + slots) + mx + slots,
                                          kSpmmWaves)) +
                        nnz);
  return bytes;
}

}  // namespace mcsvt
