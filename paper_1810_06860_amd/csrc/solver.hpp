// Host-side state machine of fast SVT (Alg. 6) over the device kernels.
#pragma once

#include <array>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mcsvt.h"

namespace mcsvt {

struct StepInfo {
  int i = 0, r = 0, k = 0, p = 0, fresh = 0, recycled = 0, rejected = 0;
  int converged = 0;
  double res = 0.0, sigma_max = 0.0;
};

// Event-based timing of kernel families on the solve's own stream.
enum ProfFamily : int {
  kProfSpmmFwd = 0,   // Y X       (CSR)
  kProfSpmmBwd = 1,   // Y^T X     (CSC)
  kProfSddmm = 2,     // fused SDDMM + residual + update
  kProfGram = 3,      // Gram / cross-Gram
  kProfGemm = 4,      // panel GEMMs
  kProfChol = 5,      // Cholesky + inverse
  kProfEig = 6,       // whole eigensolve (kernels + convergence checks)
  kProfRng = 7,       // Gaussian test matrix
  kProfCount = 8
};

struct Profiler {
  bool on = false;
  struct Rec { int fam; double bytes, flops; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  double ms[kProfCount] = {}, bytes[kProfCount] = {}, flops[kProfCount] = {};
  int64_t count[kProfCount] = {};
  ~Profiler();
  hipEvent_t ev();
  void begin(int fam, double bytes, double flops, hipStream_t st);
  void end(hipStream_t st);
  void collect();           // synchronises, folds records into the totals
  void reset();
};

// The control of Alg. 6 (rank search, adaptive p, recycling gate, Ritz
// guard, stop test) -- independent of the arithmetic precision.  The device
// work of one SVD call and of the SDDMM update is supplied by SolverT.
class Solver {
 public:
  Solver(int64_t m, int64_t n, int64_t nnz, const mc_svt_params& prm,
         hipStream_t st);
  virtual ~Solver();

  // Phi and M_Phi from COO arrays (int64 rows, int32 cols), host arrays or,
  // with on_device, device arrays on the solve's stream.  Returns a status.
  virtual int init(const int64_t* rows, const int32_t* cols, const double* vals,
                   bool scale_for_svt, bool on_device = false) = 0;
  // One step, waiting for each device round trip.
  StepInfo step();
  // The same step split at its device round trips, so the host can drive
  // many solves at once: step_begin() makes the step's host decisions and
  // enqueues its first SVD call; step_poll() advances the step whenever the
  // last enqueued work has finished (blocking when `block`) and returns true
  // once the step is complete, its result in step_result().
  void step_begin();
  bool step_poll(bool block);
  bool step_busy() const { return phase_ != kIdle; }

  // Grouped stepping (several solves' sparse products merged into shared
  // launches): with set_deferred(true) the SVD calls of step_begin() and
  // step_poll() are not enqueued but left pending for a driver, which
  // enqueues recycled calls with launch_pending() and runs fresh ones stage
  // by stage (fresh_group_begin, fresh_group_stage until it returns false,
  // fresh_group_end), collecting each stage's sparse product in a task list
  // that it launches for all solves together.  group_kind() says which
  // solves may share launches (same value types), or -1 for none.
  void set_deferred(bool on) { defer_ = on; }
  bool svd_pending() const { return phase_ == kSvdPending; }
  bool pending_fresh() const { return pend_.fresh; }
  void launch_pending();
  virtual int group_kind() const = 0;
  void fresh_group_begin();
  virtual bool fresh_group_stage(int t, std::vector<SpmmTask>* sink) = 0;
  void fresh_group_end();
  const StepInfo& step_result() const { return cur_; }
  // truncated SVD of the current operator: one rSVD-BKI call (Alg. 5)
  void rsvd(int k, int p, uint32_t step_id, uint32_t attempt) {
    fresh_svd(k, p, step_id, attempt);
  }
  // truncated SVD by rSVD-PI (Alg. 4): the same test matrix, p power
  // iterations with the block re-normalised after each one, and the
  // Rayleigh-Ritz step on the last block alone (width k + s)
  void rsvd_pi(int k, int p, uint32_t step_id, uint32_t attempt) {
    struct Reset {
      bool& f;
      ~Reset() { f = false; }
    } reset{power_};
    power_ = true;
    fresh_svd(k, p, step_id, attempt);
  }

  // results
  virtual void get_factors(double* U, double* sig, double* V, int64_t ldu,
                           int64_t ldv) = 0;
  virtual void get_rsvd(double* U, double* S, double* V) = 0;
  virtual void get_observed(double* x_phi) = 0;
  virtual void get_y(double* y_host) = 0;
  virtual int chol_shifts() = 0;

  const mc_svt_params& params() const { return prm_; }
  int64_t m() const { return m_; }
  int64_t n() const { return n_; }
  int64_t nnz() const { return nnz_; }
  int rank() const { return r_; }
  int iters() const { return i_; }
  bool converged() const { return converged_; }
  double c() const { return c_; }
  double norm2() const { return norm2_; }
  double mnorm() const { return mnorm_; }
  double last_res() const { return err_hist_.empty() ? 1.0 : err_hist_.back(); }
  int fresh_total() const { return fresh_total_; }
  int recycled_total() const { return recycled_total_; }
  int rejected_total() const { return rejected_total_; }
  int shifts_seen() const { return shifts_seen_; }
  int redone_total() const { return redone_total_; }
  const std::vector<double>& last_sigma() const { return lastS_; }
  hipStream_t stream() const { return st_; }

  std::string last_error;
  Profiler prof;

 protected:
  // One rSVD-BKI call: enqueues the device work and the copy of its k
  // singular values to the host, sets k_last_, the recycling basis, q_ = 0.
  // Unguarded, the orthonormalisation runs two passes per block; guarded, it
  // adds the third pass that a shifted Cholesky factorisation needs (gated on
  // the device by a flag).
  virtual void fresh_launch(int k, int p, uint32_t step_id, uint32_t attempt,
                            bool guarded) = 0;
  // after the enqueued work finished: lastS_ (k, descending).  False when an
  // unguarded call needed a shifted factorisation: the call must be redone
  // guarded (same test matrix), which gives the result of the guarded form.
  virtual bool fresh_finish(int k) = 0;
  // One recycled SVD from the saved basis (enqueue), then lastS_ and the
  // worst Ritz ratio when the guard is on (else 0).
  virtual void recycled_launch(int k) = 0;
  virtual double recycled_finish(int k) = 0;
  // SDDMM + update with X = U[:, :r] diag(sig_host_) V[:, :r]^T (enqueue),
  // then the sum of squared residuals on Phi
  virtual void sddmm_launch(int r) = 0;
  virtual double sddmm_finish() = 0;
  // blocking forms
  void fresh_svd(int k, int p, uint32_t step_id, uint32_t attempt);
  double sddmm(int r);
  void widths(int k, int p, int& b, int& p_eff) const;
  void mark();                  // record the completion event on the stream
  void wait();                  // wait for it

  bool power_ = false;          // fresh calls run rSVD-PI instead of rSVD-BKI
  enum Phase { kIdle, kSvd, kSddmm, kSvdPending };
  Phase phase_ = kIdle;
  // a deferred SVD call (grouped stepping)
  struct Pending {
    bool fresh = false, guarded = false;
    int k = 0, p = 0;
    uint32_t step = 0, attempt = 0;
  };
  bool defer_ = false;
  Pending pend_;
  void defer_svd(bool fresh, int k, int p, uint32_t step, uint32_t attempt, bool guarded);
  // the parts of a fresh call around its device body (fresh_launch is
  // begin, body, end); `grouped` leaves the body to fresh_group_stage
  virtual void fresh_begin(int k, int p, uint32_t step_id, uint32_t attempt,
                           bool guarded) = 0;
  virtual void fresh_end() = 0;
  StepInfo cur_;
  int k_cur_ = 0;
  bool cur_recycled_ = false;
  uint32_t attempt_ = 0, last_attempt_ = 0;
  hipEvent_t done_ev_ = nullptr;
  void launch_svd(bool force_fresh);

  int64_t m_, n_, nnz_;
  mc_svt_params prm_;
  hipStream_t st_;
  int kcap_ = 1;
  int64_t lim_k_ = 1, lim_b_ = 1, lim_L_ = 1;   // solve_dims of this solve

  // Alg. 6 state
  int i_ = 0, r_ = 0, q_ = 0, p_ = 3, streak_ = 0;
  int rej_i_ = 0;               // last step whose recycled call was rejected
  int rej_run_ = 0;             // rejections since the last accepted recycled call
  int basis_cols_ = 0;
  int64_t basis_ld_ = 0;
  int k_last_ = 0;              // columns of U, V, S of the last SVD call
  std::vector<double> err_hist_;
  std::vector<double> lastS_;
  std::vector<double> sig_host_;
  bool converged_ = false;
  double c_ = 0.0, norm2_ = 0.0, mnorm_ = 0.0;
  int fresh_total_ = 0, recycled_total_ = 0, rejected_total_ = 0;
  int shifts_seen_ = 0;         // shift count read back with the last fresh call
  int redone_total_ = 0;        // fresh calls redone guarded
};

// One step of each solver with their fresh calls' sparse products launched
// together (group.hip); per-solver status codes and messages.
void step_group(const std::vector<Solver*>& ss, std::vector<int>& status,
                std::vector<std::string>& err);

// FP64, FP32 or BF16-value solver according to prm.precision
std::unique_ptr<Solver> make_solver(int64_t m, int64_t n, int64_t nnz,
                                    const mc_svt_params& prm, hipStream_t st);

void resolve_params(int64_t m, int64_t n, int64_t nnz, mc_svt_params& p);
// Largest rank k, block width b and Krylov basis width L a solve with these
// parameters can reach: the rank search stops at min(m, n, k_max) (min(m, n)
// when k_max = 0), p stays <= p_max, and the spectral-norm run at set-up
// uses k = 1, s = 10, p = 10.  The footprint prices these, and the solver's
// buffers never grow past them.
void solve_dims(int64_t m, int64_t n, const mc_svt_params& p, int64_t& k, int64_t& b,
                int64_t& L);
size_t footprint_bytes(int64_t m, int64_t n, int64_t nnz,
                       const mc_svt_params& p);

}  // namespace mcsvt
