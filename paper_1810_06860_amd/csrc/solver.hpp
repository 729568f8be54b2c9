// Host-side state machine of fast SVT (Alg. 6) over the device kernels.
#pragma once

#include <array>
#include <map>
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

class Solver {
 public:
  Solver(int64_t m, int64_t n, int64_t nnz, const mc_svt_params& prm,
         hipStream_t st);
  ~Solver();

  // Phi and M_Phi from host arrays (COO rows, int32 cols).  Returns a status.
  int init(const int64_t* rows, const int32_t* cols, const double* vals,
           bool scale_for_svt);
  StepInfo step();
  // truncated SVD of the current operator: one rSVD-BKI call (Alg. 5)
  void rsvd(int k, int p, uint32_t step_id, uint32_t attempt);

  // results
  void get_factors(double* U, double* sig, double* V, int64_t ldu, int64_t ldv);
  void get_rsvd(double* U, double* S, double* V);
  void get_observed(double* x_phi);
  void get_y(double* y_host);

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
  const std::vector<double>& last_sigma() const { return lastS_; }
  hipStream_t stream() const { return st_; }
  int eig_sweeps() const { return eig_.sweeps; }
  int chol_shifts();

  std::string last_error;
  Profiler prof;

 private:
  // workspace sizing
  void ensure(int bmax, int Lmax, int kmax);
  int kcap() const { return kcap_; }
  void widths(int k, int p, int& b, int& p_eff) const;

  void fresh_svd(int k, int p, uint32_t step_id, uint32_t attempt);
  double recycled_svd(int k);
  // eigSVD of B^T = Y^T basis (basis: m x w, leading dim ldb), keep top k;
  // U = basis Wk, V = B^T Wk S^-1, S on the device (kernels only).
  void eig_body(const double* basis, int64_t ldb, int w, int k);
  void fresh_body(int k, int b, int p_eff, int Lw);
  void ritz_body(int k);
  double read_results(int k, bool ritz);
  // kernels go to the capture stream while a graph is being recorded
  hipStream_t ls() const { return capturing_ ? cap_ : st_; }
  bool graphs_ok(int w) const;
  using GraphKey = std::array<int64_t, 8>;
  template <class F> void run_graph(const GraphKey& key, F&& body);
  void clear_graphs();
  void orth_block(int j, int b, int Lw);
  void cholqr_pass(const double* Hin, int64_t ldin, double* out, int64_t ldo,
                   int b, const int* gate);
  void project(const double* Hin, int64_t ldin, double* Hout, int jb, int b,
               int Lw, const int* gate);
  void spmm_y(const double* X, int64_t ldx, double* out, int64_t ldo, int b);
  void spmm_yt(const double* X, int64_t ldx, double* out, int64_t ldo, int b);

  int64_t m_, n_, nnz_;
  mc_svt_params prm_;
  hipStream_t st_;
  int kcap_ = 1;

  Layout L_;
  DevBuf<double> mvals_, y_, ycsc_;
  // workspace
  int cap_b_ = 0, cap_L_ = 0, cap_k_ = 0;
  DevBuf<double> omega_, Qw_, basis_, H1_, H2_, Z_, Bt_, G_, Cg_, Rinv_,
      chol_work_, gram_part_, spmm_part_, U_, V_, S_, Sinv_, D_, Wk_, sig_,
      sdd_part_, scal_, ritz_part_, ritz_out_, obs_;
  DevBuf<int> shift_count_, blk_flag_;
  DevBuf<uint32_t> ctr_;          // (step, attempt) of the Gaussian stream
  uint32_t* hctr_ = nullptr;      // pinned staging for ctr_
  std::map<GraphKey, hipGraphExec_t> graphs_;
  hipStream_t cap_ = nullptr;
  bool capturing_ = false;
  uint64_t gen_ = 0;
  int64_t gram_cap_ = 0;
  EigSolver eig_;
  double* hbuf_ = nullptr;       // pinned host scratch
  size_t hbuf_n_ = 0;

  // Alg. 6 state
  int i_ = 0, r_ = 0, q_ = 0, p_ = 3, streak_ = 0;
  int basis_cols_ = 0;
  int64_t basis_ld_ = 0;
  int k_last_ = 0;              // columns of U_, V_, S_ (last SVD)
  std::vector<double> err_hist_;
  std::vector<double> lastS_;
  std::vector<double> sig_host_;
  bool converged_ = false;
  double c_ = 0.0, norm2_ = 0.0, mnorm_ = 0.0;
  int fresh_total_ = 0, recycled_total_ = 0, rejected_total_ = 0;
};

void resolve_params(int64_t m, int64_t n, int64_t nnz, mc_svt_params& p);
size_t footprint_bytes(int64_t m, int64_t n, int64_t nnz,
                       const mc_svt_params& p);

}  // namespace mcsvt
