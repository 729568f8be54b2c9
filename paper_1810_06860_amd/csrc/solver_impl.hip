// Device work of fast SVT for one arithmetic precision.
//
// rSVD-BKI on the device (Alg. 5):
//   Omega (n x b) Gaussian; H_0 = Y Omega; for j = 1..p: H_j = Y (Y^T Q_{j-1});
//   each H_j is orthonormalised against Q_0..Q_{j-1} by block Gram-Schmidt
//   with re-orthogonalisation and Cholesky QR (two passes each), which
//   spans the same subspace as the LU-normalised blocks followed by orth()
//   (Lemmas 2 and 3), so Q = [Q_0 .. Q_p] is already orthonormal;
//   B^T = Y^T Q; eigSVD(B^T): G = B B^T, eig(G), top k, S = sqrt(lambda),
//   U = Q W_k, V = B^T W_k S^-1.
//   Because every Q_j is final once it is formed, the Krylov product
//   Y^T Q_{j-1} is already block j-1 of B^T: the loop writes it there, and
//   B^T needs one more product of width b (Y^T Q_p) instead of one of width
//   (p + 1) b.
//
// Precision: P is the type of the dense panels (Omega, H, Q, B^T, U, V), VT
// the type of the copies of Y read by the forward Krylov SpMMs Y X of Alg. 5
// (and by both products of rSVD-PI), AT the accumulator of SpMM / Gram /
// SDDMM dot products.  The products Y^T Q_j (blocks of the Rayleigh-Ritz
// product B^T = Y^T Q), the Ritz guard and the SDDMM read Y in the panel
// precision P, so the singular values are those of the computed subspace to
// that precision whatever VT is.  The master copy of Y, M_Phi, every Gram
// result, the Cholesky factors, the eigensolve and the residual sums are FP64
// in all modes:
//   FP64       P = double, VT = double, AT = double
//   FP32       P = float,  VT = float,  AT = float
//   BF16       P = float,  VT = bf16,   AT = float   (forward Krylov products: values
//                                                   and panel in BF16)
#include <cmath>
#include <cstring>
#include <type_traits>
#include <utility>

#include "solver.hpp"

namespace mcsvt {

namespace {

template <class T>
void swap_buf(DevBuf<T>& a, DevBuf<T>& b) {
  std::swap(a.p, b.p);
  std::swap(a.n, b.n);
  std::swap(a.stream, b.stream);
}

// algorithmic bytes of one SpMM: values + indices + pointers + panel in + out
// Gram products over at most this many rows finish (and factor) in the same
// launch; taller panels keep many row splits and a separate reduction
constexpr int64_t kFuseRows = 8192;
// the fused completion factors the Gram in registers up to this width; wider
// blocks go to the 1024-thread Cholesky kernel, which keeps its registers
// for b up to 128
constexpr int kFuseCholMax = 64;

double spmm_bytes(int64_t nnz, int64_t rows, int64_t cols, int b, int sv, int sx) {
  return (double)nnz * (sv + 4) + 4.0 * (rows + 1) + (double)cols * b * sx +
         (double)rows * b * sx;
}

template <class P, class VT, class AT>
class SolverT final : public Solver {
 public:
  static constexpr bool kMaster = std::is_same<VT, double>::value;
  // separate Rayleigh-Ritz copies (type P) when the Krylov copies are not P
  static constexpr bool kSplit = !std::is_same<VT, P>::value;
  // BF16 mode: the forward Krylov products also read their dense panel in
  // BF16 (a copy made just before the product)
  static constexpr bool kBfPanel = std::is_same<VT, bf16_t>::value;

  SolverT(int64_t m, int64_t n, int64_t nnz, const mc_svt_params& prm,
          hipStream_t st)
      : Solver(m, n, nnz, prm, st) {
    shift_count_.reserve(1, st_);
    blk_flag_.reserve(1, st_);
    fuse_ctr_.reserve(1, st_);
    MC_HIP(hipMemsetAsync(fuse_ctr_.p, 0, sizeof(int), st_));   // 0 between launches
    ctr_.reserve(2, st_);
    MC_HIP(hipHostMalloc((void**)&hctr_, 2 * sizeof(uint32_t)));
    MC_HIP(hipMemsetAsync(shift_count_.p, 0, sizeof(int), st_));
  }

  ~SolverT() override {
    clear_graphs();
    if (cap_) (void)hipStreamDestroy(cap_);
    if (hbuf_) (void)hipHostFree(hbuf_);
    if (hctr_) (void)hipHostFree(hctr_);
  }

  int init(const int64_t* rows, const int32_t* cols, const double* vals,
           bool scale_for_svt, bool on_device) override;
  void get_factors(double* U, double* sig, double* V, int64_t ldu,
                   int64_t ldv) override;
  void get_rsvd(double* U, double* S, double* V) override;
  void get_observed(double* x_phi) override;
  void get_y(double* y_host) override;
  int chol_shifts() override {
    int v = 0;
    MC_HIP(hipMemcpyAsync(&v, shift_count_.p, sizeof(int), hipMemcpyDeviceToHost, st_));
    MC_HIP(hipStreamSynchronize(st_));
    return v;
  }

 protected:
  void fresh_launch(int k, int p, uint32_t step_id, uint32_t attempt,
                    bool guarded) override;
  void fresh_begin(int k, int p, uint32_t step_id, uint32_t attempt,
                   bool guarded) override;
  void fresh_end() override;
  bool fresh_group_stage(int t, std::vector<SpmmTask>* sink) override;
  // solves of one kind may share grouped sparse products: FP64 and FP32
  // (values and panels of one type); BF16 mode mixes types and launches alone
  int group_kind() const override {
    if constexpr (std::is_same<VT, double>::value) return 0;
    if constexpr (std::is_same<VT, float>::value) return 1;
    return -1;
  }
  bool fresh_finish(int k) override;
  void recycled_launch(int k) override;
  double recycled_finish(int k) override;
  void sddmm_launch(int r) override;
  double sddmm_finish() override;

 private:
  using GraphKey = std::array<int64_t, 8>;
  void ensure(int bmax, int Lmax, int kmax);
  // have_bt: B^T = Y^T basis is already in Bt_ (leading dimension w)
  void eig_body(const P* basis, int64_t ldb, int w, int k, bool have_bt = false);
  void fresh_body(int k, int b, int p_eff, int Lw, bool guarded);
  // stage t of a fresh rSVD-BKI call (see fresh_stage's definition)
  bool fresh_stage(int t, int k, int b, int p_eff, int Lw, bool guarded);
  // the call fresh_begin set up: k, b, p_eff, Lw, guarded
  struct Call {
    int k = 0, b = 0, p_eff = 0, Lw = 0;
    bool guarded = false;
  } call_;
  // set while a grouped driver runs the stages: products are collected, not
  // launched
  std::vector<SpmmTask>* sink_ = nullptr;
  void ritz_body(int k);
  void read_launch(int k, bool ritz, bool count = false);
  double read_finish(int k, bool ritz);
  hipStream_t ls() const { return capturing_ ? cap_ : st_; }
  // capture needs an eigensolve without host round trips
  bool graphs_ok(int w, int k) const {
    return prm_.use_graphs && !prof.on && !graphs_broken_ && EigSolver::device_only(w, k);
  }
  bool graphs_broken_ = false;
  template <class F> void run_graph(const GraphKey& key, F&& body);
  void clear_graphs() {
    for (auto& kv : graphs_) (void)hipGraphExecDestroy(kv.second);
    graphs_.clear();
  }
  void orth_block(int j, int b, int Lw, bool guarded);
  // low: in BF16 mode the Gram runs on the BF16 matrix cores (the first of
  // the two orthonormalisation passes; the second, which restores
  // orthogonality to FP32 accuracy, keeps the FP32 Gram)
  void cholqr_pass(const P* Hin, int64_t ldin, P* out, int64_t ldo, int b,
                   const int* gate, bool low = false);
  void project(const P* Hin, int64_t ldin, P* Hout, int jb, int b, int Lw,
               const int* gate, bool low = false);
  // Krylov products (values of type VT)
  void spmm_y(const P* X, int64_t ldx, P* out, int64_t ldo, int b);
  void spmm_yt(const P* X, int64_t ldx, P* out, int64_t ldo, int b);
  // Rayleigh-Ritz / Ritz-guard products (values of type P)
  void spmm_y_rr(const P* X, int64_t ldx, P* out, int64_t ldo, int b);
  void spmm_yt_rr(const P* X, int64_t ldx, P* out, int64_t ldo, int b);
  const VT* yv() const {
    if constexpr (kMaster) return y_.p; else return yv_.p;
  }
  const P* yw() const {
    if constexpr (kSplit) return yw_.p; else return (const P*)yv();
  }
  const P* ycw() const {
    if constexpr (kSplit) return ycw_.p; else return (const P*)ycv_.p;
  }

  Layout L_;
  DevBuf<double> mvals_, y_;        // M_Phi and the FP64 master of Y (CSR)
  DevBuf<VT> yv_, ycv_;             // Krylov copies of Y: CSR (unless VT is
                                    // double: the master) and CSC
  DevBuf<P> yw_, ycw_;              // Rayleigh-Ritz copies (when VT != P)
  int cap_b_ = 0, cap_L_ = 0, cap_k_ = 0;
  DevBuf<P> omega_, Qw_, basis_, H1_, H2_, Z_, Bt_, U_, V_;
  DevBuf<VT> xb_;                 // BF16 copy of a forward product's panel
  DevBuf<AT> gram_part_, spmm_part_;
  DevBuf<double> G_, Cg_, Rinv_, chol_work_, S_, Sinv_, D_, Wk_, sig_, sdd_part_,
      scal_, ritz_part_, ritz_out_, obs_;
  DevBuf<int> shift_count_, blk_flag_, fuse_ctr_;
  DevBuf<uint32_t> ctr_;          // (step, attempt) of the Gaussian stream
  uint32_t* hctr_ = nullptr;      // pinned staging for ctr_
  std::map<GraphKey, hipGraphExec_t> graphs_;
  hipStream_t cap_ = nullptr;
  bool capturing_ = false;
  uint64_t gen_ = 0;
  int64_t gram_cap_ = 0;
  EigSolver eig_;
  double* hbuf_ = nullptr;       // pinned host scratch
  bool last_guarded_ = true;     // the last fresh call ran the gated third pass
  size_t hbuf_n_ = 0;
};

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::ensure(int bmax, int Lmax, int kmax) {
  if (bmax <= cap_b_ && Lmax <= cap_L_ && kmax <= cap_k_ && hbuf_) return;
  // buffers move: captured graphs hold their addresses
  ++gen_;
  clear_graphs();
  // grow with headroom so the rank search does not reallocate every step,
  // never past what the solve can reach (its footprint prices exactly that)
  auto grow = [&](int want, int have, int64_t lim) {
    if (want <= have) return have;
    return (int)std::min<int64_t>(lim, std::max<int64_t>(want, (int64_t)have * 5 / 4 + 8));
  };
  cap_b_ = std::max(grow(bmax, cap_b_, lim_b_), bmax);
  cap_L_ = std::max(grow(Lmax, cap_L_, lim_L_), Lmax);
  cap_k_ = std::max(grow(kmax, cap_k_, lim_k_), kmax);
  const int64_t b = cap_b_, Lc = cap_L_, k = cap_k_;
  const int64_t wide = std::max({b, Lc, k});
  omega_.reserve(n_ * b, st_);
  Qw_.reserve(m_ * Lc, st_);
  H1_.reserve(m_ * std::max(b, k), st_);
  H2_.reserve(m_ * b, st_);
  Z_.reserve(n_ * b, st_);
  if (kBfPanel) xb_.reserve(n_ * b, st_);
  Bt_.reserve(n_ * Lc, st_);
  G_.reserve(Lc * Lc, st_);
  Cg_.reserve(Lc * b, st_);
  Rinv_.reserve(b * b, st_);
  chol_work_.reserve(2 * b * b, st_);
  const int64_t mx = std::max(m_, n_);
  gram_cap_ = std::max({gram_splits(mx, (int)Lc, (int)Lc, 1) * Lc * Lc,
                        gram_splits(m_, (int)b, (int)b, 1) * b * b,
                        gram_splits(m_, (int)Lc, (int)b, 0) * Lc * b});
  gram_part_.reserve(gram_cap_, st_);
  const int64_t slots = std::max(L_.sched_csr.nslot, L_.sched_csc.nslot);
  spmm_part_.reserve(std::max<int64_t>(1, slots) * wide, st_);
  U_.reserve(m_ * k, st_);
  V_.reserve(n_ * k, st_);
  S_.reserve(k + 1, st_);         // + the shift count behind the values
  Sinv_.reserve(k, st_);
  D_.reserve(Lc, st_);
  Wk_.reserve(Lc * k, st_);
  sig_.reserve(k, st_);
  ritz_part_.reserve((int64_t)ritz_blocks(m_) * k, st_);
  ritz_out_.reserve(k, st_);
  eig_.reserve((int)Lc, st_);
  const size_t need = (size_t)(2 * std::max(Lc, k) + 64);
  if (!hbuf_ || hbuf_n_ < need) {
    if (hbuf_) MC_HIP(hipHostFree(hbuf_));
    // coherent: kernels write the per-call results (S, the shift count, the
    // residual) here directly, and the host reads them after the stream event
    MC_HIP(hipHostMalloc((void**)&hbuf_, need * sizeof(double), hipHostMallocCoherent));
    hbuf_n_ = need;
  }
}

template <class P, class VT, class AT>
int SolverT<P, VT, AT>::init(const int64_t* rows, const int32_t* cols,
                             const double* vals, bool scale_for_svt, bool on_device) {
  DevBuf<int64_t> d_rows;
  DevBuf<int32_t> d_cols;
  DevBuf<double> d_vals;
  if (!on_device) {
    d_rows.reserve(nnz_, st_);
    d_cols.reserve(nnz_, st_);
    d_vals.reserve(nnz_, st_);
    MC_HIP(hipMemcpyAsync(d_rows.p, rows, nnz_ * sizeof(int64_t), hipMemcpyHostToDevice, st_));
    MC_HIP(hipMemcpyAsync(d_cols.p, cols, nnz_ * sizeof(int32_t), hipMemcpyHostToDevice, st_));
    MC_HIP(hipMemcpyAsync(d_vals.p, vals, nnz_ * sizeof(double), hipMemcpyHostToDevice, st_));
  }
  const int64_t* pr = on_device ? rows : d_rows.p;
  const int32_t* pc = on_device ? cols : d_cols.p;
  const double* pv = on_device ? vals : d_vals.p;
  const int status = build_layout(m_, n_, nnz_, pr, pc, pv, L_, st_);
  if (status != kOK) return status;
  mvals_.reserve(nnz_, st_);
  y_.reserve(nnz_, st_);
  ycv_.reserve(nnz_, st_);
  if (!kMaster) yv_.reserve(nnz_, st_);
  if (kSplit) {
    yw_.reserve(nnz_, st_);
    ycw_.reserve(nnz_, st_);
  }
  launch_gather(nnz_, L_.order.p, pv, mvals_.p, st_);
  ensure(1, 1, 1);
  sdd_part_.reserve(sddmm_partials(L_), st_);
  scal_.reserve(8, st_);
  launch_sumsq(nnz_, mvals_.p, sdd_part_.p, scal_.p, st_);
  MC_HIP(hipMemcpyAsync(hbuf_, scal_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
  mnorm_ = std::sqrt(hbuf_[0]);
  MC_REQUIRE(std::isfinite(mnorm_), kEINVAL, "non-finite value in M_Phi");
  // the operator copies start as M_Phi (for ||P_Phi(M)||_2)
  auto refresh_operator = [&](double scale) {
    launch_scale(nnz_, mvals_.p, scale, y_.p, st_);
    // CSC copy through a gather of the master, cast to VT
    DevBuf<double> tmp;
    tmp.reserve(nnz_, st_);
    launch_gather(nnz_, L_.perm.p, y_.p, tmp.p, st_);
    launch_cast<double, VT>(nnz_, tmp.p, ycv_.p, st_);
    if (!kMaster) launch_cast<double, VT>(nnz_, y_.p, yv_.p, st_);
    if (kSplit) {
      launch_cast<double, P>(nnz_, tmp.p, ycw_.p, st_);
      launch_cast<double, P>(nnz_, y_.p, yw_.p, st_);
    }
    MC_HIP(hipStreamSynchronize(st_));
  };
  refresh_operator(1.0);
  if (scale_for_svt) {
    MC_REQUIRE(mnorm_ > 0, kEINVAL, "M_Phi is identically zero");
    // ||P_Phi(M)||_2 by a block Krylov run on M itself (k = 1, s = 10)
    const int saved_s = prm_.s;
    prm_.s = 10;
    fresh_svd(1, 10, 0u, 0u);
    prm_.s = saved_s;
    norm2_ = lastS_[0];
    MC_REQUIRE(std::isfinite(norm2_) && norm2_ > 0, kENUMERIC,
               "spectral norm of P_Phi(M) is not positive");
    c_ = prm_.c > 0 ? prm_.c : std::ceil(prm_.tau / (prm_.delta * norm2_));
    refresh_operator(c_ * prm_.delta);                   // Y^0 = c delta M_Phi
    basis_cols_ = 0;
    k_last_ = 0;
    lastS_.clear();
  }
  MC_HIP(hipStreamSynchronize(st_));
  return kOK;
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::spmm_y(const P* X, int64_t ldx, P* out, int64_t ldo, int b) {
  if (sink_ && !kBfPanel) {
    sink_->push_back(make_spmm_task(L_.sched_csr, L_.col_idx.p, yv(), X, ldx, out, ldo, b,
                                    spmm_part_.p, sizeof(P)));
    return;
  }
  if constexpr (kBfPanel) {
    // values and panel in BF16, FP32 accumulation; the panel's BF16 copy is
    // made here (n b elements)
    const double bytes = (double)nnz_ * (sizeof(VT) + 4) + 4.0 * (m_ + 1) +
                         (double)n_ * b * sizeof(VT) + (double)m_ * b * sizeof(P) +
                         (double)n_ * b * (sizeof(P) + sizeof(VT));     // + the copy
    prof.begin(kProfSpmmFwd, bytes, 2.0 * nnz_ * b, ls());
    launch_cast_panel<P, VT>(n_, b, X, ldx, xb_.p, b, ls());
    launch_spmm<VT, VT, AT, P>(L_.sched_csr, L_.col_idx.p, yv(), xb_.p, b, out, ldo, b,
                               spmm_part_.p, ls());
  } else {
    prof.begin(kProfSpmmFwd, spmm_bytes(nnz_, m_, n_, b, sizeof(VT), sizeof(P)),
               2.0 * nnz_ * b, ls());
    launch_spmm<VT, P, AT, P>(L_.sched_csr, L_.col_idx.p, yv(), X, ldx, out, ldo, b,
                              spmm_part_.p, ls());
  }
  prof.end(ls());
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::spmm_yt(const P* X, int64_t ldx, P* out, int64_t ldo, int b) {
  prof.begin(kProfSpmmBwd, spmm_bytes(nnz_, n_, m_, b, sizeof(VT), sizeof(P)),
             2.0 * nnz_ * b, ls());
  launch_spmm<VT, P, AT, P>(L_.sched_csc, L_.row_idx.p, ycv_.p, X, ldx, out, ldo, b,
                            spmm_part_.p, ls());
  prof.end(ls());
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::spmm_y_rr(const P* X, int64_t ldx, P* out, int64_t ldo, int b) {
  prof.begin(kProfSpmmFwd, spmm_bytes(nnz_, m_, n_, b, sizeof(P), sizeof(P)),
             2.0 * nnz_ * b, ls());
  launch_spmm<P, P, AT, P>(L_.sched_csr, L_.col_idx.p, yw(), X, ldx, out, ldo, b,
                           spmm_part_.p, ls());
  prof.end(ls());
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::spmm_yt_rr(const P* X, int64_t ldx, P* out, int64_t ldo, int b) {
  if (sink_) {
    sink_->push_back(make_spmm_task(L_.sched_csc, L_.row_idx.p, ycw(), X, ldx, out, ldo, b,
                                    spmm_part_.p, sizeof(P)));
    return;
  }
  prof.begin(kProfSpmmBwd, spmm_bytes(nnz_, n_, m_, b, sizeof(P), sizeof(P)),
             2.0 * nnz_ * b, ls());
  launch_spmm<P, P, AT, P>(L_.sched_csc, L_.row_idx.p, ycw(), X, ldx, out, ldo, b,
                           spmm_part_.p, ls());
  prof.end(ls());
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::cholqr_pass(const P* Hin, int64_t ldin, P* out, int64_t ldo,
                                     int b, const int* gate, bool low) {
  // Gram, its completion and the Cholesky inverse in one launch
  prof.begin(kProfGram, (double)sizeof(P) * m_ * b,
             1.0 * m_ * b * (b + 1) + (double)b * b * b, ls());
  if constexpr (kBfPanel) {
    low = low && !gate && gram_bf16_fits(m_, b, b, 1);
  } else {
    low = false;
  }
  if (low) {
    if constexpr (kBfPanel) {
      launch_gram_bf16(m_, b, b, Hin, ldin, Hin, ldin, G_.p, b, 1, gram_part_.p,
                       gram_cap_, ls());
      launch_chol_inv(b, G_.p, b, Rinv_.p, b, chol_work_.p, m_, shift_count_.p, ls(),
                      blk_flag_.p, gate);
    }
  } else if (b <= kFuseCholMax && m_ <= kFuseRows) {
    launch_gram_fused<P, AT>(m_, b, b, Hin, ldin, Hin, ldin, G_.p, b, 1, gram_part_.p,
                             gram_cap_, fuse_ctr_.p, Rinv_.p, b, m_, shift_count_.p,
                             blk_flag_.p, ls(), gate);
  } else {
    launch_gram<P, AT>(m_, b, b, Hin, ldin, Hin, ldin, G_.p, b, 1, gram_part_.p,
                       gram_cap_, ls(), gate);
    launch_chol_inv(b, G_.p, b, Rinv_.p, b, chol_work_.p, m_, shift_count_.p, ls(),
                    blk_flag_.p, gate);
  }
  prof.end(ls());
  prof.begin(kProfGemm, 2.0 * sizeof(P) * m_ * b, 2.0 * m_ * b * b, ls());
  launch_panel_gemm<P, P>(m_, b, b, Hin, ldin, Rinv_.p, b, 1.0, nullptr, 0.0,
                          nullptr, 0, out, ldo, ls(), gate);
  prof.end(ls());
}

// Hout = Hin - Qp (Qp^T Hin) with Qp = the first jb columns of Qw_
template <class P, class VT, class AT>
void SolverT<P, VT, AT>::project(const P* Hin, int64_t ldin, P* Hout, int jb, int b,
                                 int Lw, const int* gate, bool low) {
  prof.begin(kProfGram, (double)sizeof(P) * m_ * (jb + b), 2.0 * m_ * jb * b, ls());
  if constexpr (kBfPanel) {
    low = low && !gate && gram_bf16_fits(m_, jb, b, 0);
  } else {
    low = false;
  }
  if (low) {
    if constexpr (kBfPanel)
      launch_gram_bf16(m_, jb, b, Qw_.p, Lw, Hin, ldin, Cg_.p, b, 0, gram_part_.p,
                       gram_cap_, ls());
  } else if ((int64_t)jb * b <= 128 * 128 && m_ <= kFuseRows)
    launch_gram_fused<P, AT>(m_, jb, b, Qw_.p, Lw, Hin, ldin, Cg_.p, b, 0, gram_part_.p,
                             gram_cap_, fuse_ctr_.p, nullptr, 0, 0, nullptr, nullptr,
                             ls(), gate);
  else
    launch_gram<P, AT>(m_, jb, b, Qw_.p, Lw, Hin, ldin, Cg_.p, b, 0, gram_part_.p,
                       gram_cap_, ls(), gate);
  prof.end(ls());
  prof.begin(kProfGemm, (double)sizeof(P) * m_ * (jb + 2 * b), 2.0 * m_ * jb * b, ls());
  launch_panel_gemm<P, P>(m_, jb, b, Qw_.p, Lw, Cg_.p, b, -1.0, nullptr, 1.0, Hin,
                          ldin, Hout, b, ls(), gate);
  prof.end(ls());
}

// Orthonormalise the raw Krylov block in H1_ against Q_0..Q_{j-1} and write
// it to columns [j b, (j+1) b) of Qw_: block Gram-Schmidt + Cholesky QR, two
// passes, and a third one only when a Cholesky factorisation needed a shift
// (the device flag gates it; no host round trip).
template <class P, class VT, class AT>
void SolverT<P, VT, AT>::orth_block(int j, int b, int Lw, bool guarded) {
  P* out = Qw_.p + (int64_t)j * b;
  const int* gate = blk_flag_.p;
  if (guarded) launch_set_int(blk_flag_.p, 0, ls());
  if (j == 0) {
    cholqr_pass(H1_.p, b, H2_.p, b, b, nullptr, true);
    cholqr_pass(H2_.p, b, out, Lw, b, nullptr);
    if (guarded) {
      cholqr_pass(out, Lw, H1_.p, b, b, gate);
      launch_copy_gated<P>(m_, b, H1_.p, b, out, Lw, gate, ls());
    }
    return;
  }
  const int jb = j * b;
  project(H1_.p, b, H2_.p, jb, b, Lw, nullptr, true);
  cholqr_pass(H2_.p, b, H1_.p, b, b, nullptr, true);
  project(H1_.p, b, H2_.p, jb, b, Lw, nullptr);
  cholqr_pass(H2_.p, b, out, Lw, b, nullptr);
  // the gated pass writes the block directly (it reads H2, not the block)
  if (guarded) {
    project(out, Lw, H2_.p, jb, b, Lw, gate);
    cholqr_pass(H2_.p, b, out, Lw, b, gate);
  }
}

// S (k values) and, with the Ritz guard, the k Ritz ratios: enqueued copies
// to pinned host memory, read once the stream has reached them
template <class P, class VT, class AT>
void SolverT<P, VT, AT>::read_launch(int k, bool ritz, bool count) {
  // S (and, with `count`, the shift count behind it) were written to hbuf_ by
  // the eigSVD step's reciprocal kernel; the Ritz ratios are copied over the
  // count's slot
  (void)count;
  if (ritz)
    MC_HIP(hipMemcpyAsync(hbuf_ + k, ritz_out_.p, k * sizeof(double),
                          hipMemcpyDeviceToHost, st_));
}

template <class P, class VT, class AT>
double SolverT<P, VT, AT>::read_finish(int k, bool ritz) {
  lastS_.assign(hbuf_, hbuf_ + k);
  for (double v : lastS_)
    MC_REQUIRE(std::isfinite(v), kENUMERIC, "non-finite singular value");
  double worst = 0.0;
  if (ritz)
    for (int j = 0; j < k; ++j) worst = std::max(worst, hbuf_[k + j]);
  return worst;
}

// eigSVD of B^T = Y^T basis (Alg. 3 on B^T, the Rayleigh-Ritz end of Alg. 5):
// kernels only
template <class P, class VT, class AT>
void SolverT<P, VT, AT>::eig_body(const P* basis, int64_t ldb, int w, int k,
                                  bool have_bt) {
  if (!have_bt) spmm_yt_rr(basis, ldb, Bt_.p, w, w);         // B^T = Y^T basis
  prof.begin(kProfGram, (double)sizeof(P) * n_ * w, 1.0 * n_ * w * (w + 1), ls());
  launch_gram<P, AT>(n_, w, w, Bt_.p, w, Bt_.p, w, G_.p, w, 1, gram_part_.p,
                     gram_cap_, ls());                       // G = B B^T (FP64)
  prof.end(ls());
  // algorithmic work of a top-k symmetric eigensolve: the tridiagonal
  // reduction (4/3 w^3) and the back-transformation of k vectors (2 w^2 k)
  prof.begin(kProfEig, 16.0 * w * w, 4.0 / 3.0 * w * w * w + 2.0 * w * w * k, ls());
  eig_.solve_topk(w, G_.p, w, k, S_.p, D_.p, Wk_.p, k, ls());
  prof.end(ls());
  prof.begin(kProfGemm, (double)sizeof(P) * (m_ + n_) * (w + k),
             2.0 * (m_ + n_) * w * k, ls());
  launch_panel_gemm<P, P>(m_, w, k, basis, ldb, Wk_.p, k, 1.0, nullptr, 0.0, nullptr,
                          0, U_.p, k, ls());                 // U = Q W
  // S and the shift count go straight to the pinned read-back buffer
  launch_recip(k, S_.p, Sinv_.p, ls(), shift_count_.p, S_.p + k, hbuf_);
  launch_panel_gemm<P, P>(n_, w, k, Bt_.p, w, Wk_.p, k, 1.0, Sinv_.p, 0.0, nullptr, 0,
                          V_.p, k, ls());                    // V = B^T W S^-1
  prof.end(ls());
}

// Ritz residual ratios ||Y v_j - s_j u_j|| / s_j into ritz_out_
template <class P, class VT, class AT>
void SolverT<P, VT, AT>::ritz_body(int k) {
  spmm_y_rr(V_.p, k, H1_.p, k, k);                           // R = Y V
  launch_ritz<P>(m_, k, H1_.p, k, U_.p, k, S_.p, ritz_part_.p, ritz_out_.p, ls());
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::fresh_body(int k, int b, int p_eff, int Lw, bool guarded) {
  if (power_) {
    // rSVD-PI (Alg. 4): each power iteration replaces the block; the
    // normalisation between iterations only has to keep its range (Lemma 3)
    prof.begin(kProfRng, (double)sizeof(P) * n_ * b, 0.0, ls());
    launch_gaussian_ctr<P>(omega_.p, n_, b, b, prm_.seed, ctr_.p, ls());
    prof.end(ls());
    spmm_y(omega_.p, b, H1_.p, b, b);                        // H_0 = Y Omega
    orth_block(0, b, Lw, guarded);
    for (int j = 1; j <= p_eff; ++j) {
      spmm_yt(Qw_.p, Lw, Z_.p, b, b);                        // Y^T Q
      spmm_y(Z_.p, b, H1_.p, b, b);                          // Y Y^T Q
      orth_block(0, b, Lw, guarded);
    }
    eig_body(Qw_.p, Lw, Lw, k);
    return;
  }
  for (int t = 0; fresh_stage(t, k, b, p_eff, Lw, guarded); ++t) {
  }
}

// rSVD-BKI (Alg. 5) in stages that each end with one sparse product, so that
// a grouped driver can launch the products of several solves together:
//   t = 0            Omega;                 product H_0 = Y Omega
//   t = 2j + 1       orthonormalise block j; product Y^T Q_j -> block j of B^T
//   t = 2j (j >= 1)                          product H_j = Y (block j-1 of B^T)
//   t = 2 p_eff + 2  eigSVD of B^T (no product); returns false
// Y^T Q_j is the Krylov product that feeds block j + 1 and, Q_j being final,
// block j of the Rayleigh-Ritz product B^T = Y^T Q; it reads Y in the
// Rayleigh-Ritz precision, as B^T does.
template <class P, class VT, class AT>
bool SolverT<P, VT, AT>::fresh_stage(int t, int k, int b, int p_eff, int Lw,
                                     bool guarded) {
  if (t == 0) {
    prof.begin(kProfRng, (double)sizeof(P) * n_ * b, 0.0, ls());
    launch_gaussian_ctr<P>(omega_.p, n_, b, b, prm_.seed, ctr_.p, ls());
    prof.end(ls());
    spmm_y(omega_.p, b, H1_.p, b, b);                        // H_0 = Y Omega
    return true;
  }
  if (t == 2 * p_eff + 2) {
    eig_body(Qw_.p, Lw, Lw, k, true);
    return false;
  }
  const int j = t / 2;
  if (t % 2 == 1) {
    orth_block(j, b, Lw, guarded);
    spmm_yt_rr(Qw_.p + (int64_t)j * b, Lw, Bt_.p + (int64_t)j * b, Lw, b);
  } else {
    spmm_y(Bt_.p + (int64_t)(j - 1) * b, Lw, H1_.p, b, b);
  }
  return true;
}

template <class P, class VT, class AT>
template <class F>
void SolverT<P, VT, AT>::run_graph(const GraphKey& key, F&& body) {
  auto it = graphs_.find(key);
  if (it == graphs_.end()) {
    if (!cap_) MC_HIP(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
    if (graphs_.size() >= 64) clear_graphs();
    hipGraph_t g = nullptr;
    // relaxed: solves driven from other host threads may allocate meanwhile
    // (nothing inside the captured body allocates)
    MC_HIP(hipStreamBeginCapture(cap_, hipStreamCaptureModeRelaxed));
    capturing_ = true;
    bool ok = true;
    try {
      body();
    } catch (const Error&) {
      ok = false;
    }
    capturing_ = false;
    const hipError_t ee = hipStreamEndCapture(cap_, &g);
    hipGraphExec_t ge = nullptr;
    if (ok && ee == hipSuccess && g) ok = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok || ee != hipSuccess || !ge) {
      // the runtime gave up the capture (it can, when other host threads use
      // the device meanwhile): run this call kernel by kernel, and keep this
      // solve on direct launches from now on; results are the same
      (void)hipGetLastError();
      if (ge) (void)hipGraphExecDestroy(ge);
      graphs_broken_ = true;
      body();
      return;
    }
    it = graphs_.emplace(key, ge).first;
  }
  MC_HIP(hipGraphLaunch(it->second, st_));
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::fresh_begin(int k, int p, uint32_t step_id, uint32_t attempt,
                                     bool guarded) {
  int b, p_eff;
  widths(k, p, b, p_eff);
  const int Lw = power_ ? b : (p_eff + 1) * b;
  ensure(b, Lw, k);
  Qw_.reserve(m_ * (int64_t)cap_L_, st_);
  hctr_[0] = step_id;
  hctr_[1] = attempt;
  MC_HIP(hipMemcpyAsync(ctr_.p, hctr_, 2 * sizeof(uint32_t), hipMemcpyHostToDevice, st_));
  call_.k = k;
  call_.b = b;
  call_.p_eff = p_eff;
  call_.Lw = Lw;
  call_.guarded = guarded;
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::fresh_launch(int k, int p, uint32_t step_id, uint32_t attempt,
                                      bool guarded) {
  fresh_begin(k, p, step_id, attempt, guarded);
  const Call c = call_;
  if (graphs_ok(c.Lw, k)) {
    const GraphKey key{power_ ? 4 : 1, k, c.b, c.p_eff, c.Lw, (int64_t)gen_,
                       (int64_t)(intptr_t)Qw_.p, guarded ? 1 : 0};
    run_graph(key, [&] { fresh_body(k, c.b, c.p_eff, c.Lw, guarded); });
  } else {
    fresh_body(k, c.b, c.p_eff, c.Lw, guarded);
  }
  fresh_end();
}

template <class P, class VT, class AT>
bool SolverT<P, VT, AT>::fresh_group_stage(int t, std::vector<SpmmTask>* sink) {
  MC_REQUIRE(!power_, kEINVAL, "grouped stepping runs rSVD-BKI only");
  sink_ = group_kind() >= 0 ? sink : nullptr;   // BF16 mode launches its own
  struct Reset {
    std::vector<SpmmTask>*& s;
    ~Reset() { s = nullptr; }
  } reset{sink_};
  return fresh_stage(t, call_.k, call_.b, call_.p_eff, call_.Lw, call_.guarded);
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::fresh_end() {
  const int k = call_.k, Lw = call_.Lw;
  last_guarded_ = call_.guarded;
  k_last_ = k;
  read_launch(k, false, true);
  if (prm_.recycle == 1) {
    swap_buf(Qw_, basis_);
    basis_ld_ = Lw;
    basis_cols_ = Lw;
  } else if (prm_.recycle == 2) {
    if (basis_.n < (size_t)(m_ * (int64_t)k)) basis_.reserve(m_ * (int64_t)cap_k_, st_);
    MC_HIP(hipMemcpyAsync(basis_.p, U_.p, m_ * (int64_t)k * sizeof(P),
                          hipMemcpyDeviceToDevice, st_));
    basis_ld_ = k;
    basis_cols_ = k;
  }
  q_ = 0;
}

template <class P, class VT, class AT>
bool SolverT<P, VT, AT>::fresh_finish(int k) {
  read_finish(k, false);
  const int sc = (int)hbuf_[k];
  const bool redo = !last_guarded_ && sc != shifts_seen_;
  shifts_seen_ = sc;
  return !redo;
}

// Recycled SVD from the saved basis (Sec. IV.B); the finish returns the
// worst Ritz ratio when the guard is on (else 0).
template <class P, class VT, class AT>
void SolverT<P, VT, AT>::recycled_launch(int k) {
  const int w = basis_cols_;
  ensure(std::min<int>(k + prm_.s, (int)std::min(m_, n_)), w, k);
  const bool ritz = prm_.ritz_tol > 0;
  auto body = [&] {
    eig_body(basis_.p, basis_ld_, w, k);
    if (ritz) ritz_body(k);
  };
  if (graphs_ok(w, k)) {
    const GraphKey key{2, k, w, (int)basis_ld_, ritz ? 1 : 0, (int64_t)gen_,
                       (int64_t)(intptr_t)basis_.p, 0};
    run_graph(key, body);
  } else {
    body();
  }
  k_last_ = k;
  read_launch(k, ritz);
}

template <class P, class VT, class AT>
double SolverT<P, VT, AT>::recycled_finish(int k) {
  return read_finish(k, prm_.ritz_tol > 0);
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::sddmm_launch(int r) {
  double* hs = hbuf_ + hbuf_n_ / 2;
  for (int j = 0; j < r; ++j) hs[j] = sig_host_[j];
  if (r > 0)
    MC_HIP(hipMemcpyAsync(sig_.p, hs, r * sizeof(double), hipMemcpyHostToDevice, st_));
  // bytes: row, col, invperm (4 each), M, Y master in and out (8 each), the
  // operator copies of Y (VT each, two when VT is not the master), and the
  // r-wide factor rows of U and V
  const double vbytes = (kMaster ? sizeof(VT) : 2.0 * sizeof(VT)) +
                        (kSplit ? 2.0 * sizeof(P) : 0.0);
  prof.begin(kProfSddmm, (double)nnz_ * (3 * 4 + 3 * 8 + vbytes) +
                             (double)sizeof(P) * (m_ + n_) * r,
             2.0 * nnz_ * r, st_);
  launch_sddmm_update<P, AT, VT, P>(L_, mvals_.p, y_.p, kMaster ? nullptr : yv_.p,
                                    ycv_.p, kSplit ? yw_.p : nullptr,
                                    kSplit ? ycw_.p : nullptr, U_.p, k_last_, V_.p,
                                    k_last_, sig_.p, r, prm_.delta, 1, sdd_part_.p,
                                    hbuf_, st_);       // the residual sum straight to the host
  prof.end(st_);
}

template <class P, class VT, class AT>
double SolverT<P, VT, AT>::sddmm_finish() {
  return hbuf_[0];
}

namespace {
// The first `cols` columns of a row-major device panel into the caller's
// (pageable) host array: one contiguous copy into library-owned host memory,
// then the columns are picked and widened on the host.
template <class P>
void copy_cols_to_host(double* dst, int64_t ldd, const P* src, int64_t lds_,
                       int cols, int64_t rows, hipStream_t st) {
  std::vector<P> tmp((size_t)rows * lds_);
  MC_HIP(hipMemcpyAsync(tmp.data(), src, tmp.size() * sizeof(P),
                        hipMemcpyDeviceToHost, st));
  MC_HIP(hipStreamSynchronize(st));
  for (int64_t i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) dst[i * ldd + j] = (double)tmp[i * lds_ + j];
}
}  // namespace

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::get_factors(double* U, double* sig, double* V,
                                     int64_t ldu, int64_t ldv) {
  const int r = r_;
  if (r > 0) {
    if (U) copy_cols_to_host(U, ldu, U_.p, k_last_, r, m_, st_);
    if (V) copy_cols_to_host(V, ldv, V_.p, k_last_, r, n_, st_);
  }
  MC_HIP(hipStreamSynchronize(st_));
  if (sig) for (int j = 0; j < r; ++j) sig[j] = sig_host_[j];
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::get_rsvd(double* U, double* S, double* V) {
  const int k = k_last_;
  if (U) copy_cols_to_host(U, k, U_.p, k, k, m_, st_);
  if (V) copy_cols_to_host(V, k, V_.p, k, k, n_, st_);
  for (int j = 0; j < k; ++j) S[j] = lastS_[j];
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::get_observed(double* x_phi) {
  obs_.reserve(nnz_, st_);
  if (r_ == 0) {
    MC_HIP(hipMemsetAsync(obs_.p, 0, nnz_ * sizeof(double), st_));
  } else {
    for (int j = 0; j < r_; ++j) hbuf_[j] = sig_host_[j];
    MC_HIP(hipMemcpyAsync(sig_.p, hbuf_, r_ * sizeof(double), hipMemcpyHostToDevice, st_));
    launch_eval_observed<P>(L_, U_.p, k_last_, V_.p, k_last_, sig_.p, r_, obs_.p, st_);
  }
  MC_HIP(hipMemcpyAsync(x_phi, obs_.p, nnz_ * sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
}

template <class P, class VT, class AT>
void SolverT<P, VT, AT>::get_y(double* y_host) {
  obs_.reserve(nnz_, st_);
  launch_scatter(nnz_, L_.order.p, y_.p, obs_.p, st_);
  MC_HIP(hipMemcpyAsync(y_host, obs_.p, nnz_ * sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
}

}  // namespace

std::unique_ptr<Solver> make_solver(int64_t m, int64_t n, int64_t nnz,
                                    const mc_svt_params& prm, hipStream_t st) {
  switch (prm.precision) {
    case MC_FP32_EIG64:
      return std::unique_ptr<Solver>(new SolverT<float, float, float>(m, n, nnz, prm, st));
    case MC_BF16_EIG64:
      return std::unique_ptr<Solver>(new SolverT<float, bf16_t, float>(m, n, nnz, prm, st));
    default:
      return std::unique_ptr<Solver>(new SolverT<double, double, double>(m, n, nnz, prm, st));
  }
}

}  // namespace mcsvt
