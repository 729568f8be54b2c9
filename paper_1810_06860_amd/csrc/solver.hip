// Fast SVT (Alg. 6) driven from the host over the device kernels.
//
// One step:
//   k = r + 1; adjust p (Sec. IV.C)
//   repeat
//     fresh rSVD-BKI (Alg. 5) when i < i_reuse, q == q_reuse or there is no
//     usable basis; otherwise recycle the last call's Q (strategy 1) or U
//     (strategy 2) (Sec. IV.B), optionally checked by the Ritz residual
//   until the k-th singular value <= tau (k += l otherwise)
//   r = #{S_j > tau}; fused SDDMM: residual on Phi and Y += delta P_Phi(M - X)
//
// rSVD-BKI on the device:
//   Omega (n x b) Gaussian; H_0 = Y Omega; for j = 1..p: H_j = Y (Y^T Q_{j-1});
//   each H_j is orthonormalised against Q_0..Q_{j-1} by block Gram-Schmidt
//   with re-orthogonalisation and Cholesky QR (two passes each), which
//   spans the same subspace as the LU-normalised blocks followed by orth()
//   (Lemmas 2 and 3), so Q = [Q_0 .. Q_p] is already orthonormal;
//   B^T = Y^T Q; eigSVD(B^T): G = B B^T, eig(G), top k, S = sqrt(lambda),
//   U = Q W_k, V = B^T W_k S^-1.
#include "solver.hpp"

#include <cmath>
#include <cstring>
#include <utility>

namespace mcsvt {

namespace {
template <class T>
void swap_buf(DevBuf<T>& a, DevBuf<T>& b) {
  std::swap(a.p, b.p);
  std::swap(a.n, b.n);
  std::swap(a.stream, b.stream);
}
}  // namespace

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
  shift_count_.reserve(1, st_);
  blk_flag_.reserve(1, st_);
  ctr_.reserve(2, st_);
  MC_HIP(hipHostMalloc((void**)&hctr_, 2 * sizeof(uint32_t)));
  MC_HIP(hipMemsetAsync(shift_count_.p, 0, sizeof(int), st_));
}

Solver::~Solver() {
  clear_graphs();
  if (cap_) (void)hipStreamDestroy(cap_);
  if (hbuf_) (void)hipHostFree(hbuf_);
  if (hctr_) (void)hipHostFree(hctr_);
}

int Solver::chol_shifts() {
  int v = 0;
  MC_HIP(hipMemcpyAsync(&v, shift_count_.p, sizeof(int), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
  return v;
}

void Solver::widths(int k, int p, int& b, int& p_eff) const {
  const int64_t mn = std::min(m_, n_);
  b = (int)std::min<int64_t>((int64_t)k + prm_.s, mn);
  p_eff = (int)std::max<int64_t>(0, std::min<int64_t>(p, mn / b - 1));
}

void Solver::ensure(int bmax, int Lmax, int kmax) {
  if (bmax <= cap_b_ && Lmax <= cap_L_ && kmax <= cap_k_ && hbuf_) return;
  // buffers move: captured graphs hold their addresses
  ++gen_;
  clear_graphs();
  const int64_t mn = std::min(m_, n_);
  // grow with headroom so the rank search does not reallocate every step
  auto grow = [&](int want, int have) {
    if (want <= have) return have;
    return (int)std::min<int64_t>(mn, std::max<int64_t>(want, (int64_t)have * 5 / 4 + 8));
  };
  cap_b_ = std::max(grow(bmax, cap_b_), bmax);
  cap_L_ = std::max(grow(Lmax, cap_L_), Lmax);
  cap_k_ = std::max(grow(kmax, cap_k_), kmax);
  const int64_t b = cap_b_, Lc = cap_L_, k = cap_k_;
  const int64_t wide = std::max({b, Lc, k});
  omega_.reserve(n_ * b, st_);
  Qw_.reserve(m_ * Lc, st_);
  H1_.reserve(m_ * std::max(b, k), st_);
  H2_.reserve(m_ * b, st_);
  Z_.reserve(n_ * b, st_);
  Bt_.reserve(n_ * Lc, st_);
  G_.reserve(Lc * Lc, st_);
  Cg_.reserve(Lc * b, st_);
  Rinv_.reserve(b * b, st_);
  chol_work_.reserve(b * b, st_);
  const int64_t mx = std::max(m_, n_);
  gram_cap_ = std::max({gram_splits(mx, (int)Lc, (int)Lc, 1) * Lc * Lc,
                        gram_splits(m_, (int)b, (int)b, 1) * b * b,
                        gram_splits(m_, (int)Lc, (int)b, 0) * Lc * b});
  gram_part_.reserve(gram_cap_, st_);
  const int64_t slots = std::max(L_.sched_csr.nslot, L_.sched_csc.nslot);
  spmm_part_.reserve(std::max<int64_t>(1, slots) * wide, st_);
  U_.reserve(m_ * k, st_);
  V_.reserve(n_ * k, st_);
  S_.reserve(k, st_);
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
    MC_HIP(hipHostMalloc((void**)&hbuf_, need * sizeof(double)));
    hbuf_n_ = need;
  }
}

int Solver::init(const int64_t* rows, const int32_t* cols, const double* vals,
                 bool scale_for_svt) {
  DevBuf<int64_t> d_rows;
  DevBuf<int32_t> d_cols;
  DevBuf<double> d_vals;
  d_rows.reserve(nnz_, st_);
  d_cols.reserve(nnz_, st_);
  d_vals.reserve(nnz_, st_);
  MC_HIP(hipMemcpyAsync(d_rows.p, rows, nnz_ * sizeof(int64_t), hipMemcpyHostToDevice, st_));
  MC_HIP(hipMemcpyAsync(d_cols.p, cols, nnz_ * sizeof(int32_t), hipMemcpyHostToDevice, st_));
  MC_HIP(hipMemcpyAsync(d_vals.p, vals, nnz_ * sizeof(double), hipMemcpyHostToDevice, st_));
  const int status = build_layout(m_, n_, nnz_, d_rows.p, d_cols.p, d_vals.p, L_, st_);
  if (status != kOK) return status;
  mvals_.reserve(nnz_, st_);
  y_.reserve(nnz_, st_);
  ycsc_.reserve(nnz_, st_);
  launch_gather(nnz_, L_.order.p, d_vals.p, mvals_.p, st_);
  ensure(1, 1, 1);
  sdd_part_.reserve(sddmm_partials(nnz_), st_);
  scal_.reserve(8, st_);
  launch_sumsq(nnz_, mvals_.p, sdd_part_.p, scal_.p, st_);
  MC_HIP(hipMemcpyAsync(hbuf_, scal_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
  mnorm_ = std::sqrt(hbuf_[0]);
  MC_REQUIRE(std::isfinite(mnorm_), kEINVAL, "non-finite value in M_Phi");
  MC_HIP(hipMemcpyAsync(y_.p, mvals_.p, nnz_ * sizeof(double), hipMemcpyDeviceToDevice, st_));
  launch_gather(nnz_, L_.perm.p, mvals_.p, ycsc_.p, st_);
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
    const double a = c_ * prm_.delta;
    launch_scale(nnz_, mvals_.p, a, y_.p, st_);
    launch_scale(nnz_, ycsc_.p, a, ycsc_.p, st_);
    basis_cols_ = 0;
    k_last_ = 0;
    lastS_.clear();
  }
  MC_HIP(hipStreamSynchronize(st_));
  return kOK;
}

// algorithmic bytes of one SpMM: values + indices + pointers + panel in + out
static double spmm_bytes(int64_t nnz, int64_t rows, int64_t cols, int b, int sv,
                         int sx) {
  return (double)nnz * (sv + 4) + 4.0 * (rows + 1) + (double)cols * b * sx +
         (double)rows * b * sx;
}

void Solver::spmm_y(const double* X, int64_t ldx, double* out, int64_t ldo, int b) {
  prof.begin(kProfSpmmFwd, spmm_bytes(nnz_, m_, n_, b, 8, 8), 2.0 * nnz_ * b, ls());
  launch_spmm<double, double, double, double>(L_.sched_csr, L_.col_idx.p, y_.p, X,
                                              ldx, out, ldo, b, spmm_part_.p, ls());
  prof.end(ls());
}

void Solver::spmm_yt(const double* X, int64_t ldx, double* out, int64_t ldo, int b) {
  prof.begin(kProfSpmmBwd, spmm_bytes(nnz_, n_, m_, b, 8, 8), 2.0 * nnz_ * b, ls());
  launch_spmm<double, double, double, double>(L_.sched_csc, L_.row_idx.p, ycsc_.p,
                                              X, ldx, out, ldo, b, spmm_part_.p,
                                              ls());
  prof.end(ls());
}

void Solver::cholqr_pass(const double* Hin, int64_t ldin, double* out,
                         int64_t ldo, int b, const int* gate) {
  prof.begin(kProfGram, 8.0 * m_ * b, 1.0 * m_ * b * (b + 1), ls());
  launch_gram<double, double>(m_, b, b, Hin, ldin, Hin, ldin, G_.p, b, 1,
                              gram_part_.p, gram_cap_, ls(), gate);
  prof.end(ls());
  prof.begin(kProfChol, 16.0 * b * b, b * (double)b * b, ls());
  launch_chol_inv(b, G_.p, b, Rinv_.p, b, chol_work_.p, m_, shift_count_.p, ls(),
                  blk_flag_.p, gate);
  prof.end(ls());
  prof.begin(kProfGemm, 16.0 * m_ * b, 2.0 * m_ * b * b, ls());
  launch_panel_gemm<double, double>(m_, b, b, Hin, ldin, Rinv_.p, b, 1.0,
                                    nullptr, 0.0, nullptr, 0, out, ldo, ls(), gate);
  prof.end(ls());
}

// Hout = Hin - Qp (Qp^T Hin) with Qp = the first jb columns of Qw_
void Solver::project(const double* Hin, int64_t ldin, double* Hout, int jb, int b,
                     int Lw, const int* gate) {
  prof.begin(kProfGram, 8.0 * m_ * (jb + b), 2.0 * m_ * jb * b, ls());
  launch_gram<double, double>(m_, jb, b, Qw_.p, Lw, Hin, ldin, Cg_.p, b, 0,
                              gram_part_.p, gram_cap_, ls(), gate);
  prof.end(ls());
  prof.begin(kProfGemm, 8.0 * m_ * (jb + 2 * b), 2.0 * m_ * jb * b, ls());
  launch_panel_gemm<double, double>(m_, jb, b, Qw_.p, Lw, Cg_.p, b, -1.0, nullptr,
                                    1.0, Hin, ldin, Hout, b, ls(), gate);
  prof.end(ls());
}

// Orthonormalise the raw Krylov block in H1_ against Q_0..Q_{j-1} and write
// it to columns [j b, (j+1) b) of Qw_: block Gram-Schmidt + Cholesky QR, two
// passes, and a third one only when a Cholesky factorisation needed a shift
// (the device flag gates it; no host round trip).
void Solver::orth_block(int j, int b, int Lw) {
  double* out = Qw_.p + (int64_t)j * b;
  const int* gate = blk_flag_.p;
  launch_set_int(blk_flag_.p, 0, ls());
  if (j == 0) {
    cholqr_pass(H1_.p, b, H2_.p, b, b, nullptr);
    cholqr_pass(H2_.p, b, out, Lw, b, nullptr);
    cholqr_pass(out, Lw, H1_.p, b, b, gate);
    launch_copy_gated(m_, b, H1_.p, b, out, Lw, gate, ls());
    return;
  }
  const int jb = j * b;
  project(H1_.p, b, H2_.p, jb, b, Lw, nullptr);
  cholqr_pass(H2_.p, b, H1_.p, b, b, nullptr);
  project(H1_.p, b, H2_.p, jb, b, Lw, nullptr);
  cholqr_pass(H2_.p, b, out, Lw, b, nullptr);
  project(out, Lw, H2_.p, jb, b, Lw, gate);
  cholqr_pass(H2_.p, b, H1_.p, b, b, gate);
  launch_copy_gated(m_, b, H1_.p, b, out, Lw, gate, ls());
}

// S (k values) and, with the Ritz guard, the k Ritz ratios: one round trip
double Solver::read_results(int k, bool ritz) {
  MC_HIP(hipMemcpyAsync(hbuf_, S_.p, k * sizeof(double), hipMemcpyDeviceToHost, st_));
  if (ritz)
    MC_HIP(hipMemcpyAsync(hbuf_ + k, ritz_out_.p, k * sizeof(double),
                          hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
  lastS_.assign(hbuf_, hbuf_ + k);
  for (double v : lastS_)
    MC_REQUIRE(std::isfinite(v), kENUMERIC, "non-finite singular value");
  double worst = 0.0;
  if (ritz)
    for (int j = 0; j < k; ++j) worst = std::max(worst, hbuf_[k + j]);
  return worst;
}

// eigSVD of B^T = Y^T basis (Alg. 3 on B^T, Alg. 5 steps 8-10): kernels only
void Solver::eig_body(const double* basis, int64_t ldb, int w, int k) {
  spmm_yt(basis, ldb, Bt_.p, w, w);                          // B^T = Y^T basis
  prof.begin(kProfGram, 8.0 * n_ * w, 1.0 * n_ * w * (w + 1), ls());
  launch_gram<double, double>(n_, w, w, Bt_.p, w, Bt_.p, w, G_.p, w, 1,
                              gram_part_.p, gram_cap_, ls()); // G = B B^T
  prof.end(ls());
  prof.begin(kProfEig, 16.0 * w * w, 0.0, ls());
  eig_.solve_topk(w, G_.p, w, k, S_.p, D_.p, Wk_.p, k, ls());
  prof.end(ls());
  prof.begin(kProfGemm, 8.0 * (m_ + n_) * (w + k), 2.0 * (m_ + n_) * w * k, ls());
  launch_panel_gemm<double, double>(m_, w, k, basis, ldb, Wk_.p, k, 1.0, nullptr,
                                    0.0, nullptr, 0, U_.p, k, ls());  // U = Q W
  launch_recip(k, S_.p, Sinv_.p, ls());
  launch_panel_gemm<double, double>(n_, w, k, Bt_.p, w, Wk_.p, k, 1.0, Sinv_.p,
                                    0.0, nullptr, 0, V_.p, k, ls());  // V = B^T W S^-1
  prof.end(ls());
}

// Ritz residual ratios ||Y v_j - s_j u_j|| / s_j into ritz_out_
void Solver::ritz_body(int k) {
  spmm_y(V_.p, k, H1_.p, k, k);                              // R = Y V
  launch_ritz(m_, k, H1_.p, k, U_.p, k, S_.p, ritz_part_.p, ritz_out_.p, ls());
}

void Solver::fresh_body(int k, int b, int p_eff, int Lw) {
  prof.begin(kProfRng, 8.0 * n_ * b, 0.0, ls());
  launch_gaussian_ctr<double>(omega_.p, n_, b, b, prm_.seed, ctr_.p, ls());
  prof.end(ls());
  spmm_y(omega_.p, b, H1_.p, b, b);                          // H_0 = Y Omega
  orth_block(0, b, Lw);
  for (int j = 1; j <= p_eff; ++j) {
    spmm_yt(Qw_.p + (int64_t)(j - 1) * b, Lw, Z_.p, b, b);   // Y^T Q_{j-1}
    spmm_y(Z_.p, b, H1_.p, b, b);                            // H_j
    orth_block(j, b, Lw);
  }
  eig_body(Qw_.p, Lw, Lw, k);
}

bool Solver::graphs_ok(int w) const {
  return prm_.use_graphs && !prof.on && w <= EigSolver::single_max();
}

template <class F>
void Solver::run_graph(const GraphKey& key, F&& body) {
  auto it = graphs_.find(key);
  if (it == graphs_.end()) {
    if (!cap_) MC_HIP(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
    if (graphs_.size() >= 64) clear_graphs();
    hipGraph_t g = nullptr;
    MC_HIP(hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal));
    capturing_ = true;
    try {
      body();
    } catch (...) {
      capturing_ = false;
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(cap_, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      throw;
    }
    capturing_ = false;
    MC_HIP(hipStreamEndCapture(cap_, &g));
    hipGraphExec_t ge = nullptr;
    const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    MC_HIP(e);
    it = graphs_.emplace(key, ge).first;
  }
  MC_HIP(hipGraphLaunch(it->second, st_));
}

void Solver::clear_graphs() {
  for (auto& kv : graphs_) (void)hipGraphExecDestroy(kv.second);
  graphs_.clear();
}

void Solver::fresh_svd(int k, int p, uint32_t step_id, uint32_t attempt) {
  int b, p_eff;
  widths(k, p, b, p_eff);
  const int Lw = (p_eff + 1) * b;
  ensure(b, Lw, k);
  Qw_.reserve(m_ * (int64_t)cap_L_, st_);
  hctr_[0] = step_id;
  hctr_[1] = attempt;
  MC_HIP(hipMemcpyAsync(ctr_.p, hctr_, 2 * sizeof(uint32_t), hipMemcpyHostToDevice, st_));
  if (graphs_ok(Lw)) {
    const GraphKey key{1, k, b, p_eff, Lw, (int64_t)gen_, (int64_t)(intptr_t)Qw_.p, 0};
    run_graph(key, [&] { fresh_body(k, b, p_eff, Lw); });
  } else {
    fresh_body(k, b, p_eff, Lw);
  }
  k_last_ = k;
  read_results(k, false);
  if (prm_.recycle == 1) {
    swap_buf(Qw_, basis_);
    basis_ld_ = Lw;
    basis_cols_ = Lw;
  } else if (prm_.recycle == 2) {
    if (basis_.n < (size_t)(m_ * (int64_t)k)) basis_.reserve(m_ * (int64_t)cap_k_, st_);
    MC_HIP(hipMemcpyAsync(basis_.p, U_.p, m_ * (int64_t)k * sizeof(double),
                          hipMemcpyDeviceToDevice, st_));
    basis_ld_ = k;
    basis_cols_ = k;
  }
  q_ = 0;
}

// Recycled SVD from the saved basis (Sec. IV.B); returns the worst Ritz
// ratio when the guard is on (else 0).
double Solver::recycled_svd(int k) {
  const int w = basis_cols_;
  ensure(std::min<int>(k + prm_.s, (int)std::min(m_, n_)), w, k);
  const bool ritz = prm_.ritz_tol > 0;
  auto body = [&] {
    eig_body(basis_.p, basis_ld_, w, k);
    if (ritz) ritz_body(k);
  };
  if (graphs_ok(w)) {
    const GraphKey key{2, k, w, (int)basis_ld_, ritz ? 1 : 0, (int64_t)gen_,
                       (int64_t)(intptr_t)basis_.p, 0};
    run_graph(key, body);
  } else {
    body();
  }
  k_last_ = k;
  return read_results(k, ritz);
}

void Solver::rsvd(int k, int p, uint32_t step_id, uint32_t attempt) {
  fresh_svd(k, p, step_id, attempt);
}

StepInfo Solver::step() {
  MC_REQUIRE(!converged_, kEDONE, "the solve has already converged");
  StepInfo info;
  ++i_;
  int k = std::min(r_ + 1, kcap_);
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
  uint32_t attempt = 0;
  while (true) {
    bool use_fresh = prm_.recycle == 0 || i_ < prm_.i_reuse ||
                     q_ == prm_.q_reuse || basis_cols_ == 0 || k > basis_cols_;
    if (!use_fresh) {
      const double ratio = recycled_svd(k);
      ++q_;
      ++info.recycled;
      if (prm_.ritz_tol > 0 && ratio > prm_.ritz_tol) {
        use_fresh = true;
        ++info.rejected;
      }
    }
    if (use_fresh) {
      fresh_svd(k, p_, (uint32_t)i_, attempt++);
      ++info.fresh;
    }
    if (lastS_[k - 1] <= prm_.tau || k >= kcap_) break;
    k = std::min(k + prm_.l, kcap_);
  }
  int r = 0;
  while (r < k && lastS_[r] > prm_.tau) ++r;
  r_ = r;
  sig_host_.assign(r, 0.0);
  double* hs = hbuf_ + hbuf_n_ / 2;
  for (int j = 0; j < r; ++j) hs[j] = sig_host_[j] = lastS_[j] - prm_.tau;
  if (r > 0)
    MC_HIP(hipMemcpyAsync(sig_.p, hs, r * sizeof(double), hipMemcpyHostToDevice, st_));
  // bytes: row, col, invperm (4 each), M, Y in, Y out, Y^T out (8 each), and
  // the r-wide factor rows of U and V
  prof.begin(kProfSddmm, (double)nnz_ * (3 * 4 + 4 * 8) + 8.0 * (m_ + n_) * r,
             2.0 * nnz_ * r, st_);
  launch_sddmm_update<double>(L_, mvals_.p, y_.p, ycsc_.p, U_.p, k_last_, V_.p,
                              k_last_, sig_.p, r, prm_.delta, 1, sdd_part_.p,
                              scal_.p, st_);
  prof.end(st_);
  MC_HIP(hipMemcpyAsync(hbuf_, scal_.p, sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
  const double res = std::sqrt(hbuf_[0]) / mnorm_;
  MC_REQUIRE(std::isfinite(res), kENUMERIC, "non-finite residual");
  err_hist_.push_back(res);
  fresh_total_ += info.fresh;
  recycled_total_ += info.recycled;
  rejected_total_ += info.rejected;
  converged_ = res < prm_.eps;
  info.i = i_;
  info.r = r;
  info.k = k;
  info.p = p_;
  info.res = res;
  info.converged = converged_ ? 1 : 0;
  info.sigma_max = lastS_.empty() ? 0.0 : lastS_[0];
  return info;
}

void Solver::get_factors(double* U, double* sig, double* V, int64_t ldu,
                         int64_t ldv) {
  const int r = r_;
  if (r > 0) {
    if (U)
      MC_HIP(hipMemcpy2DAsync(U, ldu * sizeof(double), U_.p, k_last_ * sizeof(double),
                              r * sizeof(double), m_, hipMemcpyDeviceToHost, st_));
    if (V)
      MC_HIP(hipMemcpy2DAsync(V, ldv * sizeof(double), V_.p, k_last_ * sizeof(double),
                              r * sizeof(double), n_, hipMemcpyDeviceToHost, st_));
  }
  MC_HIP(hipStreamSynchronize(st_));
  if (sig) for (int j = 0; j < r; ++j) sig[j] = sig_host_[j];
}

void Solver::get_rsvd(double* U, double* S, double* V) {
  const int k = k_last_;
  MC_HIP(hipMemcpyAsync(U, U_.p, m_ * (int64_t)k * sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipMemcpyAsync(V, V_.p, n_ * (int64_t)k * sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
  for (int j = 0; j < k; ++j) S[j] = lastS_[j];
}

void Solver::get_observed(double* x_phi) {
  obs_.reserve(nnz_, st_);
  if (r_ == 0) {
    MC_HIP(hipMemsetAsync(obs_.p, 0, nnz_ * sizeof(double), st_));
  } else {
    launch_eval_observed<double>(L_, U_.p, k_last_, V_.p, k_last_, sig_.p, r_,
                                 obs_.p, st_);
  }
  MC_HIP(hipMemcpyAsync(x_phi, obs_.p, nnz_ * sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
}

void Solver::get_y(double* y_host) {
  obs_.reserve(nnz_, st_);
  launch_scatter(nnz_, L_.order.p, y_.p, obs_.p, st_);
  MC_HIP(hipMemcpyAsync(y_host, obs_.p, nnz_ * sizeof(double), hipMemcpyDeviceToHost, st_));
  MC_HIP(hipStreamSynchronize(st_));
}

size_t footprint_bytes(int64_t m, int64_t n, int64_t nnz, const mc_svt_params& p) {
  const int64_t mn = std::min(m, n);
  int64_t k = p.k_max > 0 ? std::min<int64_t>(p.k_max, mn) : std::min<int64_t>(mn, 256);
  const int64_t b = std::min<int64_t>(k + std::max(p.s, 10), mn);
  const int64_t L = std::min<int64_t>((int64_t)(p.p_max + 1) * b, mn);
  const int64_t Lp = round_up(L, 32);
  const int64_t mx = std::max(m, n);
  size_t bytes = 0;
  bytes += (size_t)nnz * (8 * 3 + 4 * 6);                 // values + layout
  bytes += (size_t)(m + n + 2) * 4 + (size_t)(m + n) * 16; // pointers + schedules
  bytes += (size_t)8 * (n * b + 2 * m * L + m * std::max(b, k) + m * b + n * b +
                        n * L + L * L + L * b + 2 * b * b + m * k + n * k +
                        L * k + 4 * L);
  bytes += (size_t)8 * (gram_splits(mx, (int)L, (int)L, 1) * L * L);
  bytes += (size_t)8 * (3 * Lp * Lp);
  bytes += (size_t)8 * (mx * L / 4 + ceil_div(nnz, 256) + nnz);
  return bytes;
}

}  // namespace mcsvt
