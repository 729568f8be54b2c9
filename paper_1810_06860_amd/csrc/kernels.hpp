// Internal declarations: device layouts and kernel launchers.
#pragma once

#include <algorithm>
#include <vector>

#include "common.hpp"

namespace mcsvt {

// Work schedule of a CSR-like structure for the segmented SpMM:
// segs[w] = (row, begin, end, slot) with slot = -1 for whole rows, and
// fix[f] = (row, first_slot, count, 0) for rows split into several segments.
// A segment with row -1 is padding and does nothing.
//
// Structures whose gathered dimension (the rows of the dense panel) is large
// also get a banded form: the gathered rows are cut into kBands equal ranges,
// long rows are split at the range boundaries, and the pieces of range r go
// to workgroups r, r + kBands, r + 2 kBands, ...; the hardware hands
// consecutive workgroups to the eight XCDs in turn, so each XCD's caches see
// one range of the panel instead of all of it.  Only rows long enough that
// their band pieces stay near the segment length are split (band_split_len),
// so the banded form has about as many segments as the plain one.  Narrow
// panels take it whenever the panel is large; wide panels when a good share
// of the entries lies in split rows (without such rows the form only
// reorders whole rows across the XCDs, which gives them no locality).
constexpr int kBands = 8;
constexpr int kSpmmWaves = 4;                      // wavefronts per SpMM workgroup
constexpr int64_t kBandMinRows = 8192;             // gathered rows for a banded form
constexpr int64_t kBandPanelBytes = 2 << 20;       // smaller panels stay unbanded
constexpr int kBandWide = 128;                     // wider panels need split rows
// shortest row the banded form splits, for segments of at most `cap` entries
inline int64_t band_split_len(int64_t cap) { return cap * 4 > 256 ? cap * 4 : 256; }
// segment length of the work schedules of a structure with nnz entries: about
// 16K segments in flight fill the chip (256 CUs x several waves), capped so
// long rows of power-law matrices are split
inline int64_t spmm_segment_cap(int64_t nnz) {
  return std::min<int64_t>(1024, std::max<int64_t>(64, ceil_div(nnz, 16384)));
}
// upper bound of the partial rows of either schedule form: a row split in the
// plain form (len > cap) has ceil(len / cap) < 2 len / cap pieces, one split
// at the bands (len >= 4 cap) at most len / cap + kBands <= 3 len / cap
inline int64_t spmm_slot_bound(int64_t nnz) {
  return 3 * ceil_div(nnz, spmm_segment_cap(nnz));
}
struct Schedule {
  int64_t nseg = 0, nfix = 0;
  int64_t nslot = 0;                           // partial rows, either form
  DevBuf<int4> segs;
  DevBuf<int4> fix;
  int64_t gathered = 0;                        // rows of the gathered panel
  bool long_share = false;                     // >= 1/4 of nnz in rows the bands split
  int64_t band_nseg = 0, band_nfix = 0;        // banded form; 0 if not built
  DevBuf<int4> band_segs;
  DevBuf<int4> band_fix;
};

// Canonical layout of the sampled set Phi.
struct Layout {
  int64_t m = 0, n = 0, nnz = 0;
  DevBuf<int32_t> row_ptr;   // m + 1
  DevBuf<int32_t> col_idx;   // nnz, CSR order
  DevBuf<int32_t> row_of;    // nnz, row of each CSR entry
  DevBuf<int32_t> order;     // nnz, CSR position -> input position
  DevBuf<int32_t> col_ptr;   // n + 1
  DevBuf<int32_t> row_idx;   // nnz, CSC order
  DevBuf<int32_t> perm;      // nnz, CSC position -> CSR position
  DevBuf<int32_t> invperm;   // nnz, CSR position -> CSC position
  Schedule sched_csr, sched_csc;
};

int build_layout(int64_t m, int64_t n, int64_t nnz, const int64_t* d_rows,
                 const int32_t* d_cols, const double* d_vals, Layout& L,
                 hipStream_t st);
// COO row ids (nnz) of a device CSR row pointer (m + 1); returns kEINVAL when
// the pointer does not start at 0, end at nnz and never decrease
int csr_rows_device(int64_t m, int64_t nnz, const int64_t* d_ptr, int64_t* d_rows,
                    hipStream_t st);
// The banded segments and fix-up records of a host CSR-like structure (host
// code only; build_schedule uploads them).
void band_schedule(const int32_t* ptr, const int32_t* idx, int64_t rows,
                   int64_t gathered, int64_t cap, int nb, std::vector<int4>& segs,
                   std::vector<int4>& fix, int32_t& slot);
// host_idx (the gathered index of every entry, sorted within each row) may
// be null: then no banded form is built
void build_schedule(const int32_t* host_ptr, int64_t rows, Schedule& S,
                    hipStream_t st, const int32_t* host_idx = nullptr,
                    int64_t gathered = 0);

template <class S, class D>
void launch_cast(int64_t n, const S* src, D* dst, hipStream_t st);
template <class T>
void launch_gather(int64_t nnz, const int32_t* idx, const T* src, T* dst,
                   hipStream_t st);
template <class T>
void launch_scatter(int64_t nnz, const int32_t* idx, const T* src, T* dst,
                    hipStream_t st);

template <class T>
void launch_gaussian(T* out, int64_t rows, int64_t cols, int64_t ld,
                     uint64_t seed, uint32_t step, uint32_t attempt,
                     hipStream_t st);

template <class T>
void launch_gaussian_ctr(T* out, int64_t rows, int64_t cols, int64_t ld,
                         uint64_t seed, const uint32_t* d_ctr, hipStream_t st);

// out (rows x b, ldo) = A X ; A given by schedule + idx + val; part is the
// partial-row buffer (nslot * b elements).
// One sparse product of a grouped launch (products of several solves in one
// kernel): its schedule (the form launch_spmm would take), operands and, set
// by the launcher, its first workgroup and first fix-up item.
struct SpmmTask {
  const int4* segs;
  int64_t nseg;
  const int4* fix;
  int64_t nfix;
  const int32_t* idx;
  const void* val;
  const void* X;
  int64_t ldx;
  void* out;
  int64_t ldo;
  void* part;
  int64_t b;
  int64_t wg0, fx0;
};
SpmmTask make_spmm_task(const Schedule& S, const int32_t* idx, const void* val,
                        const void* X, int64_t ldx, void* out, int64_t ldo, int b,
                        void* part, size_t x_bytes);
template <class VT, class XT, class AT, class OT>
void launch_spmm_group(const std::vector<SpmmTask>& tasks, SpmmTask* staging,
                       SpmmTask* table, int64_t cap, hipStream_t st);

template <class VT, class XT, class AT, class OT>
void launch_spmm(const Schedule& S, const int32_t* idx, const VT* val,
                 const XT* X, int64_t ldx, OT* out, int64_t ldo, int b,
                 AT* part, hipStream_t st);

int64_t sddmm_partials(const Layout& L);   // residual partial sums of the SDDMM (and of launch_sumsq)
// FT factor type, AT accumulator, VT / WT types of the operator copies of Y
// (Krylov / Rayleigh-Ritz products); null copies are skipped
template <class FT, class AT, class VT, class WT>
void launch_sddmm_update(const Layout& L, const double* mvals, double* y, VT* yv,
                         VT* ycv, WT* yw, WT* ycw, const FT* U, int64_t ldu,
                         const FT* V, int64_t ldv, const double* sig, int r,
                         double delta, int apply, double* partial, double* out_sum,
                         hipStream_t st);   // out_sum: device or pinned host memory
template <class FT>
void launch_eval_observed(const Layout& L, const FT* U, int64_t ldu,
                          const FT* V, int64_t ldv, const double* sig, int r,
                          double* out_input_order, hipStream_t st);
void launch_sumsq(int64_t n, const double* a, double* partial, double* out,
                  hipStream_t st);
void launch_scale(int64_t n, const double* a, double alpha, double* out,
                  hipStream_t st);

// C (p x q, FP64) = A^T B with A (N x p), B (N x q); sym: A == B, p == q.
// gram_splits: the most row splits a launch_gram or launch_gram_fused call of
// that shape uses (its partial buffer holds gram_splits * p * q elements; a
// smaller buffer means fewer splits).
int64_t gram_splits(int64_t N, int p, int q, int sym);
// gate: optional device flag; when it reads 0 the kernels do nothing.
template <class IT, class AT>
void launch_gram(int64_t N, int p, int q, const IT* A, int64_t lda, const IT* B,
                 int64_t ldb, double* C, int64_t ldc, int sym, AT* part,
                 int64_t part_cap, hipStream_t st, const int* gate = nullptr);

// C (FP64) = A^T B for FP32 panels on the BF16 matrix cores (operands rounded
// to BF16, FP32 accumulation), for the shapes gram_bf16_fits accepts (one
// output block of a panel tall enough to stream); partial buffer as
// launch_gram's.
bool gram_bf16_fits(int64_t N, int p, int q, int sym);
void launch_gram_bf16(int64_t N, int p, int q, const float* A, int64_t lda, const float* B,
                      int64_t ldb, double* C, int64_t ldc, int sym, float* part,
                      int64_t part_cap, hipStream_t st);

// The same with the completion in one launch: C (mode "cross", Rinv null), or
// with A = B also Rinv = R^{-1} for C = R^T R (shifted retry as in
// launch_chol_inv).  `counter` is a device int that is 0 between launches.
template <class IT, class AT>
void launch_gram_fused(int64_t N, int p, int q, const IT* A, int64_t lda, const IT* B,
                       int64_t ldb, double* C, int64_t ldc, int sym, AT* part,
                       int64_t part_cap, int* counter, double* Rinv, int64_t ldr,
                       int64_t nrows, int* shifted, int* flag, hipStream_t st,
                       const int* gate = nullptr);

// C = beta C0 + alpha X W diag(colscale)   (colscale may be null)
template <class XT, class OT>
void launch_panel_gemm(int64_t N, int p, int q, const XT* X, int64_t ldx,
                       const double* W, int64_t ldw, double alpha,
                       const double* colscale, double beta, const OT* C0,
                       int64_t ldc0, OT* C, int64_t ldc, hipStream_t st,
                       const int* gate = nullptr);

// The Cholesky factorisation and R^-1 of a b x b Gram matrix work in
// b*b + 3b doubles: in LDS up to this b (134 KB at b = 128)
constexpr int kCholLdsMax = 128;
constexpr int kCholLdsDoubles = kCholLdsMax * kCholLdsMax + 3 * kCholLdsMax;
// flag (optional) is set to 1 when a diagonal shift was needed
// work: b*b + 2b doubles (global), used when b > kCholLdsMax
void launch_chol_inv(int b, const double* G, int64_t ldg, double* Rinv,
                     int64_t ldr, double* work, int64_t nrows, int* shifted,
                     hipStream_t st, int* flag = nullptr,
                     const int* gate = nullptr);
void launch_set_int(int* p, int v, hipStream_t st);
// dst (rows x cols, ldd) = src (rows x cols, lds_) converted to D
template <class S, class D>
void launch_cast_panel(int64_t rows, int cols, const S* src, int64_t lds_, D* dst,
                       int64_t ldd, hipStream_t st);
template <class T>
void launch_copy_gated(int64_t rows, int cols, const T* src, int64_t lds_, T* dst,
                       int64_t ldd, const int* gate, hipStream_t st);

// out = 1 / S (0 where S <= 0); with `count`, also count_out[0] = *count.
// With `host` (pinned host memory), also host[0..k) = S and, with `count`,
// host[k] = *count: the values reach the host without a copy launch, and
// are there once the stream has passed this kernel.
void launch_recip(int k, const double* S, double* out, hipStream_t st,
                  const int* count = nullptr, double* count_out = nullptr,
                  double* host = nullptr);
// out[j] = ||R_j - S_j U_j|| / S_j  (Ritz residual ratios, k columns)
int ritz_blocks(int64_t m);
template <class T>
void launch_ritz(int64_t m, int k, const T* R, int64_t ldr, const T* U,
                 int64_t ldu, const double* S, double* partial, double* out,
                 hipStream_t st);

// Block-Jacobi symmetric eigensolver (FP64).
// one-workgroup tridiagonal top-k eigensolver (tridiag.hip)
bool tri_fits(int L, int k, size_t lds_bytes);
const void* tri_kernel_ptr();
void tri_set_lds_attributes(size_t lds_bytes);
// the multi-launch path for L up to tri_big_max() (tridiag.hip)
int tri_big_max();
int tri_big_kmax();
struct TriBigWork {
  static size_t doubles(int L, int k);   // workspace it needs
};
void launch_tri_big(int L, const double* G, int64_t ldg, int k, double* S, double* D,
                    double* W, int64_t ldw, double* ws, size_t ws_doubles,
                    size_t lds_bytes, hipStream_t st);
void launch_tri_topk(int L, const double* G, int64_t ldg, int k, double* S, double* D,
                     double* W, int64_t ldw, double* hh, size_t lds_bytes,
                     hipStream_t st);

struct EigSolver {
  static constexpr int kMaxSweeps = 30;
  DevBuf<double> A, V, J, Sd, scal, cslog, hh, big;
  DevBuf<int> rrlog;
  DevBuf<int> flags;
  int* hflags = nullptr;
  int L = 0, Lp = 0, sweeps = 0;
  ~EigSolver();
  void reserve(int L, hipStream_t st);
  // eigen-decompose the symmetric L x L matrix G (row-major, ldg)
  int solve(int L, const double* G, int64_t ldg, hipStream_t st);
  // largest L solved inside one workgroup by Jacobi (LDS-resident)
  static int single_max();
  // whether solve_topk(L, .., k, ..) runs without host round trips
  static bool device_only(int L, int k);
  // Jacobi sweeps of the last solve (synchronises for the one-workgroup path)
  int device_sweeps(hipStream_t st);
  // eigenpairs of the k largest eigenvalues (descending): S = sqrt(max(
  // lambda, 0)), Wk (L x k, ldw) vectors, D (optional, L) all eigenvalues
  // descending; one kernel without host round trips when L <= single_max()
  void solve_topk(int L, const double* G, int64_t ldg, int k, double* S,
                  double* D, double* Wk, int64_t ldw, hipStream_t st);
  // top-k of the last solve() (block path)
  void select_topk(int k, double* S, double* D, double* Wk, int64_t ldw,
                   hipStream_t st);
};

}  // namespace mcsvt
