// Sparse kernels of the SVT step.
//
// * Layout of Phi (Sec. II.C): the iterate Y lives on the sampled set, so
//   its CSR (row-major) and CSC (column-major) structures are built once on
//   the device, canonical (entries sorted by (row, col) / (col, row)).
// * SpMM  out = A X  for the Krylov products A Omega, A (A^T H) and
//   B^T = A^T Q of rSVD-BKI (Alg. 5), with A the CSR of Y or
//   the CSC of Y (= CSR of Y^T).  One wavefront per row segment; lanes span
//   the panel columns; long rows are split into segments whose partial rows
//   are summed in a fixed order by a second kernel, so results are
//   deterministic.
// * Fused SDDMM + residual + update (Eq. (6), Alg. 6): for every
//   (i, j) in Phi, x = sum_t U_it sig_t V_jt, e = M_ij - x, Y_ij += delta e,
//   and the squares e^2 are summed per block for the stop test.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "kernels.hpp"

namespace mcsvt {

namespace {

constexpr int kErrRange = 1;
constexpr int kErrNonFinite = 2;
constexpr int kErrDup = 4;

__global__ void coo_keys_kernel(int64_t nnz, int64_t m, int64_t n,
                                const int64_t* __restrict__ rows,
                                const int32_t* __restrict__ cols,
                                const double* __restrict__ vals,
                                uint64_t* __restrict__ keys,
                                int32_t* __restrict__ iota,
                                int* __restrict__ err) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = rows[e];
    const int64_t c = cols[e];
    int bad = 0;
    if (r < 0 || r >= m || c < 0 || c >= n) bad |= kErrRange;
    if (vals && !isfinite(vals[e])) bad |= kErrNonFinite;
    if (bad) atomicOr(err, bad);
    keys[e] = bad ? 0ull : (uint64_t)r * (uint64_t)n + (uint64_t)c;
    iota[e] = (int32_t)e;
  }
}

// sorted (row, col) keys -> row_of, col_idx, order; duplicate detection
__global__ void csr_split_kernel(int64_t nnz, int64_t n,
                                 const uint64_t* __restrict__ keys,
                                 const int32_t* __restrict__ src,
                                 int32_t* __restrict__ row_of,
                                 int32_t* __restrict__ col_idx,
                                 int32_t* __restrict__ order,
                                 int* __restrict__ err) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[e];
    row_of[e] = (int32_t)(k / (uint64_t)n);
    col_idx[e] = (int32_t)(k % (uint64_t)n);
    order[e] = src[e];
    if (e > 0 && keys[e - 1] == k) atomicOr(err, kErrDup);
  }
}

// ptr[i] = first position whose group id is >= i (lower bound), i in [0, g]
__global__ void group_ptr_kernel(int64_t nnz, int64_t groups,
                                 const int32_t* __restrict__ gid,
                                 int32_t* __restrict__ ptr) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= groups;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (gid[mid] < i) lo = mid + 1; else hi = mid;
    }
    ptr[i] = (int32_t)lo;
  }
}

__global__ void csc_keys_kernel(int64_t nnz, int64_t m,
                                const int32_t* __restrict__ row_of,
                                const int32_t* __restrict__ col_idx,
                                uint64_t* __restrict__ keys,
                                int32_t* __restrict__ iota) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    keys[e] = (uint64_t)col_idx[e] * (uint64_t)m + (uint64_t)row_of[e];
    iota[e] = (int32_t)e;
  }
}

__global__ void csc_split_kernel(int64_t nnz, int64_t m,
                                 const uint64_t* __restrict__ keys,
                                 const int32_t* __restrict__ src,
                                 int32_t* __restrict__ row_idx,
                                 int32_t* __restrict__ col_of,
                                 int32_t* __restrict__ perm,
                                 int32_t* __restrict__ invperm) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[e];
    row_idx[e] = (int32_t)(k % (uint64_t)m);
    col_of[e] = (int32_t)(k / (uint64_t)m);
    const int32_t s = src[e];
    perm[e] = s;
    invperm[s] = (int32_t)e;
  }
}

template <class T>
__global__ void gather_kernel(int64_t nnz, const int32_t* __restrict__ idx,
                              const T* __restrict__ src, T* __restrict__ dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[idx[e]];
}

template <class T>
__global__ void scatter_kernel(int64_t nnz, const int32_t* __restrict__ idx,
                               const T* __restrict__ src, T* __restrict__ dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[idx[e]] = src[e];
}

// row i's entries [ptr[i], ptr[i+1]) get row id i; a pointer that does not
// start at 0, end at nnz or never decrease sets err and writes nothing out of
// [0, nnz)
__global__ void csr_rows_kernel(int64_t m, int64_t nnz, const int64_t* __restrict__ ptr,
                                int64_t* __restrict__ rows, int* __restrict__ err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = ptr[i], e = ptr[i + 1];
    if ((i == 0 && b != 0) || (i == m - 1 && e != nnz) || e < b || b < 0 || e > nnz) {
      atomicOr(err, 1);
      continue;
    }
    for (int64_t q = b; q < e; ++q) rows[q] = i;
  }
}

inline unsigned grid_for(int64_t n, int threads) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, threads),
                                                          kMaxGrid));
}

int bits_for(uint64_t maxval) {
  int b = 1;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

}  // namespace

int csr_rows_device(int64_t m, int64_t nnz, const int64_t* d_ptr, int64_t* d_rows,
                    hipStream_t st) {
  DevBuf<int> err;
  err.reserve(1, st);
  MC_HIP(hipMemsetAsync(err.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(csr_rows_kernel, dim3(grid_for(m, 256)), dim3(256), 0, st, m, nnz,
                     d_ptr, d_rows, err.p);
  MC_CHECK_LAUNCH();
  int herr = 0;
  MC_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  MC_HIP(hipStreamSynchronize(st));
  return herr ? kEINVAL : kOK;
}

// ---------------------------------------------------------------------------
// Canonical CSR / CSC build of Phi.
// ---------------------------------------------------------------------------
int build_layout(int64_t m, int64_t n, int64_t nnz, const int64_t* d_rows,
                 const int32_t* d_cols, const double* d_vals, Layout& L,
                 hipStream_t st) {
  L.m = m;
  L.n = n;
  L.nnz = nnz;
  DevBuf<uint64_t> keys_a, keys_b;
  DevBuf<int32_t> idx_a, idx_b, col_of;
  DevBuf<int> err;
  keys_a.reserve(nnz, st);
  keys_b.reserve(nnz, st);
  idx_a.reserve(nnz, st);
  idx_b.reserve(nnz, st);
  err.reserve(1, st);
  MC_HIP(hipMemsetAsync(err.p, 0, sizeof(int), st));
  const int T = 256;
  hipLaunchKernelGGL(coo_keys_kernel, dim3(grid_for(nnz, T)), dim3(T), 0, st,
                     nnz, m, n, d_rows, d_cols, d_vals, keys_a.p, idx_a.p,
                     err.p);
  MC_CHECK_LAUNCH();
  int herr = 0;
  MC_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  MC_HIP(hipStreamSynchronize(st));
  if (herr & kErrRange) return kERANGE;
  if (herr & kErrNonFinite) return kEINVAL;

  const int end_bit = bits_for((uint64_t)m * (uint64_t)n - 1);
  size_t tmp_bytes = 0;
  MC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys_a.p,
                                            keys_b.p, idx_a.p, idx_b.p,
                                            (int)nnz, 0, end_bit, st));
  DevBuf<char> tmp;
  tmp.reserve(tmp_bytes, st);
  MC_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, keys_a.p,
                                            keys_b.p, idx_a.p, idx_b.p,
                                            (int)nnz, 0, end_bit, st));
  L.row_of.reserve(nnz, st);
  L.col_idx.reserve(nnz, st);
  L.order.reserve(nnz, st);
  hipLaunchKernelGGL(csr_split_kernel, dim3(grid_for(nnz, T)), dim3(T), 0, st,
                     nnz, n, keys_b.p, idx_b.p, L.row_of.p, L.col_idx.p,
                     L.order.p, err.p);
  MC_CHECK_LAUNCH();
  MC_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  MC_HIP(hipStreamSynchronize(st));
  if (herr & kErrDup) return kEDUP;
  L.row_ptr.reserve(m + 1, st);
  hipLaunchKernelGGL(group_ptr_kernel, dim3(grid_for(m + 1, T)), dim3(T), 0, st,
                     nnz, m, L.row_of.p, L.row_ptr.p);
  MC_CHECK_LAUNCH();

  // CSC: sort the CSR positions by (col, row)
  hipLaunchKernelGGL(csc_keys_kernel, dim3(grid_for(nnz, T)), dim3(T), 0, st,
                     nnz, m, L.row_of.p, L.col_idx.p, keys_a.p, idx_a.p);
  MC_CHECK_LAUNCH();
  const int end_bit2 = bits_for((uint64_t)n * (uint64_t)m - 1);
  size_t tmp2 = 0;
  MC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp2, keys_a.p, keys_b.p,
                                            idx_a.p, idx_b.p, (int)nnz, 0,
                                            end_bit2, st));
  tmp.reserve(tmp2, st);
  MC_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp2, keys_a.p, keys_b.p,
                                            idx_a.p, idx_b.p, (int)nnz, 0,
                                            end_bit2, st));
  L.row_idx.reserve(nnz, st);
  L.perm.reserve(nnz, st);
  L.invperm.reserve(nnz, st);
  col_of.reserve(nnz, st);
  hipLaunchKernelGGL(csc_split_kernel, dim3(grid_for(nnz, T)), dim3(T), 0, st,
                     nnz, m, keys_b.p, idx_b.p, L.row_idx.p, col_of.p, L.perm.p,
                     L.invperm.p);
  MC_CHECK_LAUNCH();
  L.col_ptr.reserve(n + 1, st);
  hipLaunchKernelGGL(group_ptr_kernel, dim3(grid_for(n + 1, T)), dim3(T), 0, st,
                     nnz, n, col_of.p, L.col_ptr.p);
  MC_CHECK_LAUNCH();

  // host copies of the pointers (and, for a large gathered dimension, of
  // the indices) -> SpMM segment schedules
  std::vector<int32_t> hptr(std::max(m, n) + 1);
  std::vector<int32_t> hidx;
  auto schedule = [&](const int32_t* d_ptr, int64_t rows, const int32_t* d_idx,
                      int64_t gathered, Schedule& S) {
    MC_HIP(hipMemcpyAsync(hptr.data(), d_ptr, (rows + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, st));
    const bool band = gathered >= kBandMinRows;
    if (band) {
      hidx.resize(nnz);
      MC_HIP(hipMemcpyAsync(hidx.data(), d_idx, nnz * sizeof(int32_t),
                            hipMemcpyDeviceToHost, st));
    }
    MC_HIP(hipStreamSynchronize(st));
    build_schedule(hptr.data(), rows, S, st, band ? hidx.data() : nullptr, gathered);
  };
  schedule(L.row_ptr.p, m, L.col_idx.p, n, L.sched_csr);
  schedule(L.col_ptr.p, n, L.row_idx.p, m, L.sched_csc);
  MC_HIP(hipStreamSynchronize(st));
  return kOK;
}

namespace {

// pieces of [b, e) of at most `cap` entries each
int64_t cap_pieces(int64_t len, int64_t cap) { return len <= cap ? 1 : ceil_div(len, cap); }

// Appends the segments of row i's range [b, e) cut into `pieces` near-equal
// parts, with slots from `slot` on when the row has partial rows.
template <class Push>
void push_pieces(int64_t i, int32_t b, int32_t e, int64_t pieces, bool partial,
                 int32_t& slot, Push&& push) {
  const int64_t len = e - b;
  for (int64_t q = 0; q < pieces; ++q) {
    const int32_t sb = b + (int32_t)(q * len / pieces);
    const int32_t se = b + (int32_t)((q + 1) * len / pieces);
    push(make_int4((int)i, sb, se, partial ? slot++ : -1));
  }
}

void upload_segs(const std::vector<int4>& v, DevBuf<int4>& d, hipStream_t st) {
  d.reserve(std::max<int64_t>((int64_t)v.size(), 1), st);
  if (!v.empty())
    MC_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(int4),
                          hipMemcpyHostToDevice, st));
}

}  // namespace

// Banded form (see Schedule) with nb = kBands * t bands: rows of at least
// band_split_len(cap) entries are cut at the band boundaries of their (sorted)
// gathered indices, then by `cap`; band r belongs to XCD r % kBands, which
// takes its bands in the order r % kBands, r % kBands + kBands, ... so that
// its L2 holds one band at a time.  Shorter rows stay whole (or cut by `cap`)
// and go to the XCDs with the fewest segments.  XCD x's segments take
// workgroup slots x, x + kBands, ...; the slots left over hold padding.
void band_schedule(const int32_t* ptr, const int32_t* idx, int64_t rows,
                   int64_t gathered, int64_t cap, int nb, std::vector<int4>& segs,
                   std::vector<int4>& fix, int32_t& slot) {
  std::vector<std::vector<int4>> band(nb);
  std::vector<int4> loose;
  std::vector<int32_t> bound(nb + 1), cut(nb + 1);
  for (int r = 0; r <= nb; ++r) bound[r] = (int32_t)(r * gathered / nb);
  const int64_t split = band_split_len(cap);
  for (int64_t i = 0; i < rows; ++i) {
    const int32_t b = ptr[i], e = ptr[i + 1];
    const int64_t len = e - b;
    if (len < split) {
      const int64_t pieces = cap_pieces(len, cap);
      if (pieces > 1) fix.push_back(make_int4((int)i, slot, (int)pieces, 0));
      push_pieces(i, b, e, pieces, pieces > 1, slot,
                  [&](int4 sg) { loose.push_back(sg); });
      continue;
    }
    cut[0] = b;
    cut[nb] = e;
    for (int r = 1; r < nb; ++r)
      cut[r] = (int32_t)(std::lower_bound(idx + cut[r - 1], idx + e, bound[r]) - idx);
    int64_t pieces = 0;
    for (int r = 0; r < nb; ++r)
      if (cut[r + 1] > cut[r]) pieces += cap_pieces(cut[r + 1] - cut[r], cap);
    if (pieces > 1) fix.push_back(make_int4((int)i, slot, (int)pieces, 0));
    for (int r = 0; r < nb; ++r)
      if (cut[r + 1] > cut[r])
        push_pieces(i, cut[r], cut[r + 1], cap_pieces(cut[r + 1] - cut[r], cap),
                    pieces > 1, slot, [&](int4 sg) { band[r].push_back(sg); });
  }
  std::vector<std::vector<int4>> xcd(kBands);
  for (int r = 0; r < nb; ++r)
    xcd[r % kBands].insert(xcd[r % kBands].end(), band[r].begin(), band[r].end());
  for (const int4& sg : loose) {
    int x = 0;
    for (int t = 1; t < kBands; ++t)
      if (xcd[t].size() < xcd[x].size()) x = t;
    xcd[x].push_back(sg);
  }
  size_t nwg = 0;
  for (int x = 0; x < kBands; ++x)
    nwg = std::max(nwg, (size_t)ceil_div((int64_t)xcd[x].size(), kSpmmWaves));
  segs.assign(nwg * kBands * kSpmmWaves, make_int4(-1, 0, 0, -1));
  for (int x = 0; x < kBands; ++x)
    for (size_t q = 0; q < xcd[x].size(); ++q)
      segs[((q / kSpmmWaves) * kBands + x) * kSpmmWaves + q % kSpmmWaves] = xcd[x][q];
}

// Split rows into work segments of at most `cap` entries.  Rows that need
// several segments get partial slots and a fix-up record.  With the gathered
// indices given and a large gathered dimension, the banded form as well.
void build_schedule(const int32_t* ptr, int64_t rows, Schedule& S,
                    hipStream_t st, const int32_t* idx, int64_t gathered) {
  const int64_t nnz = ptr[rows];
  const int64_t cap = spmm_segment_cap(nnz);
  std::vector<int4> segs;
  std::vector<int4> fix;
  segs.reserve(rows + 16);
  int32_t slot = 0;
  for (int64_t i = 0; i < rows; ++i) {
    const int32_t b = ptr[i], e = ptr[i + 1];
    const int64_t pieces = cap_pieces(e - b, cap);
    if (pieces > 1) fix.push_back(make_int4((int)i, slot, (int)pieces, 0));
    push_pieces(i, b, e, pieces, pieces > 1, slot, [&](int4 sg) { segs.push_back(sg); });
  }
  S.nseg = (int64_t)segs.size();
  S.nfix = (int64_t)fix.size();
  S.nslot = slot;
  upload_segs(segs, S.segs, st);
  upload_segs(fix, S.fix, st);
  MC_HIP(hipStreamSynchronize(st));
  S.gathered = gathered;
  int64_t in_long = 0;
  for (int64_t i = 0; i < rows; ++i)
    if (ptr[i + 1] - ptr[i] >= band_split_len(cap)) in_long += ptr[i + 1] - ptr[i];
  S.long_share = 4 * in_long >= nnz;
  S.band_nseg = S.band_nfix = 0;
  if (idx && gathered >= kBandMinRows && nnz > 0) {
    std::vector<int4> bsegs, bfix;
    int32_t bslot = 0;
    band_schedule(ptr, idx, rows, gathered, cap, kBands, bsegs, bfix, bslot);
    S.band_nseg = (int64_t)bsegs.size();
    S.band_nfix = (int64_t)bfix.size();
    S.nslot = std::max<int64_t>(S.nslot, bslot);
    upload_segs(bsegs, S.band_segs, st);
    upload_segs(bfix, S.band_fix, st);
    MC_HIP(hipStreamSynchronize(st));
  }
}

namespace {
template <class S, class D>
__global__ void cast_kernel(int64_t n, const S* __restrict__ src, D* __restrict__ dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (D)src[e];
}
}  // namespace

template <class S, class D>
void launch_cast(int64_t n, const S* src, D* dst, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((cast_kernel<S, D>), dim3(grid_for(n, 256)), dim3(256), 0, st,
                     n, src, dst);
  MC_CHECK_LAUNCH();
}
template void launch_cast<double, float>(int64_t, const double*, float*, hipStream_t);
template void launch_cast<float, double>(int64_t, const float*, double*, hipStream_t);
template void launch_cast<double, bf16_t>(int64_t, const double*, bf16_t*, hipStream_t);
template void launch_cast<double, double>(int64_t, const double*, double*, hipStream_t);

template <class T>
void launch_gather(int64_t nnz, const int32_t* idx, const T* src, T* dst,
                   hipStream_t st) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(gather_kernel<T>, dim3(grid_for(nnz, 256)), dim3(256), 0,
                     st, nnz, idx, src, dst);
  MC_CHECK_LAUNCH();
}
template <class T>
void launch_scatter(int64_t nnz, const int32_t* idx, const T* src, T* dst,
                    hipStream_t st) {
  if (nnz <= 0) return;
  hipLaunchKernelGGL(scatter_kernel<T>, dim3(grid_for(nnz, 256)), dim3(256), 0,
                     st, nnz, idx, src, dst);
  MC_CHECK_LAUNCH();
}
template void launch_gather<double>(int64_t, const int32_t*, const double*,
                                    double*, hipStream_t);
template void launch_gather<float>(int64_t, const int32_t*, const float*,
                                   float*, hipStream_t);
template void launch_gather<int32_t>(int64_t, const int32_t*, const int32_t*,
                                     int32_t*, hipStream_t);
template void launch_scatter<double>(int64_t, const int32_t*, const double*,
                                     double*, hipStream_t);

// ---------------------------------------------------------------------------
// SpMM  out (rows x b) = A (rows x cols, segments) . X (cols x b)
// ---------------------------------------------------------------------------
namespace {

// loads of data read once (non-temporal)
template <class T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <>
__device__ __forceinline__ bf16_t ld_stream<bf16_t>(const bf16_t* p) {
  bf16_t v;
  v.bits = __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
  return v;
}

// One wavefront per segment.  BW lanes share one nonzero and cover BW
// columns per load, each lane accumulating CPL columns (c, c + BW, ...), so a
// nonzero's index and value are broadcast once for up to BW * CPL columns;
// 64 / BW nonzeros are in flight side by side.  Columns beyond b read an
// in-bounds address with weight zero.  The same device function serves the
// single-product kernel and the grouped one (products of several solves in
// one launch), so a product's arithmetic does not depend on how it was
// launched.
template <class VT, class XT, class AT, class OT, int BW, int CPL>
__device__ __forceinline__ void spmm_segment(
    const int4 sg, const int32_t* __restrict__ idx, const VT* __restrict__ val,
    const XT* __restrict__ X, int64_t ldx, OT* __restrict__ out, int64_t ldo,
    AT* __restrict__ part, int b) {
  constexpr int G = 64 / BW;       // nonzeros processed side by side
  constexpr int CB = BW * CPL;     // columns per pass
  const int lane = threadIdx.x & 63;
  if (sg.x < 0) return;                        // padding of a banded schedule
  const int g = lane / BW;
  const int c = lane % BW;
  for (int c0 = 0; c0 < b; c0 += CB) {
    int colc[CPL];
    AT acc[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const int col = c0 + c + t * BW;
      colc[t] = col < b ? col : b - 1;
      acc[t] = 0;
    }
    for (int base = sg.y; base < sg.z; base += 64) {
      const int e = base + lane;
      const bool ok = e < sg.z;
      // lanes past the segment carry index 0 and value 0; the index and
      // value streams are read once, so they bypass the caches that hold X
      const int my_idx = ok ? ld_stream(idx + e) : 0;
      const AT my_val = ok ? (AT)ld_stream(val + e) : (AT)0;
      const int left = sg.z - base;            // nonzeros left in the segment
      // two halves of 32 nonzeros: the gathers of a half are independent and
      // issued back to back; a short tail skips the second half
#pragma unroll
      for (int h = 0; h < 64; h += 32) {
        if (h >= left) break;                  // uniform: the wave's segment
#pragma unroll
        for (int jj = h; jj < h + 32; jj += G) {
          const int jc = __shfl(my_idx, jj + g);
          const AT jv = __shfl(my_val, jj + g);
          const XT* xr = X + (int64_t)jc * ldx;
#pragma unroll
          for (int t = 0; t < CPL; ++t) acc[t] += jv * (AT)xr[colc[t]];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
#pragma unroll
      for (int off = BW; off < 64; off <<= 1) acc[t] += __shfl_xor(acc[t], off);
    }
    if (g == 0) {
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int col = c0 + c + t * BW;
        if (col >= b) continue;
        if (sg.w < 0)
          out[(int64_t)sg.x * ldo + col] = (OT)acc[t];
        else
          part[(int64_t)sg.w * b + col] = acc[t];
      }
    }
  }
}

template <class VT, class XT, class AT, class OT, int BW, int CPL>
__global__ __launch_bounds__(256) void spmm_kernel(
    int64_t nseg, const int4* __restrict__ segs,
    const int32_t* __restrict__ idx, const VT* __restrict__ val,
    const XT* __restrict__ X, int64_t ldx, OT* __restrict__ out, int64_t ldo,
    AT* __restrict__ part, int b) {
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (wave >= nseg) return;
  spmm_segment<VT, XT, AT, OT, BW, CPL>(segs[wave], idx, val, X, ldx, out, ldo, part, b);
}

// Products of several solves in one launch: task t owns workgroups
// [wg0_t, wg0_t + ceil(nseg_t / waves)), its first workgroup a multiple of
// kBands so that a banded schedule keeps its workgroup-to-XCD placement.
template <class VT, class XT, class AT, class OT, int BW, int CPL>
__global__ __launch_bounds__(256) void spmm_group_kernel(const SpmmTask* __restrict__ tasks,
                                                         int ntask) {
  const int64_t wg = blockIdx.x;
  int t = 0;
  while (t + 1 < ntask && tasks[t + 1].wg0 <= wg) ++t;   // few tasks: a scan
  const SpmmTask& k = tasks[t];
  const int64_t wave = (wg - k.wg0) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (wave < 0 || wave >= k.nseg) return;
  spmm_segment<VT, XT, AT, OT, BW, CPL>(k.segs[wave], k.idx, (const VT*)k.val,
                                        (const XT*)k.X, k.ldx, (OT*)k.out, k.ldo,
                                        (AT*)k.part, k.b);
}

template <class AT, class OT>
__device__ __forceinline__ void spmm_fixup_one(const int4 fx, int col,
                                               const AT* __restrict__ part,
                                               OT* __restrict__ out, int64_t ldo, int b) {
  // the partial rows come from other workgroups (other XCDs): their loads go
  // out eight at a time and are added in slot order
  const AT* __restrict__ pp = part + (int64_t)fx.y * b + col;
  AT acc = 0;
  int q = 0;
  for (; q + 8 <= fx.z; q += 8) {
    AT v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = pp[(int64_t)(q + u) * b];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; q < fx.z; ++q) acc += pp[(int64_t)q * b];
  out[(int64_t)fx.x * ldo + col] = (OT)acc;
}

template <class AT, class OT>
__global__ void spmm_fixup_kernel(int64_t nfix, const int4* __restrict__ fix,
                                  const AT* __restrict__ part, OT* __restrict__ out,
                                  int64_t ldo, int b) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nfix * b) return;
  spmm_fixup_one<AT, OT>(fix[t / b], (int)(t % b), part, out, ldo, b);
}

// the fix-ups of a grouped launch: task t owns items [fx0_t, fx0_t + nfix_t b)
template <class AT, class OT>
__global__ void spmm_group_fixup_kernel(const SpmmTask* __restrict__ tasks, int ntask) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int t = 0;
  while (t + 1 < ntask && tasks[t + 1].fx0 <= i) ++t;
  const SpmmTask& k = tasks[t];
  const int64_t r = i - k.fx0;
  if (r < 0 || r >= k.nfix * k.b) return;
  spmm_fixup_one<AT, OT>(k.fix[r / k.b], (int)(r % k.b), (const AT*)k.part, (OT*)k.out,
                         k.ldo, k.b);
}

}  // namespace

namespace {
// The lane split of a product of width b: BW lanes per nonzero, CPL columns
// per lane (see spmm_segment), as a form number 0..18.
constexpr int kForms = 19;
constexpr int kFormBW[kForms] = {8, 16, 8, 16, 8, 16, 8, 16, 8, 16, 16, 16, 32,
                                 64, 64, 64, 64, 64, 64};
constexpr int kFormCPL[kForms] = {1, 1, 3, 2, 5, 3, 7, 4, 9, 5, 6, 7, 4,
                                  3, 4, 5, 6, 7, 8};
int spmm_form(int b) {
  if (b <= 8) return 0;
  if (b <= 16) return 1;
  if (b <= 24) return 2;
  if (b <= 32) return 3;
  if (b <= 40) return 4;
  if (b <= 48) return 5;
  if (b <= 56) return 6;
  if (b <= 64) return 7;
  if (b <= 72) return 8;
  if (b <= 80) return 9;
  if (b <= 96) return 10;
  if (b <= 112) return 11;
  if (b <= 128) return 12;
  // wide panels: 64 lanes per nonzero and the fewest passes of at most 512
  // columns, each as narrow as covers b
  const int passes = (int)ceil_div(b, 512);
  const int cpl = (int)ceil_div(ceil_div(b, passes), 64);   // 3..8
  return 13 + std::min(std::max(cpl, 3), 8) - 3;
}

// launch `K<..., BW, CPL>` for form f (a switch over the table above)
#define MC_FORM_SWITCH(f, LAUNCH) \
  switch (f) {                    \
    case 0: LAUNCH(8, 1); break;  \
    case 1: LAUNCH(16, 1); break; \
    case 2: LAUNCH(8, 3); break;  \
    case 3: LAUNCH(16, 2); break; \
    case 4: LAUNCH(8, 5); break;  \
    case 5: LAUNCH(16, 3); break; \
    case 6: LAUNCH(8, 7); break;  \
    case 7: LAUNCH(16, 4); break; \
    case 8: LAUNCH(8, 9); break;  \
    case 9: LAUNCH(16, 5); break; \
    case 10: LAUNCH(16, 6); break; \
    case 11: LAUNCH(16, 7); break; \
    case 12: LAUNCH(32, 4); break; \
    case 13: LAUNCH(64, 3); break; \
    case 14: LAUNCH(64, 4); break; \
    case 15: LAUNCH(64, 5); break; \
    case 16: LAUNCH(64, 6); break; \
    case 17: LAUNCH(64, 7); break; \
    default: LAUNCH(64, 8); break; \
  }
}  // namespace

SpmmTask make_spmm_task(const Schedule& S, const int32_t* idx, const void* val,
                        const void* X, int64_t ldx, void* out, int64_t ldo, int b,
                        void* part, size_t x_bytes) {
  SpmmTask t{};
  // the banded form for large panels (see Schedule)
  const bool band = S.band_nseg > 0 &&
                    S.gathered * (int64_t)b * (int64_t)x_bytes >= kBandPanelBytes &&
                    (b <= kBandWide || S.long_share);
  t.nseg = band ? S.band_nseg : S.nseg;
  t.segs = band ? S.band_segs.p : S.segs.p;
  t.nfix = band ? S.band_nfix : S.nfix;
  t.fix = band ? S.band_fix.p : S.fix.p;
  t.idx = idx;
  t.val = val;
  t.X = X;
  t.ldx = ldx;
  t.out = out;
  t.ldo = ldo;
  t.part = part;
  t.b = b;
  return t;
}

template <class VT, class XT, class AT, class OT>
void launch_spmm(const Schedule& S, const int32_t* idx, const VT* val,
                 const XT* X, int64_t ldx, OT* out, int64_t ldo, int b,
                 AT* part, hipStream_t st) {
  if (S.nseg == 0 || b <= 0) return;
  const int T = 64 * kSpmmWaves;
  const SpmmTask k = make_spmm_task(S, idx, val, X, ldx, out, ldo, b, part, sizeof(XT));
  const unsigned grid = (unsigned)ceil_div(k.nseg, kSpmmWaves);
#define MC_SPMM(BW, CPL)                                                          \
  hipLaunchKernelGGL((spmm_kernel<VT, XT, AT, OT, BW, CPL>), dim3(grid), dim3(T), 0, \
                     st, k.nseg, k.segs, idx, val, X, ldx, out, ldo, part, b)
  MC_FORM_SWITCH(spmm_form(b), MC_SPMM)
#undef MC_SPMM
  MC_CHECK_LAUNCH();
  if (k.nfix) {
    const int64_t work = k.nfix * b;
    hipLaunchKernelGGL((spmm_fixup_kernel<AT, OT>), dim3((unsigned)ceil_div(work, T)),
                       dim3(T), 0, st, k.nfix, k.fix, part, out, ldo, b);
    MC_CHECK_LAUNCH();
  }
}

// Grouped launches: the tasks are split by lane form; each form's tasks go
// out in one product launch (and one fix-up launch) whose task table is
// copied from `staging` (pinned host memory, `cap` entries, left untouched
// until the stream has passed the copies) to `table` (device).
template <class VT, class XT, class AT, class OT>
void launch_spmm_group(const std::vector<SpmmTask>& tasks, SpmmTask* staging,
                       SpmmTask* table, int64_t cap, hipStream_t st) {
  const int T = 64 * kSpmmWaves;
  int64_t used = 0;
  for (int f = 0; f < kForms; ++f) {
    int64_t first = used, wg = 0, fx = 0;
    for (const SpmmTask& k : tasks) {
      if (k.nseg == 0 || k.b <= 0 || spmm_form((int)k.b) != f) continue;
      MC_REQUIRE(used < cap, kEINVAL, "grouped SpMM: task table full");
      SpmmTask e = k;
      e.wg0 = wg;
      e.fx0 = fx;
      wg += round_up(ceil_div(k.nseg, kSpmmWaves), kBands);
      fx += k.nfix * k.b;
      staging[used++] = e;
    }
    const int n = (int)(used - first);
    if (n == 0) continue;
    MC_HIP(hipMemcpyAsync(table + first, staging + first, n * sizeof(SpmmTask),
                          hipMemcpyHostToDevice, st));
#define MC_SPMM_G(BW, CPL)                                                           \
  hipLaunchKernelGGL((spmm_group_kernel<VT, XT, AT, OT, BW, CPL>), dim3((unsigned)wg), \
                     dim3(T), 0, st, table + first, n)
    MC_FORM_SWITCH(f, MC_SPMM_G)
#undef MC_SPMM_G
    MC_CHECK_LAUNCH();
    if (fx) {
      hipLaunchKernelGGL((spmm_group_fixup_kernel<AT, OT>), dim3((unsigned)ceil_div(fx, T)),
                         dim3(T), 0, st, table + first, n);
      MC_CHECK_LAUNCH();
    }
  }
}
template void launch_spmm_group<float, float, float, float>(
    const std::vector<SpmmTask>&, SpmmTask*, SpmmTask*, int64_t, hipStream_t);
template void launch_spmm_group<double, double, double, double>(
    const std::vector<SpmmTask>&, SpmmTask*, SpmmTask*, int64_t, hipStream_t);

template void launch_spmm<double, double, double, double>(
    const Schedule&, const int32_t*, const double*, const double*, int64_t,
    double*, int64_t, int, double*, hipStream_t);
template void launch_spmm<float, float, float, float>(
    const Schedule&, const int32_t*, const float*, const float*, int64_t,
    float*, int64_t, int, float*, hipStream_t);
template void launch_spmm<bf16_t, float, float, float>(
    const Schedule&, const int32_t*, const bf16_t*, const float*, int64_t,
    float*, int64_t, int, float*, hipStream_t);
template void launch_spmm<bf16_t, bf16_t, float, float>(
    const Schedule&, const int32_t*, const bf16_t*, const bf16_t*, int64_t,
    float*, int64_t, int, float*, hipStream_t);

// ---------------------------------------------------------------------------
// Fused SDDMM + residual + update.
// ---------------------------------------------------------------------------
namespace {


template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// x = sum_t (u_t sig_t) v_t accumulated in AT; e = M - x and the update of the
// FP64 master Y in double; the operator copies of Y are refreshed from the
// master: CSR / CSC copies of type VT (Krylov products) and WT (Rayleigh-Ritz
// products); a null pointer skips a copy (e.g. when the master serves).
//
// One wavefront per CSR segment (a row, or a piece of a long row).  The
// row's u_i diag(sig) stays in registers (CPL columns per lane); BW lanes
// share one nonzero and gather its row of V, a butterfly over those BW lanes
// completes the dot product, and a shuffle hands the sum to the lane that
// holds the nonzero's M, Y and index, which forms the residual and the
// update.  Columns beyond r carry weight zero; ranks above BW * CPL take
// several passes.  Partial residual sums: one per workgroup, in a fixed
// order.
template <class FT, class AT, class VT, class WT, int BW, int CPL>
__global__ __launch_bounds__(64 * kSpmmWaves) void sddmm_update_kernel(
    int64_t nseg, const int4* __restrict__ segs, const int32_t* __restrict__ col_idx,
    const double* __restrict__ mvals, double* __restrict__ y, VT* __restrict__ yv,
    VT* __restrict__ ycv, WT* __restrict__ yw, WT* __restrict__ ycw,
    const int32_t* __restrict__ invperm, const FT* __restrict__ U, int64_t ldu,
    const FT* __restrict__ V, int64_t ldv, const double* __restrict__ sig, int r,
    double delta, int apply, double* __restrict__ partial) {
  constexpr int G = 64 / BW;       // nonzeros side by side
  constexpr int CB = BW * CPL;     // columns per pass
  __shared__ double red[kSpmmWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t wave = (int64_t)blockIdx.x * kSpmmWaves + wv;
  double d2 = 0.0;
  const int4 sg = wave < nseg ? segs[wave] : make_int4(-1, 0, 0, -1);
  if (sg.x >= 0) {
    const int g = lane / BW, c = lane % BW;
    const FT* urow = U + (int64_t)sg.x * ldu;
    // this lane's u_i sig entries of the row for pass c0: loads from clamped
    // columns (issued together), zeroed past r by a select
    auto row_weights = [&](int c0, AT* uu, int* colc) {
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int col = c0 + c + t * BW;
        colc[t] = col < r ? col : r - 1;
        const AT w = (AT)urow[colc[t]] * (AT)sig[colc[t]];
        uu[t] = col < r ? w : (AT)0;
      }
    };
    // the first pass's weights serve every 64-entry chunk of the segment when
    // registers allow (measured: held across the segment they slow the forms
    // with more than 32 gathers per half-chunk or more than 5 columns per lane)
    constexpr bool kHold = CPL <= 5 && (32 / G) * CPL <= 32;
    AT uu0[CPL];
    int colc0[CPL];
    if (kHold && r > 0) row_weights(0, uu0, colc0);
    for (int base = sg.y; base < sg.z; base += 64) {
      const int e = base + lane;
      const bool ok = e < sg.z;
      const int my_col = ok ? ld_stream(col_idx + e) : 0;
      const int left = sg.z - base;
      AT xl = 0;                               // x of nonzero `e` (this lane)
      // this lane's M, Y and CSC position, requested once the first half's
      // gathers are out (loads complete in issue order: requested before
      // them, these streaming loads would hold up the gathers' use).  The
      // master Y is read and written non-temporally, so that it does not
      // evict V's rows or the lines the CSC copy is being scattered into.
      double mv = 0.0, yo = 0.0;
      int ecp = 0;
      bool req = false;
      auto request = [&]() {
        if (ok) {
          mv = ld_stream(mvals + e);
          if (apply) {
            yo = ld_stream(y + e);
            ecp = ld_stream(invperm + e);
          }
        }
        req = true;
      };
      for (int c0 = 0; c0 < r; c0 += CB) {
        AT uu[CPL];
        int colc[CPL];
        if (kHold && c0 == 0) {
#pragma unroll
          for (int t = 0; t < CPL; ++t) {
            uu[t] = uu0[t];
            colc[t] = colc0[t];
          }
        } else {
          row_weights(c0, uu, colc);
        }
        // two halves of 32 nonzeros: the gathers of a half are issued back to
        // back into registers, then their dot products formed; a short tail
        // skips the second half
#pragma unroll
        for (int h = 0; h < 64; h += 32) {
          if (h >= left) break;                // uniform: the wave's segment
          AT gv[32 / G][CPL];
#pragma unroll
          for (int u = 0; u < 32 / G; ++u) {
            const int jc = __shfl(my_col, h + u * G + g);
            const FT* vr = V + (int64_t)jc * ldv;
#pragma unroll
            for (int t = 0; t < CPL; ++t) gv[u][t] = (AT)vr[colc[t]];
          }
          if (!req) request();
#pragma unroll
          for (int u = 0; u < 32 / G; ++u) {
            const int jj = h + u * G;
            AT pdot = 0;
#pragma unroll
            for (int t = 0; t < CPL; ++t) pdot += uu[t] * gv[u][t];
#pragma unroll
            for (int off = 1; off < BW; off <<= 1) pdot += __shfl_xor(pdot, off);
            // nonzero jj + g's sum sits in every lane of group g; lane
            // jj + g' takes group g''s
            const bool mine = lane >= jj && lane < jj + G;
            const AT got = __shfl(pdot, mine ? (lane - jj) * BW : 0);
            if (mine) xl += got;
          }
        }
      }
      if (!req) request();
      if (ok) {
        const double d = mv - (double)xl;
        d2 += d * d;
        if (apply) {
          const double yn = yo + delta * d;
          __builtin_nontemporal_store(yn, y + e);
          const int32_t ec = ecp;
          if (yv) yv[e] = (VT)yn;
          if (ycv) ycv[ec] = (VT)yn;
          if (yw) yw[e] = (WT)yn;
          if (ycw) ycw[ec] = (WT)yn;
        }
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d2 += __shfl_xor(d2, off);
  if (lane == 0) red[wv] = d2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kSpmmWaves; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

template <class FT>
__global__ void eval_observed_kernel(int64_t nnz, const int32_t* __restrict__ row_of,
                                     const int32_t* __restrict__ col_idx,
                                     const FT* __restrict__ U, int64_t ldu,
                                     const FT* __restrict__ V, int64_t ldv,
                                     const double* __restrict__ sig, int r,
                                     const int32_t* __restrict__ order,
                                     double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const FT* u = U + (int64_t)row_of[e] * ldu;
    const FT* v = V + (int64_t)col_idx[e] * ldv;
    double x = 0.0;
    for (int t = 0; t < r; ++t) x += ((double)u[t] * sig[t]) * (double)v[t];
    out[order[e]] = x;
  }
}

__global__ void sumsq_kernel(int64_t n, const double* __restrict__ a,
                             double* __restrict__ partial) {
  __shared__ double sh[256];
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  const double v = e < n ? a[e] : 0.0;
  const double s = block_sum<256>(v * v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// single block: out[0] = sum of partial[0..n) in a fixed order
__global__ void reduce_kernel(int64_t n, const double* __restrict__ partial,
                              double* __restrict__ out) {
  __shared__ double sh[1024];
  double acc = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 7 * 1024 < n; i += 8 * 1024) {      // loads eight at a time, added in order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partial[i + u * 1024];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; i < n; i += 1024) acc += partial[i];
  const double s = block_sum<1024>(acc, sh);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void scale_kernel(int64_t n, const double* __restrict__ a,
                             double alpha, double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = alpha * a[e];
}

}  // namespace

int64_t sddmm_partials(const Layout& L) {
  return std::max({ceil_div(L.nnz, 256), ceil_div(L.sched_csr.nseg, kSpmmWaves),
                   ceil_div(L.sched_csr.band_nseg, kSpmmWaves)});
}

template <class FT, class AT, class VT, class WT>
void launch_sddmm_update(const Layout& L, const double* mvals, double* y, VT* yv,
                         VT* ycv, WT* yw, WT* ycw, const FT* U, int64_t ldu,
                         const FT* V, int64_t ldv, const double* sig, int r,
                         double delta, int apply, double* partial, double* out_sum,
                         hipStream_t st) {
  MC_REQUIRE(r >= 0, kEINVAL, "negative rank");
  const Schedule& S = L.sched_csr;
  // the banded form, as the forward SpMM takes it, once the gathered rows of
  // V outgrow one XCD's L2: each XCD then gathers from its own column band
  // (a row cut at the bands needs no partial sums here: every nonzero's dot
  // product is whole within its piece)
  const bool band = S.band_nseg > 0 &&
                    S.gathered * (int64_t)std::max(r, 1) * (int64_t)sizeof(FT) >= kBandPanelBytes;
  const int64_t nseg = band ? S.band_nseg : S.nseg;
  const int4* segs = band ? S.band_segs.p : S.segs.p;
  const int64_t nb = std::max<int64_t>(1, ceil_div(nseg, kSpmmWaves));
#define MC_SDDMM(BW, CPL)                                                           \
  hipLaunchKernelGGL((sddmm_update_kernel<FT, AT, VT, WT, BW, CPL>), dim3((unsigned)nb), \
                     dim3(64 * kSpmmWaves), 0, st, nseg, segs, L.col_idx.p, mvals,      \
                     y, yv, ycv, yw, ycw, L.invperm.p, U, ldu, V, ldv, sig, r, delta,  \
                     apply, partial)
  // lanes per nonzero and columns per lane as the SpMM's forms
  if (r <= 8)
    MC_SDDMM(8, 1);
  else if (r <= 16)
    MC_SDDMM(16, 1);
  else if (r <= 24)
    MC_SDDMM(8, 3);
  else if (r <= 32)
    MC_SDDMM(16, 2);
  else if (r <= 40)
    MC_SDDMM(8, 5);
  else if (r <= 48)
    MC_SDDMM(16, 3);
  else if (r <= 56)
    MC_SDDMM(8, 7);
  else if (r <= 64)
    MC_SDDMM(16, 4);
  else if (r <= 80)
    MC_SDDMM(16, 5);
  else if (r <= 96)
    MC_SDDMM(16, 6);
  else if (r <= 112)
    MC_SDDMM(16, 7);
  else
    MC_SDDMM(32, 4);                 // passes of 128 columns
#undef MC_SDDMM
  MC_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, nb, partial,
                     out_sum);
  MC_CHECK_LAUNCH();
}
template void launch_sddmm_update<double, double, double, double>(
    const Layout&, const double*, double*, double*, double*, double*, double*,
    const double*, int64_t, const double*, int64_t, const double*, int, double, int,
    double*, double*, hipStream_t);
template void launch_sddmm_update<float, float, float, float>(
    const Layout&, const double*, double*, float*, float*, float*, float*,
    const float*, int64_t, const float*, int64_t, const double*, int, double, int,
    double*, double*, hipStream_t);
template void launch_sddmm_update<float, float, bf16_t, float>(
    const Layout&, const double*, double*, bf16_t*, bf16_t*, float*, float*,
    const float*, int64_t, const float*, int64_t, const double*, int, double, int,
    double*, double*, hipStream_t);

template <class FT>
void launch_eval_observed(const Layout& L, const FT* U, int64_t ldu,
                          const FT* V, int64_t ldv, const double* sig, int r,
                          double* out_input_order, hipStream_t st) {
  hipLaunchKernelGGL(eval_observed_kernel<FT>, dim3(grid_for(L.nnz, 256)),
                     dim3(256), 0, st, L.nnz, L.row_of.p, L.col_idx.p, U, ldu,
                     V, ldv, sig, r, L.order.p, out_input_order);
  MC_CHECK_LAUNCH();
}
template void launch_eval_observed<double>(const Layout&, const double*,
                                           int64_t, const double*, int64_t,
                                           const double*, int, double*,
                                           hipStream_t);
template void launch_eval_observed<float>(const Layout&, const float*, int64_t,
                                          const float*, int64_t, const double*,
                                          int, double*, hipStream_t);

void launch_sumsq(int64_t n, const double* a, double* partial, double* out,
                  hipStream_t st) {
  const int64_t nb = ceil_div(n, 256);
  hipLaunchKernelGGL(sumsq_kernel, dim3((unsigned)nb), dim3(256), 0, st, n, a,
                     partial);
  MC_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, nb, partial,
                     out);
  MC_CHECK_LAUNCH();
}

void launch_scale(int64_t n, const double* a, double alpha, double* out,
                  hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, n,
                     a, alpha, out);
  MC_CHECK_LAUNCH();
}

}  // namespace mcsvt
