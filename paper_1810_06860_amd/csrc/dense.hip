// Dense kernels of rSVD-BKI and eigSVD.
//
// * gram:  C = A^T B for tall-skinny A (N x p), B (N x q), row-major.  The
//   N dimension is split over workgroups; each writes its partial tile and a
//   second kernel sums the partials in a fixed order (deterministic).  Used
//   for the Gram B B^T of eigSVD (Alg. 3) and for the Gram / cross-Gram
//   products of the block orthonormalisation of the Krylov blocks.  The
//   products run on the matrix cores (16x16x4 FP64 or FP32 MFMA); the fused
//   form for short blocks (completion and Cholesky in the last workgroup)
//   uses vector FMAs on 32 x 32 tiles.
// * panel GEMM:  C = beta C0 + alpha X W diag(colscale), X tall (N x p),
//   W small (p x q).  Used for H - Q (Q^T H), H R^-1, U = Q W and
//   V = B^T W S^-1 (Alg. 3, Alg. 5).
// * Cholesky + triangular inverse of a small SPD matrix in one workgroup,
//   with a diagonal shift when a pivot breaks down (shifted Cholesky QR).
#include <type_traits>

#include "chol_regs.hpp"
#include "kernels.hpp"

namespace mcsvt {

namespace {

constexpr int GT = 32;   // gram tile
constexpr int GramTailThreads = 256;   // workgroup size of the fused Gram

// G (b x b, SPD; its upper triangle is read) = R^T R and Rinv = R^{-1}
// (upper triangular, zeros below), in one workgroup.  Gaussian elimination
// without pivoting on [G | I], in place in A (b x b): after step j the rows
// i > j hold the Schur complement on and above the diagonal and, below it,
// the row operations applied so far to I (L^{-1}, unit diagonal implied), so
// no separate triangular inversion follows.  With G = L D L^T, R = D^{1/2} L^T
// and R^{-1} = L^{-T} D^{-1/2}: Rinv[a][c] = Linv[c][a] / sqrt(d_c), a <= c.
// One barrier per column.  A pivot that is not positive or falls below 1e-13
// of its original diagonal retries with G + shift I (shifted Cholesky QR).
// aux holds 2 b doubles.  NC = ceil(b / 32) column strides of a lane (0: any b).
template <int NC>
__device__ __forceinline__ void chol_inv_block_nc(int b, const double* __restrict__ G, int64_t ldg,
                                  double* __restrict__ Rinv, int64_t ldr, double* A,
                                  double* aux, int64_t nrows, int* __restrict__ shifted,
                                  int* __restrict__ flag) {
  __shared__ double trace;
  const int tid = threadIdx.x;
  const int tx = tid & 31, ty = tid >> 5, ny = (int)(blockDim.x >> 5);
  // the diagonal of G in LDS: the breakdown test reads it every column
  double* gd = aux;
  double* sc = aux + b;
  for (int i = tid; i < b; i += blockDim.x) gd[i] = G[(int64_t)i * ldg + i];
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < b; ++i) t += gd[i];
    trace = t;
  }
  __syncthreads();
  const double u = 1.1102230246251565e-16;
  double shift = 0.0;
  // a lane's columns, clamped into the row so every load is in range
  // (NC = 0: any b, plain loops)
  int cc[NC > 0 ? NC : 1];
#pragma unroll
  for (int m = 0; m < NC; ++m) cc[m] = min(tx + 32 * m, b - 1);
  for (int attempt = 0; attempt < 6; ++attempt) {
    // the upper triangle of G (lower one zeroed by a factor: no branch
    // around the load)
    for (int i = ty; i < b; i += ny)
      for (int c = tx; c < b; c += 32) {
        double v = G[(int64_t)i * ldg + c] * (i <= c ? 1.0 : 0.0);
        if (i == c) v += shift;
        A[i * b + c] = v;
      }
    __syncthreads();
    bool failed = false;
    for (int j = 0; j < b; ++j) {
      // a pivot below 1e-13 of its original diagonal means kappa(H) of
      // order 1e6 or worse: Cholesky QR would lose all orthogonality
      const double d = A[j * b + j];
      const double gjj = gd[j] + shift;
      if (!(d > 1e-13 * gjj) || !(d > 1e-300)) {
        failed = true;                               // the same for every thread
        break;
      }
      const double rd = rcp_nr(d);
      // row j is only read in this step: its Schur part (c >= j) and its
      // L^{-1} part (c < j)
      if constexpr (NC > 0) {
        double rj[NC];
#pragma unroll
        for (int m = 0; m < NC; ++m) rj[m] = A[j * b + cc[m]];
        for (int i = j + 1 + ty; i < b; i += ny) {
          const double l = A[j * b + i] * rd;        // multiplier of row i
          double v[NC];
#pragma unroll
          for (int m = 0; m < NC; ++m) v[m] = A[i * b + cc[m]];
#pragma unroll
          for (int m = 0; m < NC; ++m) {
            const int c = tx + 32 * m;
            if (c < b) {
              if (c >= i || c < j)
                A[i * b + c] = v[m] - l * rj[m];
              else if (c == j)
                A[i * b + c] = -l;                   // L^{-1}[j][j] = 1
            }
          }
        }
      } else {
        for (int i = j + 1 + ty; i < b; i += ny) {
          const double l = A[j * b + i] * rd;
          for (int c = tx; c < b; c += 32) {
            if (c >= i || c < j)
              A[i * b + c] -= l * A[j * b + c];
            else if (c == j)
              A[i * b + c] = -l;
          }
        }
      }
      __syncthreads();
    }
    if (!failed) break;
    // shifted Cholesky QR: s = 11 (N b + b (b + 1)) u ||X||^2, ||X||^2 <= tr G
    shift = (shift == 0.0)
                ? 11.0 * ((double)nrows * b + (double)b * (b + 1)) * u *
                      fmax(trace, 1e-300)
                : shift * 100.0;
    if (tid == 0 && shifted) atomicAdd(shifted, 1);
    if (tid == 0 && flag) *flag = 1;
    __syncthreads();
  }
  for (int i = tid; i < b; i += blockDim.x) sc[i] = 1.0 / sqrt(A[i * b + i]);
  __syncthreads();
  for (int a = ty; a < b; a += ny)
    for (int c = tx; c < b; c += 32) {
      const double lv = A[c * b + min(a, c)] * (a < c ? 1.0 : 0.0) + (a == c ? 1.0 : 0.0);
      Rinv[(int64_t)a * ldr + c] = lv * sc[c];
    }
}

__device__ __forceinline__ void chol_inv_block(int b, const double* __restrict__ G, int64_t ldg,
                               double* __restrict__ Rinv, int64_t ldr, double* A,
                               double* aux, int64_t nrows, int* __restrict__ shifted,
                               int* __restrict__ flag) {
  if (b <= 32)
    chol_inv_block_nc<1>(b, G, ldg, Rinv, ldr, A, aux, nrows, shifted, flag);
  else if (b <= 64)
    chol_inv_block_nc<2>(b, G, ldg, Rinv, ldr, A, aux, nrows, shifted, flag);
  else if (b <= 96)
    chol_inv_block_nc<3>(b, G, ldg, Rinv, ldr, A, aux, nrows, shifted, flag);
  else if (b <= 128)
    chol_inv_block_nc<4>(b, G, ldg, Rinv, ldr, A, aux, nrows, shifted, flag);
  else
    chol_inv_block_nc<0>(b, G, ldg, Rinv, ldr, A, aux, nrows, shifted, flag);
}

// Fused completion (mode 1: sum the partials into C; mode 2: also Cholesky +
// R^{-1} of C, p = q): every participating workgroup counts itself on
// `counter` after its partial is written; the last one does the completion
// and resets the counter (no waiting on other workgroups).
struct GramTail {
  int mode = 0;
  int* counter = nullptr;
  int expected = 0, nsplit = 0;
  double* C = nullptr;
  int64_t ldc = 0;
  double* Rinv = nullptr;
  int64_t ldr = 0, nrows = 0;
  int* shifted = nullptr;
  int* flag = nullptr;
};

template <class IT, class AT>
__global__ __launch_bounds__(GramTailThreads) void gram_kernel(
    int64_t N, int p, int q, const IT* __restrict__ A, int64_t lda,
    const IT* __restrict__ B, int64_t ldb, AT* __restrict__ part,
    int64_t rows_per_split, int sym, const int* __restrict__ gate, GramTail tail) {
  if (gate && *gate == 0) return;
  const int ti = blockIdx.x, tj = blockIdx.y, sp = blockIdx.z;
  if (sym && tj < ti) return;
  __shared__ AT As[GT][GT + 1];
  __shared__ AT Bs[GT][GT + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  AT acc00 = 0, acc01 = 0, acc10 = 0, acc11 = 0;
  const int64_t n0 = (int64_t)sp * rows_per_split;
  const int64_t n1 = min(N, n0 + rows_per_split);
  const int a0 = ti * GT, b0 = tj * GT;
  // Out-of-range elements load from a clamped in-range address and are
  // zeroed by a factor 0 (not a select, which the compiler would turn back
  // into a branch around each load and a wait after it).
  const int c = threadIdx.x % GT;
  const AT fa = a0 + c < p ? AT(1) : AT(0), fb = b0 + c < q ? AT(1) : AT(0);
  const IT* Ac = A + (a0 + c < p ? a0 + c : 0);
  const IT* Bc = B + (b0 + c < q ? b0 + c : 0);
  for (int64_t nb = n0; nb < n1; nb += GT) {
    AT va[GT * GT / 256], vb[GT * GT / 256];
#pragma unroll
    for (int i = 0; i < GT * GT / 256; ++i) {
      const int64_t row = nb + threadIdx.x / GT + (256 / GT) * i;
      const bool rin = row < n1;
      const int64_t rr = rin ? row : n0;
      const AT m = rin ? AT(1) : AT(0);
      va[i] = (AT)Ac[rr * lda] * (m * fa);
      vb[i] = (AT)Bc[rr * ldb] * (m * fb);
    }
#pragma unroll
    for (int i = 0; i < GT * GT / 256; ++i) {
      As[threadIdx.x / GT + (256 / GT) * i][c] = va[i];
      Bs[threadIdx.x / GT + (256 / GT) * i][c] = vb[i];
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < GT; ++kk) {
      const AT x0 = As[kk][ty * 2], x1 = As[kk][ty * 2 + 1];
      const AT y0 = Bs[kk][tx * 2], y1 = Bs[kk][tx * 2 + 1];
      acc00 += x0 * y0;
      acc01 += x0 * y1;
      acc10 += x1 * y0;
      acc11 += x1 * y1;
    }
    __syncthreads();
  }
  AT* out = part + (int64_t)sp * p * q;
  const int i0 = a0 + ty * 2, j0 = b0 + tx * 2;
  if (i0 < p && j0 < q) out[(int64_t)i0 * q + j0] = acc00;
  if (i0 < p && j0 + 1 < q) out[(int64_t)i0 * q + j0 + 1] = acc01;
  if (i0 + 1 < p && j0 < q) out[(int64_t)(i0 + 1) * q + j0] = acc10;
  if (i0 + 1 < p && j0 + 1 < q) out[(int64_t)(i0 + 1) * q + j0 + 1] = acc11;
  if (tail.mode == 0) return;
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(tail.counter, 1) == tail.expected - 1;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  extern __shared__ double lds[];
  // the register Cholesky (p <= 64) reads the summed Gram from LDS, after its
  // own 3 p doubles
  const bool g_lds = tail.mode == 2 && p <= 64;
  double* Gl = lds + 3 * p;
  const int64_t tot = (int64_t)p * q;
  const int nt = (int)blockDim.x;
  for (int64_t t = threadIdx.x; t < tot; t += 2 * nt) {
    // two entries per thread, the split loads of both in flight together
    // (groups of 16), each summed in split order
    const int64_t t2 = t + nt < tot ? t + nt : t;
    const AT* pp[2];
    for (int e = 0; e < 2; ++e) {
      const int64_t te = e ? t2 : t;
      const int i = (int)(te / q), j = (int)(te % q);
      int si = i, sj = j;
      if (sym && (i / GT) > (j / GT)) { si = j; sj = i; }   // mirrored tile
      pp[e] = part + (int64_t)si * q + sj;
    }
    double acc[2] = {0.0, 0.0};
    int sp2 = 0;
    for (; sp2 + 16 <= tail.nsplit; sp2 += 16) {
      double v[2][16];
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int u = 0; u < 16; ++u) v[e][u] = (double)pp[e][(int64_t)(sp2 + u) * tot];
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[e] += v[e][u];
    }
    for (; sp2 + 4 <= tail.nsplit; sp2 += 4) {
      double v[2][4];
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int u = 0; u < 4; ++u) v[e][u] = (double)pp[e][(int64_t)(sp2 + u) * tot];
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[e] += v[e][u];
    }
    for (; sp2 < tail.nsplit; ++sp2)
      for (int e = 0; e < 2; ++e) acc[e] += (double)pp[e][(int64_t)sp2 * tot];
    for (int e = 0; e < 2; ++e) {
      if (e == 1 && t2 == t) break;
      const int64_t te = e ? t2 : t;
      const int i = (int)(te / q), j = (int)(te % q);
      tail.C[(int64_t)i * tail.ldc + j] = acc[e];
      if (g_lds) Gl[te] = acc[e];
    }
  }
  if (!g_lds) __threadfence();                       // the LDS form reads C back
  __syncthreads();
  if (tail.mode == 2) {
    // 256 threads: 8 rows of 32 lanes; in registers up to p = 64, else the
    // elimination array in LDS: A (p x p), aux (2 p)
    static_assert(GramTailThreads == 256, "register tiles assume 8 thread rows");
    const double* Cc = g_lds ? Gl : tail.C;
    const int64_t lc = g_lds ? p : tail.ldc;
    if (p <= 8)
      chol_inv_regs<1, 1>(p, Cc, lc, tail.Rinv, tail.ldr, lds, tail.nrows, tail.shifted,
                          tail.flag, false);
    else if (p <= 16)
      chol_inv_regs<2, 1>(p, Cc, lc, tail.Rinv, tail.ldr, lds, tail.nrows, tail.shifted,
                          tail.flag, false);
    else if (p <= 24)
      chol_inv_regs<3, 1>(p, Cc, lc, tail.Rinv, tail.ldr, lds, tail.nrows, tail.shifted,
                          tail.flag, false);
    else if (p <= 32)
      chol_inv_regs<4, 1>(p, Cc, lc, tail.Rinv, tail.ldr, lds, tail.nrows, tail.shifted,
                          tail.flag, false);
    else if (p <= 64)
      chol_inv_regs<8, 2>(p, Cc, lc, tail.Rinv, tail.ldr, lds, tail.nrows, tail.shifted,
                          tail.flag, false);
    else
      chol_inv_block(p, Cc, lc, tail.Rinv, tail.ldr, lds, lds + (size_t)p * p, tail.nrows,
                     tail.shifted, tail.flag);
  }
  if (threadIdx.x == 0) *tail.counter = 0;
}

// Matrix-core Gram: the same partial products as gram_kernel, computed with
// the 16x16x4 FP64 / FP32 MFMA instructions.  A workgroup owns a 128 x 128
// output block and a range of rows, so each row of A and B is read by as few
// workgroups as possible.  The block's 16 x 16 instruction tiles that lie in
// p x q -- and, on a diagonal block of a symmetric product, on or above the
// diagonal (the reduction reads the others mirrored, granularity 16) -- are
// dealt round-robin to the four wavefronts, so no wavefront computes tiles
// outside the result and the matrix cores of the four SIMDs stay evenly
// loaded whatever p and q are.  Rows pass through LDS 16 at a time, loaded
// one stage ahead into registers.
constexpr int MB = 128;  // output block of gram_mfma_kernel
constexpr int MT = 16;   // instruction tile; mirror granularity
constexpr int MK = 16;   // rows per LDS stage

template <class T> struct Mfma16;
template <> struct Mfma16<double> {
  typedef double V __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V op(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held in element v of a lane (column lane % 16)
  static __device__ __forceinline__ int row(int lane, int v) { return lane / 16 + 4 * v; }
};
template <> struct Mfma16<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V op(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane / 16) + v; }
};

// The row loop of gram_mfma_kernel: SAME (diagonal block of a symmetric
// product: B is A), up to TW instruction tiles per wavefront (tile t of this
// wavefront is (ti[t], tj[t]) in units of 16 inside the block, nt of them;
// GRID: the tiles form a TW / 4 x 4 grid, tile t at row t / 4 and column
// t % 4 of it, and nt is the mask of the live ones).  Only the last, partial
// stage uses row-guarded loads.
template <class T, bool SAME, int TW, bool GRID>
__device__ __forceinline__ void gram_mfma_rows(
    int64_t n0, int64_t n1, int p, int q, const T* __restrict__ A, int64_t lda,
    const T* __restrict__ B, int64_t ldb, T* __restrict__ out, int a0, int b0,
    const int* ti, const int* tj, int nt, T (*As)[MB + 1], T (*Bs)[MB + 1]) {
  using M = Mfma16<T>;
  using V = typename M::V;
  constexpr int LPT = MK * MB / 256;          // elements per thread and stage
  const int lane = threadIdx.x & 63;
  const int lc = threadIdx.x & (MB - 1), lr = threadIdx.x / MB;
  const bool acol = a0 + lc < p, bcol = b0 + lc < q;
  // thread's column of A (B); rows lr, lr + 2, ..., lr + 14 of a stage
  const T* Ac = A + (acol ? a0 + lc : 0) + lr * lda;
  const T* Bc = B + (bcol ? b0 + lc : 0) + lr * ldb;
  T ra[LPT], rb[LPT];
  auto fetch = [&](int64_t nb) {
    if (nb + MK <= n1) {
#pragma unroll
      for (int i = 0; i < LPT; ++i) {
        ra[i] = Ac[(nb + 2 * i) * lda];
        if (!SAME) rb[i] = Bc[(nb + 2 * i) * ldb];
      }
    } else {
#pragma unroll
      for (int i = 0; i < LPT; ++i) {
        const bool rin = nb + lr + 2 * i < n1;
        ra[i] = rin ? Ac[(nb + 2 * i) * lda] : T(0);
        if (!SAME) rb[i] = rin ? Bc[(nb + 2 * i) * ldb] : T(0);
      }
    }
  };
  V acc[TW];
#pragma unroll
  for (int t = 0; t < TW; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[t][v] = T(0);
  const int cc = lane % 16, kq = lane / 16;
  fetch(n0);
  for (int64_t nb = n0; nb < n1; nb += MK) {
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      As[lr + 2 * i][lc] = acol ? ra[i] : T(0);
      if (!SAME) Bs[lr + 2 * i][lc] = bcol ? rb[i] : T(0);
    }
    __syncthreads();
    if (nb + MK < n1) fetch(nb + MK);         // in flight during the products
    T(*Bt)[MB + 1] = SAME ? As : Bs;
    auto step4 = [&](int kk) {
      const int kr = kk + kq;
      if constexpr (GRID) {
        // a TW / 4 x 4 grid of tiles: TW / 4 + 4 operands serve TW
        // products; nt is the mask of the live tiles
        T x[TW / 4], y[4];
#pragma unroll
        for (int i = 0; i < TW / 4; ++i) x[i] = As[kr][ti[4 * i] * 16 + cc];
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j] = Bt[kr][tj[j] * 16 + cc];
#pragma unroll
        for (int t = 0; t < TW; ++t)
          if ((nt >> t) & 1) acc[t] = M::op(x[t / 4], y[t % 4], acc[t]);
      } else {
#pragma unroll
        for (int t = 0; t < TW; ++t) {
          if (t < nt) {                        // uniform across the wavefront
            const T x = As[kr][ti[t] * 16 + cc];
            const T y = Bt[kr][tj[t] * 16 + cc];
            acc[t] = M::op(x, y, acc[t]);
          }
        }
      }
    };
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int kk = 0; kk < MK; kk += 4) step4(kk);
    } else {
      // FP32: one 4-row step at a time; unrolled across the stage the
      // compiler hoists every step's LDS operands and runs out of registers
      // (at eight tiles per wavefront one wavefront per SIMD, five times the
      // FP64 time); FP64 keeps the unrolled form, which measured faster
#pragma unroll 1
      for (int kk = 0; kk < MK; kk += 4) step4(kk);
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    if (GRID ? !((nt >> t) & 1) : t >= nt) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = a0 + ti[t] * 16 + M::row(lane, v);
      const int c = b0 + tj[t] * 16 + cc;
      if (r < p && c < q) out[(int64_t)r * q + c] = acc[t][v];
    }
  }
}

template <class T, int TW>
__global__ __launch_bounds__(256) void gram_mfma_kernel(
    int64_t N, int p, int q, const T* __restrict__ A, int64_t lda,
    const T* __restrict__ B, int64_t ldb, T* __restrict__ part,
    int64_t rows_per_split, int sym, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int bi = blockIdx.x, bj = blockIdx.y, sp = blockIdx.z;
  if (sym && bj < bi) return;
  __shared__ T As[MK][MB + 1];
  __shared__ T Bs[MK][MB + 1];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int a0 = bi * MB, b0 = bj * MB;
  const int64_t n0 = (int64_t)sp * rows_per_split;
  const int64_t n1 = min(N, n0 + rows_per_split);
  if (n0 >= n1) return;
  const bool same = sym && bi == bj;
  // the block's tiles inside p x q (upper ones on a symmetric diagonal
  // block) in row-major order; this wavefront takes tiles w, w + 4, ...
  const int nti = min(MB / 16, (p - a0 + 15) / 16);
  const int ntj = min(MB / 16, (q - b0 + 15) / 16);
  const int total = same ? nti * (nti + 1) / 2 : nti * ntj;
  const int nt = min(TW, (total - w + 3) / 4);
  int ti[TW], tj[TW];
  T* out = part + (int64_t)sp * p * q;
  if constexpr (TW == 16) {
    // sixteen tiles per wavefront: wavefront w takes the 4 x 4 tiles at
    // (4 (w / 2), 4 (w % 2)) of the block's 8 x 8, so that each 4-row step
    // reads four operands of each side for sixteen products; the tiles
    // inside p x q (on or above the diagonal of a symmetric diagonal block)
    // are live.  (Dealt out one by one, every product reads two operands.)
    const int gi0 = 4 * (w / 2), gj0 = 4 * (w % 2);
    int live = 0;
#pragma unroll
    for (int t = 0; t < TW; ++t) {
      ti[t] = gi0 + t / 4;
      tj[t] = gj0 + t % 4;
      if (ti[t] < nti && tj[t] < ntj && (!same || ti[t] <= tj[t])) live |= 1 << t;
    }
    if (same)
      gram_mfma_rows<T, true, TW, true>(n0, n1, p, q, A, lda, B, ldb, out, a0, b0, ti, tj,
                                        live, As, Bs);
    else
      gram_mfma_rows<T, false, TW, true>(n0, n1, p, q, A, lda, B, ldb, out, a0, b0, ti, tj,
                                         live, As, Bs);
    return;
  }
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    int g = w + 4 * t, i = 0;
    if (same) {
      while (i < nti - 1 && g >= ntj - i) {
        g -= ntj - i;
        ++i;
      }
      ti[t] = i;
      tj[t] = i + g;
    } else {
      ti[t] = g / ntj;
      tj[t] = g % ntj;
    }
  }
  if (same)
    gram_mfma_rows<T, true, TW, false>(n0, n1, p, q, A, lda, B, ldb, out, a0, b0, ti, tj,
                                       nt, As, Bs);
  else
    gram_mfma_rows<T, false, TW, false>(n0, n1, p, q, A, lda, B, ldb, out, a0, b0, ti, tj,
                                        nt, As, Bs);
}

// Tall Gram with a single output block (p, q <= 16 NT): every wavefront
// keeps all the block's 16 x 16 tiles (the upper NT (NT + 1) / 2 of a
// symmetric product, else NT x NT) and takes its own 4-row steps, loading
// the MFMA operands straight from memory (a lane reads row 4 s + lane / 16,
// column 16 i + lane % 16 of tile column i), so the row loop has no LDS
// traffic and no barriers and keeps many loads in flight.  The four
// wavefronts' tiles are summed through LDS, one tile at a time, into the
// workgroup's partial (p x q, lower tiles of a symmetric product left for
// the reduction to mirror at granularity 16).
constexpr int kRowsUnroll = 2;      // 4-row steps whose loads are issued together

template <class T, int NT, bool SYM>
__global__ __launch_bounds__(256) void gram_rows_kernel(
    int64_t N, int p, int q, const T* __restrict__ A, int64_t lda,
    const T* __restrict__ B, int64_t ldb, T* __restrict__ part,
    const int* __restrict__ gate) {
  using M = Mfma16<T>;
  using V = typename M::V;
  constexpr int NTILE = SYM ? NT * (NT + 1) / 2 : NT * NT;
  if (gate && *gate == 0) return;
  __shared__ T red[4][256];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int cc = lane % 16, kq = lane / 16;
  V acc[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[t][v] = T(0);
  bool acol[NT], bcol[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    acol[i] = i * 16 + cc < p;
    bcol[i] = i * 16 + cc < q;
  }
  const int64_t steps = (N + 3) / 4;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t s0 = (int64_t)blockIdx.x * 4 + w; s0 < steps; s0 += nw * kRowsUnroll) {
    T a[kRowsUnroll][NT], b[kRowsUnroll][SYM ? 1 : NT];
#pragma unroll
    for (int u = 0; u < kRowsUnroll; ++u) {
      const int64_t row = (s0 + u * nw) * 4 + kq;
      const bool rin = row < N;
      const T* ar = A + (rin ? row : 0) * lda;
      const T* br = B + (rin ? row : 0) * ldb;
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        a[u][i] = (rin && acol[i]) ? ar[i * 16 + cc] : T(0);
        if (!SYM) b[u][i] = (rin && bcol[i]) ? br[i * 16 + cc] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < kRowsUnroll; ++u) {
      int t = 0;
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = SYM ? i : 0; j < NT; ++j, ++t)
          acc[t] = M::op(a[u][i], SYM ? a[u][j] : b[u][j], acc[t]);
    }
  }
  // the four wavefronts' tiles into the workgroup's partial
  T* out = part + (int64_t)blockIdx.x * p * q;
  int t = 0;
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = SYM ? i : 0; j < NT; ++j, ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w][v * 64 + lane] = acc[t][v];
      __syncthreads();
      {
        const int v = threadIdx.x / 64, l = threadIdx.x % 64;
        const T sum = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                      (red[2][threadIdx.x] + red[3][threadIdx.x]);
        const int r = i * 16 + M::row(l, v), c = j * 16 + l % 16;
        if (r < p && c < q) out[(int64_t)r * q + c] = sum;
      }
      __syncthreads();
    }
}

// The row-streaming Gram on the BF16 matrix cores (16x16x16 MFMA, FP32
// accumulation) for FP32 panels: each 16-row step rounds its operands to BF16
// on load (a lane packs rows 16 s + 4 (lane / 16) + 0..3 of column
// 16 i + lane % 16), so one instruction covers four times the rows of the
// FP32 form.  Products of BF16 values are exact in FP32; only the rounding
// of the operands and the FP32 sums differ from the FP32 Gram.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float f) {
  return (short)bf16_t(f).bits;
}

template <int NT, bool SYM>
__global__ __launch_bounds__(256) void gram_rows_bf16_kernel(
    int64_t N, int p, int q, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, float* __restrict__ part) {
  using V = Mfma16<float>::V;
  constexpr int NTILE = SYM ? NT * (NT + 1) / 2 : NT * NT;
  __shared__ float red[4][256];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int cc = lane % 16, kq = lane / 16;
  V acc[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[t][v] = 0.0f;
  bool acol[NT], bcol[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    acol[i] = i * 16 + cc < p;
    bcol[i] = i * 16 + cc < q;
  }
  const int64_t steps = (N + 15) / 16;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t s = (int64_t)blockIdx.x * 4 + w; s < steps; s += nw) {
    bf16x4_t a[NT], b[SYM ? 1 : NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t row = s * 16 + kq * 4 + j;
        const bool rin = row < N;
        const int64_t rr = rin ? row : 0;
        a[i][j] = bf16_bits((rin && acol[i]) ? A[rr * lda + i * 16 + cc] : 0.0f);
        if (!SYM) b[i][j] = bf16_bits((rin && bcol[i]) ? B[rr * ldb + i * 16 + cc] : 0.0f);
      }
    }
    int t = 0;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = SYM ? i : 0; j < NT; ++j, ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], SYM ? a[j] : b[j],
                                                            acc[t], 0, 0, 0);
  }
  float* out = part + (int64_t)blockIdx.x * p * q;
  int t = 0;
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = SYM ? i : 0; j < NT; ++j, ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w][v * 64 + lane] = acc[t][v];
      __syncthreads();
      {
        const int v = threadIdx.x / 64, l = threadIdx.x % 64;
        const float sum = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                          (red[2][threadIdx.x] + red[3][threadIdx.x]);
        const int r = i * 16 + Mfma16<float>::row(l, v), c = j * 16 + l % 16;
        if (r < p && c < q) out[(int64_t)r * q + c] = sum;
      }
      __syncthreads();
    }
}

// Sum of the split partials.  A wavefront covers 64 / lanes consecutive
// outputs with `lanes` threads each (lanes a power of two, at most 16): lane
// (u, o) -- output o, u = lane / (64 / lanes) -- adds the splits u, u + lanes,
// ... in order, so that for each split the wavefront reads its outputs'
// entries side by side; the `lanes` partial sums of an output are then
// combined by a fixed butterfly, so the result does not depend on scheduling.
template <class AT>
__global__ __launch_bounds__(256) void gram_reduce_kernel(
    int p, int q, int nsplit, int lanes, const AT* __restrict__ part,
    double* __restrict__ C, int64_t ldc, int sym, int tile, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int outs = 64 / lanes;                 // outputs per wavefront
  const int lane = threadIdx.x & 63;
  const int o = lane % outs, u = lane / outs;
  const int64_t t = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * outs + o;
  const int64_t tot = (int64_t)p * q;
  int i = 0, j = 0;
  if (t < tot) {
    i = (int)(t / q);
    j = (int)(t % q);
  }
  // a symmetric product's partials hold the tiles on and above the diagonal:
  // those entries are read (side by side) and the ones below are written as
  // their mirror images
  const bool live = t < tot && !(sym && (i / tile) > (j / tile));
  const bool mirror = sym && (i / tile) < (j / tile);
  double acc = 0.0;
  if (live) {
    // the partials were written by other workgroups (other XCDs): their loads
    // go out sixteen at a time, and are added in split order
    const AT* __restrict__ pp = part + (int64_t)i * q + j;
    int s = u;
    for (; s + 15 * lanes < nsplit; s += 16 * lanes) {
      AT v[16];
#pragma unroll
      for (int w = 0; w < 16; ++w) v[w] = pp[(int64_t)(s + w * lanes) * tot];
#pragma unroll
      for (int w = 0; w < 16; ++w) acc += (double)v[w];
    }
    for (; s < nsplit; s += lanes) acc += (double)pp[(int64_t)s * tot];
  }
  for (int w = outs; w < 64; w <<= 1) acc += __shfl_xor(acc, w, 64);
  if (live && u == 0) {
    C[(int64_t)i * ldc + j] = acc;
    if (mirror) C[(int64_t)j * ldc + i] = acc;
  }
}

// C = beta*C0 + alpha * X W diag(colscale), X tall (N x p), W small (p x q),
// on the FP64 matrix cores.  A workgroup owns 64 rows and up to 128 columns
// (NT tiles of 16), so X is read once for q <= 128; each wavefront owns 16
// rows x NT 16-column instruction tiles.  W passes through LDS in chunks of
// QK rows; each lane reads its A operands (X converted to FP64) straight
// from memory, the next chunk's while the matrix cores work on this one.
// QK = 16 up to three column tiles, 32 beyond (measured: 42.9 against
// 56.9 us for 140,000 x 48 x 48, 60.2 / 75.3 against 64.2 / 80.3 us for
// 140,000 x 64 x 64 / 96 x 64); the instruction sequence is the same.
constexpr int QR = 64;   // rows per workgroup

template <class XT, class OT, int NT, int QK>
__global__ __launch_bounds__(256) void panel_mfma_kernel(
    int64_t N, int p, int q, const XT* __restrict__ X, int64_t ldx,
    const double* __restrict__ W, int64_t ldw, double alpha,
    const double* __restrict__ colscale, double beta,
    const OT* __restrict__ C0, int64_t ldc0, OT* __restrict__ C, int64_t ldc,
    const int* __restrict__ gate) {
  using M = Mfma16<double>;
  using V = M::V;
  constexpr int QC = 16 * NT;
  constexpr int KS = QK / 4;                   // 4-deep steps per chunk
  constexpr int WL = QK * QC / 256;            // W entries per thread and chunk
  if (gate && *gate == 0) return;
  __shared__ double Ws[QK][QC + 1];
  const int64_t r0 = (int64_t)blockIdx.x * QR;
  const int c0 = blockIdx.y * QC;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane / 16;
  // this lane's row of X (clamped: rows past N feed outputs that are not
  // stored), as a 32-bit offset from the workgroup's first row
  const XT* __restrict__ Xb = X + r0 * ldx;
  const int64_t xi = r0 + w * 16 + lane % 16;
  const uint32_t xo = (uint32_t)(((xi < N ? xi : N - 1) - r0) * ldx) + (uint32_t)g;
  const double* __restrict__ Wc = W + c0;
  V acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[t][v] = 0.0;
  // the A operand of step s of a chunk: X[row][k0 + 4 s + g], zero past p
  double xa[KS], xn[KS];
  auto fetch = [&](int k0, double* dst) {
    if (k0 + QK <= p) {                        // whole chunk: immediate offsets
#pragma unroll
      for (int s = 0; s < KS; ++s) dst[s] = (double)Xb[xo + (uint32_t)(k0 + 4 * s)];
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = k0 + 4 * s + g;
        const double v = (double)Xb[xo - (uint32_t)g + (uint32_t)(k < p ? k : p - 1)];
        dst[s] = k < p ? v : 0.0;
      }
    }
  };
  if (p > 0) {
    fetch(0, xa);
  } else {
#pragma unroll
    for (int s = 0; s < KS; ++s) xa[s] = 0.0;
  }
  for (int k0 = 0; k0 < p; k0 += QK) {
    double wv[WL];
#pragma unroll
    for (int i = 0; i < WL; ++i) {
      const int t = threadIdx.x + 256 * i, r = t / QC, c = t % QC;
      const bool ok = k0 + r < p && c0 + c < q;
      const double v = Wc[ok ? (uint32_t)((k0 + r) * ldw + c) : 0u];
      wv[i] = ok ? v : 0.0;
    }
    const bool more = k0 + QK < p;
    if (more) fetch(k0 + QK, xn);              // the next chunk's X in flight meanwhile
#pragma unroll
    for (int i = 0; i < WL; ++i) {
      const int t = threadIdx.x + 256 * i;
      Ws[t / QC][t % QC] = wv[i];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = M::op(xa[s], Ws[4 * s + g][t * 16 + lane % 16], acc[t]);
    __syncthreads();
    if (more) {
#pragma unroll
      for (int s = 0; s < KS; ++s) xa[s] = xn[s];
    }
  }
  // epilogue: the column scales and C0 entries of all of this lane's outputs
  // are requested together (clamped addresses, uniform conditions), then the
  // results are formed and stored
  double cs[NT], cz[NT][4];
  const OT* __restrict__ Cb = C0 + r0 * ldc0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = min(c0 + t * 16 + lane % 16, q - 1);
    cs[t] = colscale ? colscale[col] : 1.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = min<int64_t>(r0 + w * 16 + M::row(lane, v), N - 1);
      cz[t][v] = beta != 0.0 ? (double)Cb[(uint32_t)((row - r0) * ldc0 + col)] : 0.0;
    }
  }
  OT* __restrict__ Co = C + r0 * ldc;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + w * 16 + M::row(lane, v);
      const int col = c0 + t * 16 + lane % 16;
      if (row < N && col < q) {
        double x = alpha * acc[t][v];
        if (colscale) x *= cs[t];
        if (beta != 0.0) x += beta * cz[t][v];
        Co[(uint32_t)((row - r0) * ldc + col)] = (OT)x;
      }
    }
}

// Gram (or cross-Gram) of a short block in one workgroup on the matrix
// cores: C = A^T B for A (N x p), B (N x q), N <= kSmallRows, at most
// kSmallTiles 16 x 16 output tiles (TP x TQ, or the TP (TP + 1) / 2 upper
// tiles of a symmetric product: SYM, B is A).  Each of the 16 wavefronts
// takes every 16th 4-row step (16x16x4 MFMA; a lane loads row 4 s + lane / 16,
// column lane % 16 of each tile, so operands come straight from memory), the
// wavefronts' tiles are summed in a fixed tree in LDS, and mode 2 (SYM) then
// forms R^{-1} of C = R^T R in registers.  No partial buffer, no counter.
constexpr int kSmallThreads = 1024;
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr int kSmallTiles = 6;
constexpr int64_t kSmallRows = 2048;
constexpr int kSmallUnroll = 4;    // 4-row steps in flight per wavefront (16 measured no faster)

template <class T, bool SYM, int TP, int TQ>
__global__ __launch_bounds__(kSmallThreads) void gram_small_kernel(
    int64_t N, int p, int q, const T* __restrict__ A, int64_t lda,
    const T* __restrict__ B, int64_t ldb, const int* __restrict__ gate, GramTail tail) {
  if (gate && *gate == 0) return;
  using M = Mfma16<T>;
  using V = typename M::V;
  static_assert(!SYM || TP == TQ, "a symmetric product has square tiling");
  constexpr int NT = SYM ? TP * (TP + 1) / 2 : TP * TQ;
  static_assert(NT <= kSmallTiles, "tile count");
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane >> 4, lc = lane & 15;
  // this lane's column in each tile (clamped, zeroed by a factor)
  const T* Ap[TP];
  T fa[TP];
#pragma unroll
  for (int ti = 0; ti < TP; ++ti) {
    const int c = ti * 16 + lc;
    fa[ti] = c < p ? T(1) : T(0);
    Ap[ti] = A + (c < p ? c : 0);
  }
  const T* Bp[TQ];
  T fb[TQ];
#pragma unroll
  for (int tj = 0; tj < TQ; ++tj) {
    const int c = tj * 16 + lc;
    fb[tj] = c < q ? T(1) : T(0);
    Bp[tj] = B + (c < q ? c : 0);
  }
  V acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = V{0, 0, 0, 0};
  const int64_t steps = (N + 3) / 4;
  for (int64_t s0 = w; s0 < steps; s0 += (int64_t)kSmallWaves * kSmallUnroll) {
    T a[kSmallUnroll][TP], b[kSmallUnroll][TQ];
#pragma unroll
    for (int u = 0; u < kSmallUnroll; ++u) {
      const int64_t r = 4 * (s0 + (int64_t)kSmallWaves * u) + lr;
      const bool rin = r < N;
      const int64_t rr = rin ? r : 0;
      const T m = rin ? T(1) : T(0);
#pragma unroll
      for (int ti = 0; ti < TP; ++ti) a[u][ti] = Ap[ti][rr * lda] * (m * fa[ti]);
      if (!SYM) {
#pragma unroll
        for (int tj = 0; tj < TQ; ++tj) b[u][tj] = Bp[tj][rr * ldb] * (m * fb[tj]);
      }
    }
#pragma unroll
    for (int u = 0; u < kSmallUnroll; ++u) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < TP; ++ti)
#pragma unroll
        for (int tj = SYM ? ti : 0; tj < TQ; ++tj, ++t)
          acc[t] = M::op(a[u][ti], SYM ? a[u][tj] : b[u][tj], acc[t]);
    }
  }
  // fixed-order tree over the wavefronts: in round h, wavefronts h .. 2h-1
  // hand their tiles to wavefronts 0 .. h-1 through LDS
  double sum[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) sum[t][v] = (double)acc[t][v];
  for (int h = kSmallWaves / 2; h >= 1; h >>= 1) {
    if (w >= h && w < 2 * h) {
      double* dst = lds + (size_t)(w - h) * NT * 256;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(t * 4 + v) * 64 + lane] = sum[t][v];
    }
    __syncthreads();
    if (w < h) {
      const double* src = lds + (size_t)w * NT * 256;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) sum[t][v] += src[(t * 4 + v) * 64 + lane];
    }
    __syncthreads();
  }
  // wavefront 0 writes C (and, for the Cholesky, a copy in LDS)
  double* Gl = lds;
  const bool chol = tail.mode == 2;
  if (w == 0) {
    int t = 0;
#pragma unroll
    for (int ti = 0; ti < TP; ++ti)
#pragma unroll
      for (int tj = SYM ? ti : 0; tj < TQ; ++tj, ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = ti * 16 + M::row(lane, v), j = tj * 16 + lc;
          if (i < p && j < q) {
            tail.C[(int64_t)i * tail.ldc + j] = sum[t][v];
            if (chol) Gl[i * q + j] = sum[t][v];
            if (SYM && ti != tj) {
              tail.C[(int64_t)j * tail.ldc + i] = sum[t][v];
              if (chol) Gl[j * q + i] = sum[t][v];
            }
          }
        }
  }
  if (!chol) return;
  __syncthreads();
  // 1024 threads: 32 rows of 32 lanes
  double* cl = lds + (size_t)p * q;
  if (p <= 32)
    chol_inv_regs<1, 1>(p, Gl, q, tail.Rinv, tail.ldr, cl, tail.nrows, tail.shifted,
                        tail.flag, false);
  else
    chol_inv_regs<2, 2>(p, Gl, q, tail.Rinv, tail.ldr, cl, tail.nrows, tail.shifted,
                        tail.flag, false);
}

// One workgroup: G (b x b, SPD) = R^T R, Rinv = R^-1 (upper triangular).
// Breakdown (a pivot that is not positive or below 1e-13 of its original
// diagonal) retries with G + shift I.  Elimination on [G | I] with one
// barrier per column: the matrix in registers up to b = 128, else in LDS
// (or, past the LDS size, in `work`).
__global__ __launch_bounds__(1024) void chol_inv_kernel(
    int b, const double* __restrict__ G, int64_t ldg, double* __restrict__ Rinv,
    int64_t ldr, double* __restrict__ work, int64_t nrows,
    int* __restrict__ shifted, int* __restrict__ flag, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double lds[];
  const bool in_lds = b <= kCholLdsMax;
  // 1024 threads: 32 rows of 32 lanes; the matrix in registers up to b = 128
  if (b <= 32)
    chol_inv_regs<1, 1>(b, G, ldg, Rinv, ldr, lds, nrows, shifted, flag, false);
  else if (b <= 64)
    chol_inv_regs<2, 2>(b, G, ldg, Rinv, ldr, lds, nrows, shifted, flag, false);
  else if (b <= 96)
    chol_inv_regs<3, 3>(b, G, ldg, Rinv, ldr, lds, nrows, shifted, flag, false);
  else if (b <= 128)
    chol_inv_regs<4, 4>(b, G, ldg, Rinv, ldr, lds, nrows, shifted, flag, false);
  else {
    double* A = in_lds ? lds : work;                 // b x b, row-major
    double* aux = A + (size_t)b * b;                 // 2 b
    chol_inv_block(b, G, ldg, Rinv, ldr, A, aux, nrows, shifted, flag);
  }
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }

template <class T>
__global__ void copy_gated_kernel(int64_t rows, int cols, const T* __restrict__ src,
                                  int64_t lds_, T* __restrict__ dst, int64_t ldd,
                                  const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int64_t i = t / cols;
  const int j = (int)(t % cols);
  dst[i * ldd + j] = src[i * lds_ + j];
}

// dst (rows x cols, ldd) = src (rows x cols, lds_) converted to D
template <class S, class D>
__global__ void cast_panel_kernel(int64_t rows, int cols, const S* __restrict__ src,
                                  int64_t lds_, D* __restrict__ dst, int64_t ldd) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int64_t i = t / cols;
  const int j = (int)(t % cols);
  dst[i * ldd + j] = (D)src[i * lds_ + j];
}

__global__ void recip_kernel(int k, const double* __restrict__ S,
                             double* __restrict__ out, const int* __restrict__ count,
                             double* __restrict__ count_out, double* __restrict__ host) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) {
    const double s = S[j];
    out[j] = s > 0.0 ? 1.0 / s : 0.0;
    if (host) host[j] = s;
  }
  if (j == 0 && count) {
    const double c = (double)*count;
    count_out[0] = c;
    if (host) host[k] = c;
  }
}

// partial[blk * k + j] = sum over the block's rows of (R_ij - S_j U_ij)^2
template <class T>
__global__ __launch_bounds__(256) void ritz_partial_kernel(
    int64_t m, int k, const T* __restrict__ R, int64_t ldr,
    const T* __restrict__ U, int64_t ldu, const double* __restrict__ S,
    int64_t rows_per_block, double* __restrict__ partial) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double s = S[j];
    double acc = 0.0;
    for (int64_t i = r0; i < r1; ++i) {
      const double d = (double)R[i * ldr + j] - s * (double)U[i * ldu + j];
      acc += d * d;
    }
    partial[(int64_t)blockIdx.x * k + j] = acc;
  }
}

__global__ void ritz_reduce_kernel(int nblk, int k, const double* __restrict__ partial,
                                   const double* __restrict__ S,
                                   double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double acc = 0.0;
  int b = 0;
  for (; b + 8 <= nblk; b += 8) {                // loads eight at a time, added in order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(b + u) * k + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; b < nblk; ++b) acc += partial[(int64_t)b * k + j];
  out[j] = S[j] > 0.0 ? sqrt(acc) / S[j] : INFINITY;
}

}  // namespace

namespace {

// Row splits of the fused Gram (gram_kernel, 32 x 32 tiles).
int64_t fused_splits(int64_t N, int p, int q, int sym) {
  const int64_t tiles = ceil_div(p, GT) * ceil_div(q, GT);
  const int64_t eff = sym ? (tiles + ceil_div(p, GT)) / 2 : tiles;
  // aim at ~2048 workgroups, chunks of at least 64 rows
  int64_t splits = std::max<int64_t>(1, 2048 / std::max<int64_t>(eff, 1));
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, ceil_div(N, 64)));
  return splits;
}

// Row splits of the matrix-core Gram: about 1024 workgroups, at least four
// LDS stages each, and partials of at most half the elements read.
int64_t gram_mfma_splits(int64_t N, int p, int q, int sym) {
  const int64_t blocks = ceil_div(p, MB) * ceil_div(q, MB);
  const int64_t eff = sym ? (blocks + ceil_div(p, MB)) / 2 : blocks;
  // about two workgroups per CU (the occupancy of the wider tilings)
  int64_t splits = std::max<int64_t>(1, 512 / std::max<int64_t>(eff, 1));
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, ceil_div(N, 4 * MK)));
  splits = std::min<int64_t>(
      splits, std::max<int64_t>(1, N * (int64_t)(p + q) / (2 * (int64_t)p * q)));
  return splits;
}

}  // namespace

namespace {
// The row-streaming form takes a single output block whose tiles fit a
// wavefront's registers: a symmetric product up to 112 wide, a cross product
// up to 80 x 80; both only for panels tall enough to fill the chip.
bool rows_form(int64_t N, int p, int q, int sym) {
  const int nt = (int)ceil_div(std::max(p, q), 16);
  return N >= 4096 && (sym ? nt <= 7 : nt <= 5);
}

// workgroups of the row-streaming form: about eight 4-row steps per
// wavefront, at most 512 workgroups (two per CU)
int64_t rows_wgs(int64_t N) {
  return std::max<int64_t>(1, std::min<int64_t>(512, ceil_div(N, 4 * 4 * 8)));
}

// C (FP64) = the sum of `splits` partials of p x q
template <class AT>
void reduce_splits(int p, int q, int64_t splits, const AT* part, double* C, int64_t ldc,
                   int sym, hipStream_t st, const int* gate) {
  const int64_t tot = (int64_t)p * q;
  int lanes = 1;   // threads per output: about 32 splits each, at most 16
  while (lanes < 16 && lanes * 32 < splits) lanes <<= 1;
  const int64_t per_block = 256 / lanes;       // outputs per workgroup
  hipLaunchKernelGGL((gram_reduce_kernel<AT>), dim3((unsigned)ceil_div(tot, per_block)),
                     dim3(256), 0, st, p, q, (int)splits, lanes, part, C, ldc, sym, MT,
                     gate);
  MC_CHECK_LAUNCH();
}
}  // namespace

int64_t gram_splits(int64_t N, int p, int q, int sym) {
  return std::max({fused_splits(N, p, q, sym), gram_mfma_splits(N, p, q, sym),
                   rows_form(N, p, q, sym) ? rows_wgs(N) : int64_t(0)});
}


template <class IT, class AT>
void launch_gram(int64_t N, int p, int q, const IT* A, int64_t lda, const IT* B,
                 int64_t ldb, double* C, int64_t ldc, int sym, AT* part,
                 int64_t part_cap, hipStream_t st, const int* gate) {
  if (p <= 0 || q <= 0) return;
  static_assert(std::is_same<IT, AT>::value, "the matrix-core Gram accumulates in its input type");
  const int nt = (int)ceil_div(std::max(p, q), 16);
  if (rows_form(N, p, q, sym)) {
    // one output block: the row-streaming form, one partial per workgroup
    int64_t nwg = rows_wgs(N);
    while (nwg > 1 && nwg * p * q > part_cap) --nwg;
    MC_REQUIRE(nwg * p * q <= part_cap, kEINVAL, "gram partial buffer too small");
#define MC_GRAM_ROWS(NT, S)                                                          \
  hipLaunchKernelGGL((gram_rows_kernel<AT, NT, S>), dim3((unsigned)nwg), dim3(256), 0, st, \
                     N, p, q, A, lda, B, ldb, part, gate)
    if (sym) {
      switch (nt) {
        case 1: MC_GRAM_ROWS(1, true); break;
        case 2: MC_GRAM_ROWS(2, true); break;
        case 3: MC_GRAM_ROWS(3, true); break;
        case 4: MC_GRAM_ROWS(4, true); break;
        case 5: MC_GRAM_ROWS(5, true); break;
        case 6: MC_GRAM_ROWS(6, true); break;
        default: MC_GRAM_ROWS(7, true); break;
      }
    } else {
      switch (nt) {
        case 1: MC_GRAM_ROWS(1, false); break;
        case 2: MC_GRAM_ROWS(2, false); break;
        case 3: MC_GRAM_ROWS(3, false); break;
        case 4: MC_GRAM_ROWS(4, false); break;
        default: MC_GRAM_ROWS(5, false); break;
      }
    }
#undef MC_GRAM_ROWS
    MC_CHECK_LAUNCH();
    reduce_splits<AT>(p, q, nwg, part, C, ldc, sym, st, gate);
    return;
  }
  int64_t splits = gram_mfma_splits(N, p, q, sym);
  while (splits > 1 && splits * p * q > part_cap) --splits;
  MC_REQUIRE(splits * p * q <= part_cap, kEINVAL, "gram partial buffer too small");
  const int64_t rps = round_up(ceil_div(std::max<int64_t>(N, 1), splits), MK);
  splits = std::max<int64_t>(1, ceil_div(std::max<int64_t>(N, 1), rps));
  dim3 grid((unsigned)ceil_div(p, MB), (unsigned)ceil_div(q, MB), (unsigned)splits);
  // tiles per wavefront of the fullest block: the first one (a diagonal
  // block of a symmetric product holds only its upper tiles)
  const int nti0 = (int)std::min<int64_t>(MB / 16, ceil_div(p, 16));
  const int ntj0 = (int)std::min<int64_t>(MB / 16, ceil_div(q, 16));
  const int most = (sym && p <= MB) ? nti0 * (nti0 + 1) / 2 : nti0 * ntj0;
  const int per_wave = (int)ceil_div(most, 4);
#define MC_GRAM_MFMA(TW)                                                        \
  hipLaunchKernelGGL((gram_mfma_kernel<AT, TW>), grid, dim3(256), 0, st, N, p, q, A, \
                     lda, B, ldb, part, rps, sym, gate)
  if (per_wave <= 1)
    MC_GRAM_MFMA(1);
  else if (per_wave <= 2)
    MC_GRAM_MFMA(2);
  else if (per_wave <= 4)
    MC_GRAM_MFMA(4);
  else if (per_wave <= 8)
    MC_GRAM_MFMA(8);
  else
    MC_GRAM_MFMA(16);
#undef MC_GRAM_MFMA
  MC_CHECK_LAUNCH();
  reduce_splits<AT>(p, q, splits, part, C, ldc, sym, st, gate);
}
template void launch_gram<double, double>(int64_t, int, int, const double*,
                                          int64_t, const double*, int64_t,
                                          double*, int64_t, int, double*,
                                          int64_t, hipStream_t, const int*);
template void launch_gram<float, float>(int64_t, int, int, const float*,
                                        int64_t, const float*, int64_t, double*,
                                        int64_t, int, float*, int64_t,
                                        hipStream_t, const int*);

bool gram_bf16_fits(int64_t N, int p, int q, int sym) { return rows_form(N, p, q, sym); }

void launch_gram_bf16(int64_t N, int p, int q, const float* A, int64_t lda, const float* B,
                      int64_t ldb, double* C, int64_t ldc, int sym, float* part,
                      int64_t part_cap, hipStream_t st) {
  MC_REQUIRE(p > 0 && q > 0 && rows_form(N, p, q, sym), kEINVAL,
             "BF16 Gram: shape outside the row-streaming form");
  const int nt = (int)ceil_div(std::max(p, q), 16);
  int64_t nwg = rows_wgs(N);
  while (nwg > 1 && nwg * p * q > part_cap) --nwg;
  MC_REQUIRE(nwg * p * q <= part_cap, kEINVAL, "gram partial buffer too small");
#define MC_GRAM_BF(NT, S)                                                             \
  hipLaunchKernelGGL((gram_rows_bf16_kernel<NT, S>), dim3((unsigned)nwg), dim3(256), 0, st, \
                     N, p, q, A, lda, B, ldb, part)
  if (sym) {
    switch (nt) {
      case 1: MC_GRAM_BF(1, true); break;
      case 2: MC_GRAM_BF(2, true); break;
      case 3: MC_GRAM_BF(3, true); break;
      case 4: MC_GRAM_BF(4, true); break;
      case 5: MC_GRAM_BF(5, true); break;
      case 6: MC_GRAM_BF(6, true); break;
      default: MC_GRAM_BF(7, true); break;
    }
  } else {
    switch (nt) {
      case 1: MC_GRAM_BF(1, false); break;
      case 2: MC_GRAM_BF(2, false); break;
      case 3: MC_GRAM_BF(3, false); break;
      case 4: MC_GRAM_BF(4, false); break;
      default: MC_GRAM_BF(5, false); break;
    }
  }
#undef MC_GRAM_BF
  MC_CHECK_LAUNCH();
  reduce_splits<float>(p, q, nwg, part, C, ldc, sym, st, nullptr);
}

// The one-workgroup form for short blocks with few tiles; false when the
// shape is outside it (the caller then takes the split form).
template <class T>
bool launch_gram_small(int64_t N, int p, int q, const T* A, int64_t lda, const T* B,
                       int64_t ldb, double* C, int64_t ldc, int sym, double* Rinv,
                       int64_t ldr, int64_t nrows, int* shifted, int* flag, hipStream_t st,
                       const int* gate) {
  const bool chol = Rinv != nullptr;
  const int tp = (int)ceil_div(p, 16), tq = (int)ceil_div(q, 16);
  if (N > kSmallRows || tp > 4 || tq > 4) return false;
  if ((sym || chol) && (p != q || A != B || lda != ldb)) return false;
  const bool sq = sym || chol;
  const int nt = sq ? tp * (tp + 1) / 2 : tp * tq;
  if (nt > kSmallTiles || (chol && p > 64)) return false;
  GramTail t;
  t.mode = chol ? 2 : 1;
  t.C = C;
  t.ldc = ldc;
  t.Rinv = Rinv;
  t.ldr = ldr;
  t.nrows = nrows;
  t.shifted = shifted;
  t.flag = flag;
  // the reduction tree (8 wavefronts' tiles) and, after it, G and the
  // Cholesky's 3 p doubles
  const size_t red = (size_t)(kSmallWaves / 2) * nt * 256;
  const size_t lds = sizeof(double) * std::max(red, (size_t)p * q + 3 * p);
  static const bool attr = [] {
    const int bytes = (int)sizeof(double) * (kSmallWaves / 2) * kSmallTiles * 256;
#define MC_SMALL_ATTR(T_, S_, P_, Q_)                                                   \
  if (hipFuncSetAttribute((const void*)gram_small_kernel<T_, S_, P_, Q_>,                \
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) \
    (void)hipGetLastError();
#define MC_SMALL_ALL(T_)                                                                \
  MC_SMALL_ATTR(T_, true, 1, 1) MC_SMALL_ATTR(T_, true, 2, 2) MC_SMALL_ATTR(T_, true, 3, 3) \
  MC_SMALL_ATTR(T_, false, 1, 1) MC_SMALL_ATTR(T_, false, 1, 2) MC_SMALL_ATTR(T_, false, 1, 3) \
  MC_SMALL_ATTR(T_, false, 1, 4) MC_SMALL_ATTR(T_, false, 2, 1) MC_SMALL_ATTR(T_, false, 2, 2) \
  MC_SMALL_ATTR(T_, false, 2, 3) MC_SMALL_ATTR(T_, false, 3, 1) MC_SMALL_ATTR(T_, false, 3, 2) \
  MC_SMALL_ATTR(T_, false, 4, 1)
    MC_SMALL_ALL(double)
    MC_SMALL_ALL(float)
#undef MC_SMALL_ALL
#undef MC_SMALL_ATTR
    return true;
  }();
  (void)attr;
#define MC_SMALL(S_, P_, Q_)                                                              \
  hipLaunchKernelGGL((gram_small_kernel<T, S_, P_, Q_>), dim3(1), dim3(kSmallThreads), lds, \
                     st, N, p, q, A, lda, B, ldb, gate, t)
  if (sq) {
    if (tp == 1) MC_SMALL(true, 1, 1);
    else if (tp == 2) MC_SMALL(true, 2, 2);
    else MC_SMALL(true, 3, 3);
  } else {
    switch (tp * 8 + tq) {
      case 9: MC_SMALL(false, 1, 1); break;
      case 10: MC_SMALL(false, 1, 2); break;
      case 11: MC_SMALL(false, 1, 3); break;
      case 12: MC_SMALL(false, 1, 4); break;
      case 17: MC_SMALL(false, 2, 1); break;
      case 18: MC_SMALL(false, 2, 2); break;
      case 19: MC_SMALL(false, 2, 3); break;
      case 25: MC_SMALL(false, 3, 1); break;
      case 26: MC_SMALL(false, 3, 2); break;
      default: MC_SMALL(false, 4, 1); break;
    }
  }
#undef MC_SMALL
  MC_CHECK_LAUNCH();
  return true;
}

// Gram (or cross-Gram) with its completion in the same launch: C = A^T B
// (mode 1) or, with A = B, also Rinv = R^{-1} of C = R^T R (mode 2).
template <class IT, class AT>
void launch_gram_fused(int64_t N, int p, int q, const IT* A, int64_t lda, const IT* B,
                       int64_t ldb, double* C, int64_t ldc, int sym, AT* part,
                       int64_t part_cap, int* counter, double* Rinv, int64_t ldr,
                       int64_t nrows, int* shifted, int* flag, hipStream_t st,
                       const int* gate) {
  if (p <= 0 || q <= 0) return;
  const bool chol = Rinv != nullptr;
  MC_REQUIRE(!chol || (p == q && p <= kCholLdsMax), kEINVAL, "fused Cholesky size");
  if (launch_gram_small<IT>(N, p, q, A, lda, B, ldb, C, ldc, sym, Rinv, ldr, nrows, shifted,
                            flag, st, gate))
    return;
  // at most 64 row splits: one workgroup sums the partials
  int64_t splits = std::min<int64_t>(64, fused_splits(N, p, q, sym));
  while (splits > 1 && splits * p * q > part_cap) --splits;
  MC_REQUIRE(splits * p * q <= part_cap, kEINVAL, "gram partial buffer too small");
  const int64_t rps = round_up(ceil_div(std::max<int64_t>(N, 1), splits), GT);
  splits = std::max<int64_t>(1, ceil_div(std::max<int64_t>(N, 1), rps));
  const int64_t tp = ceil_div(p, GT), tq = ceil_div(q, GT);
  int64_t tiles = 0;
  for (int64_t a = 0; a < tp; ++a)
    for (int64_t c = 0; c < tq; ++c)
      if (!sym || c >= a) ++tiles;
  GramTail t;
  t.mode = chol ? 2 : 1;
  t.counter = counter;
  t.expected = (int)(tiles * splits);
  t.nsplit = (int)splits;
  t.C = C;
  t.ldc = ldc;
  t.Rinv = Rinv;
  t.ldr = ldr;
  t.nrows = nrows;
  t.shifted = shifted;
  t.flag = flag;
  static const bool attr = [] {
    for (const void* f : {(const void*)gram_kernel<double, double>,
                          (const void*)gram_kernel<float, float>})
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kCholLdsDoubles * (int)sizeof(double)) !=
          hipSuccess)
        (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  const size_t lds = chol ? ((size_t)p * p + 3 * p) * sizeof(double) : 0;
  dim3 grid((unsigned)tp, (unsigned)tq, (unsigned)splits);
  hipLaunchKernelGGL((gram_kernel<IT, AT>), grid, dim3(GramTailThreads), lds, st, N, p, q, A, lda, B,
                     ldb, part, rps, sym, gate, t);
  MC_CHECK_LAUNCH();
}
template void launch_gram_fused<double, double>(int64_t, int, int, const double*, int64_t,
                                                const double*, int64_t, double*, int64_t,
                                                int, double*, int64_t, int*, double*,
                                                int64_t, int64_t, int*, int*, hipStream_t,
                                                const int*);
template void launch_gram_fused<float, float>(int64_t, int, int, const float*, int64_t,
                                              const float*, int64_t, double*, int64_t, int,
                                              float*, int64_t, int*, double*, int64_t,
                                              int64_t, int*, int*, hipStream_t, const int*);

template <class XT, class OT>
void launch_panel_gemm(int64_t N, int p, int q, const XT* X, int64_t ldx,
                       const double* W, int64_t ldw, double alpha,
                       const double* colscale, double beta, const OT* C0,
                       int64_t ldc0, OT* C, int64_t ldc, hipStream_t st,
                       const int* gate) {
  if (N <= 0 || q <= 0) return;
  // 16-column instruction tiles per workgroup: all of q up to 128
  const int nt = (int)std::min<int64_t>(8, ceil_div(q, 16));
  dim3 grid((unsigned)ceil_div(N, QR), (unsigned)ceil_div(q, 16 * nt));
#define MC_PANEL(NT)                                                                   \
  hipLaunchKernelGGL((panel_mfma_kernel<XT, OT, NT, (NT <= 3 ? 16 : 32)>), grid, dim3(256), \
                     0, st, N, p, q, X, ldx, W, ldw, alpha, colscale, beta, C0, ldc0, C, ldc, \
                     gate)
  switch (nt) {
    case 1: MC_PANEL(1); break;
    case 2: MC_PANEL(2); break;
    case 3: MC_PANEL(3); break;
    case 4: MC_PANEL(4); break;
    case 5: MC_PANEL(5); break;
    case 6: MC_PANEL(6); break;
    case 7: MC_PANEL(7); break;
    default: MC_PANEL(8); break;
  }
#undef MC_PANEL
  MC_CHECK_LAUNCH();
}
template void launch_panel_gemm<double, double>(int64_t, int, int,
                                                const double*, int64_t,
                                                const double*, int64_t, double,
                                                const double*, double,
                                                const double*, int64_t, double*,
                                                int64_t, hipStream_t, const int*);
template void launch_panel_gemm<float, float>(int64_t, int, int, const float*,
                                              int64_t, const double*, int64_t,
                                              double, const double*, double,
                                              const float*, int64_t, float*,
                                              int64_t, hipStream_t, const int*);
template void launch_panel_gemm<float, double>(int64_t, int, int, const float*,
                                               int64_t, const double*, int64_t,
                                               double, const double*, double,
                                               const double*, int64_t, double*,
                                               int64_t, hipStream_t, const int*);

void launch_chol_inv(int b, const double* G, int64_t ldg, double* Rinv,
                     int64_t ldr, double* work, int64_t nrows, int* shifted,
                     hipStream_t st, int* flag, const int* gate) {
  static const bool attr = [] {
    // the elimination array for b up to kCholLdsMax exceeds the default 64 KB
    if (hipFuncSetAttribute((const void*)chol_inv_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            kCholLdsDoubles * (int)sizeof(double)) !=
        hipSuccess)
      (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  const size_t lds = (b <= kCholLdsMax) ? ((size_t)b * b + 2 * b) * sizeof(double) : 0;
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(1024), lds, st, b, G, ldg,
                     Rinv, ldr, work, nrows, shifted, flag, gate);
  MC_CHECK_LAUNCH();
}

void launch_set_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, p, v);
  MC_CHECK_LAUNCH();
}

template <class T>
void launch_copy_gated(int64_t rows, int cols, const T* src, int64_t lds_, T* dst,
                       int64_t ldd, const int* gate, hipStream_t st) {
  const int64_t tot = rows * cols;
  if (tot <= 0) return;
  hipLaunchKernelGGL(copy_gated_kernel<T>, dim3((unsigned)ceil_div(tot, 256)),
                     dim3(256), 0, st, rows, cols, src, lds_, dst, ldd, gate);
  MC_CHECK_LAUNCH();
}
template void launch_copy_gated<double>(int64_t, int, const double*, int64_t,
                                        double*, int64_t, const int*, hipStream_t);
template void launch_copy_gated<float>(int64_t, int, const float*, int64_t, float*,
                                       int64_t, const int*, hipStream_t);

template <class S, class D>
void launch_cast_panel(int64_t rows, int cols, const S* src, int64_t lds_, D* dst,
                       int64_t ldd, hipStream_t st) {
  const int64_t tot = rows * (int64_t)cols;
  if (tot <= 0) return;
  hipLaunchKernelGGL((cast_panel_kernel<S, D>), dim3((unsigned)ceil_div(tot, 256)),
                     dim3(256), 0, st, rows, cols, src, lds_, dst, ldd);
  MC_CHECK_LAUNCH();
}
template void launch_cast_panel<float, bf16_t>(int64_t, int, const float*, int64_t,
                                               bf16_t*, int64_t, hipStream_t);

void launch_recip(int k, const double* S, double* out, hipStream_t st, const int* count,
                  double* count_out, double* host) {
  hipLaunchKernelGGL(recip_kernel, dim3((unsigned)ceil_div(k, 128)), dim3(128), 0,
                     st, k, S, out, count, count_out, host);
  MC_CHECK_LAUNCH();
}

int ritz_blocks(int64_t m) { return (int)std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(m, 64))); }

template <class T>
void launch_ritz(int64_t m, int k, const T* R, int64_t ldr, const T* U,
                 int64_t ldu, const double* S, double* partial, double* out,
                 hipStream_t st) {
  const int nblk = ritz_blocks(m);
  const int64_t rpb = ceil_div(m, nblk);
  hipLaunchKernelGGL(ritz_partial_kernel<T>, dim3(nblk), dim3(256), 0, st, m, k, R,
                     ldr, U, ldu, S, rpb, partial);
  MC_CHECK_LAUNCH();
  hipLaunchKernelGGL(ritz_reduce_kernel, dim3((unsigned)ceil_div(k, 128)),
                     dim3(128), 0, st, nblk, k, partial, S, out);
  MC_CHECK_LAUNCH();
}
template void launch_ritz<double>(int64_t, int, const double*, int64_t,
                                  const double*, int64_t, const double*, double*,
                                  double*, hipStream_t);
template void launch_ritz<float>(int64_t, int, const float*, int64_t, const float*,
                                 int64_t, const double*, double*, double*,
                                 hipStream_t);

}  // namespace mcsvt
