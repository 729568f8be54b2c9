// Cholesky factor inverse of a small SPD matrix with the matrix held in
// registers, for one workgroup (device code shared by the orthonormalisation
// and the eigensolver).
//
// G (b x b) = L D L^T is reduced by Gaussian elimination without pivoting on
// [G | I]: after step j, rows i > j hold the Schur complement on and above
// the diagonal and, below it, the row operations applied so far to I (the
// rows of L^{-1}; unit diagonal implied).  With R = D^{1/2} L^T (G = R^T R),
// R^{-1} = L^{-T} D^{-1/2}, i.e. Rinv[a][c] = Linv[c][a] / sqrt(d_c) for
// a <= c, so no triangular inversion follows the factorisation.
//
// Thread (ty, tx) of ny = blockDim.x / 32 rows of 32 lanes owns the elements
// (ty + ny n, tx + 32 m), n < NR, m < NC, in registers (needs
// NR >= ceil(b / ny), NC >= ceil(b / 32)).  In step j the owners of row j
// have published it to LDS; every thread reads its multipliers and the
// pivot row from there, updates its elements, and the owners of row j + 1
// publish that row into the other half of the buffer: one barrier per
// column.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mcsvt {

// 1/x from the hardware estimate and two Newton steps (about 1 ulp), for the
// serial chains of the factorisations; x is a positive normal number there
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  return r * (2.0 - x * r);
}

// Rinv (row-major, ldr; zeros below the diagonal) = R^{-1} for G = R^T R.
// G is read on and above its diagonal.  lds: 3 b doubles (the published
// rows and the diagonal of G).
// clamp = false: a pivot that is not positive or below 1e-13 of its
//   original diagonal restarts the factorisation of G + shift I (shift
//   11 (nrows b + b (b + 1)) u tr(G), then x100), counted in *shifted and
//   flagged in *flag (both optional).
// clamp = true: pivots are clamped below at 1e-28, no restart.
template <int NR, int NC>
__device__ __forceinline__ void chol_inv_regs(int b, const double* __restrict__ G,
                                              int64_t ldg, double* __restrict__ Rinv,
                                              int64_t ldr, double* lds, int64_t nrows,
                                              int* __restrict__ shifted,
                                              int* __restrict__ flag, bool clamp) {
  const int tid = threadIdx.x;
  const int tx = tid & 31, ty = tid >> 5, ny = (int)(blockDim.x >> 5);
  double* pub = lds;            // 2 b: row j in half (j & 1)
  double* gd = lds + 2 * b;     // b: diagonal of G
  for (int i = tid; i < b; i += blockDim.x) gd[i] = G[(int64_t)i * ldg + i];
  int ri[NR], ci[NC];
#pragma unroll
  for (int n = 0; n < NR; ++n) ri[n] = ty + ny * n;
#pragma unroll
  for (int m = 0; m < NC; ++m) ci[m] = tx + 32 * m;
  const double u = 1.1102230246251565e-16;
  double shift = 0.0;
  double a[NR][NC];
  double piv[NR];
#pragma unroll
  for (int n = 0; n < NR; ++n) piv[n] = 1.0;
  __syncthreads();
  const int attempts = clamp ? 1 : 6;
  for (int attempt = 0; attempt < attempts; ++attempt) {
    // the upper triangle of G (+ shift on the diagonal); loads from clamped
    // addresses, zeroed by a factor (no branch around them)
#pragma unroll
    for (int n = 0; n < NR; ++n)
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const int i = ri[n], c = ci[m];
        const bool in = i < b && c < b && i <= c;
        const double g = G[(int64_t)min(i, b - 1) * ldg + min(c, b - 1)];
        a[n][m] = g * (in ? 1.0 : 0.0) + ((in && i == c) ? shift : 0.0);
      }
    if (ty == 0)                                     // row 0: n = 0
#pragma unroll
      for (int m = 0; m < NC; ++m)
        if (ci[m] < b) pub[ci[m]] = a[0][m];
    __syncthreads();
    bool failed = false;
    for (int j = 0; j < b; ++j) {
      const double* row = pub + (j & 1) * b;
      double d = row[j];
      double rj[NC], li[NR];
#pragma unroll
      for (int m = 0; m < NC; ++m) rj[m] = row[min(ci[m], b - 1)];
#pragma unroll
      for (int n = 0; n < NR; ++n) li[n] = row[min(ri[n], b - 1)];
      if (clamp) {
        d = fmax(d, 1e-28);
      } else if (!(d > 1e-13 * (gd[j] + shift)) || !(d > 1e-300)) {
        // kappa(H) of order 1e6 or worse: Cholesky QR would lose all
        // orthogonality (the same decision in every thread)
        failed = true;
        break;
      }
      const double rd = rcp_nr(d);
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        const int i = ri[n];
        if (i == j) piv[n] = d;
        if (i > j && i < b) {
          const double l = li[n] * rd;               // multiplier of row i
#pragma unroll
          for (int m = 0; m < NC; ++m) {
            const int c = ci[m];
            if (c >= i || c < j)
              a[n][m] -= l * rj[m];
            else if (c == j)
              a[n][m] = -l;                          // L^{-1}[j][j] = 1
          }
        }
      }
      const int jn = j + 1;
      if (jn < b && ty == jn % ny) {
        const int nn = jn / ny;
        double* dst = pub + (jn & 1) * b;
#pragma unroll
        for (int n = 0; n < NR; ++n)
          if (n == nn)
#pragma unroll
            for (int m = 0; m < NC; ++m)
              if (ci[m] < b) dst[ci[m]] = a[n][m];
      }
      __syncthreads();
    }
    if (!failed) break;
    // shifted Cholesky QR: s = 11 (N b + b (b + 1)) u ||X||^2, ||X||^2 <= tr G
    double tr = 0.0;
    for (int i = 0; i < b; ++i) tr += gd[i];
    shift = (shift == 0.0)
                ? 11.0 * ((double)nrows * b + (double)b * (b + 1)) * u * fmax(tr, 1e-300)
                : shift * 100.0;
    if (tid == 0 && shifted) atomicAdd(shifted, 1);
    if (tid == 0 && flag) *flag = 1;
    __syncthreads();                                 // pub is rewritten next
  }
  // element (i, c) of the owner goes to Rinv[c][i]
#pragma unroll
  for (int n = 0; n < NR; ++n) {
    const int i = ri[n];
    if (i < b) {
      const double s = 1.0 / sqrt(piv[n]);
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const int c = ci[m];
        if (c < b) {
          const double v = c < i ? a[n][m] * s : (c == i ? s : 0.0);
          Rinv[(int64_t)c * ldr + i] = v;
        }
      }
    }
  }
}

}  // namespace mcsvt
