// Top-k eigenpairs of the symmetric Gram matrix of eigSVD (Alg. 3, and the
// top-k selection of Alg. 5) inside one workgroup, for L small enough that the whole
// matrix sits in LDS.
//
//   1. Householder reduction to tridiagonal form, T = Q^T G Q.  Step j
//      annihilates column j below the subdiagonal with H_j = I - beta v v^T
//      (v_{j+1} = 1), and applies it as the symmetric rank-2 update
//      A <- A - v w^T - w v^T, p = beta A v, w = p - (beta/2)(p^T v) v.
//      Two barriers per step; the reflector's data stays in row j of A.
//   2. The k largest eigenvalues of T by multisection on Sturm counts: one
//      global pass over the Gershgorin interval, then groups of lanes refine
//      one eigenvalue each until the bracket reaches round-off.
//   3. Eigenvectors of T by two steps of inverse iteration (partial-pivoting
//      LU of T - lambda I, random then previous right-hand side), with the
//      k vectors made orthonormal by Cholesky QR after each step (twice after
//      the last).  Nearly equal eigenvalues thus get an orthonormal basis of
//      their joint invariant subspace.  Rayleigh quotients on T give the
//      returned eigenvalues.
//   4. Back-transformation W = H_0 H_1 ... H_{L-3} Z, 16 lanes per vector
//      with the vector held in registers; the reflectors are stored as full
//      rows v_j (zero before j + 1, one at j + 1).
#include "chol_regs.hpp"
#include "kernels.hpp"

#include <cfloat>

namespace mcsvt {

namespace {

constexpr int kTT = 512;              // threads of the workgroup
constexpr int kTWaves = kTT / 64;
constexpr int kVecLanes = 16;         // lanes per vector in the back-transformation
constexpr int kVecRegs = 12;          // L <= kVecLanes * kVecRegs
constexpr double kU = DBL_EPSILON / 2;

// Cross-lane sums through DPP moves (VALU, no LDS round trip).  Every lane of
// the group ends with bit-identical totals: each stage adds a value and its
// partner's, in either order, and IEEE addition commutes.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL,
                                             0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL,
                                             0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int kQuadXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

// sum over aligned groups of S lanes, S in {1, 2, 4, 8, 16}
__device__ __forceinline__ double group_sum(double v, int S) {
  if (S >= 2) v += dpp<kQuadXor1>(v);
  if (S >= 4) v += dpp<kQuadXor2>(v);
  if (S >= 8) v += dpp<kRowHalfMirror>(v);
  if (S >= 16) v += dpp<kRowMirror>(v);
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// sum over the wavefront, the same value in every lane
__device__ __forceinline__ double wsum(double v) {
  v = group_sum(v, 16);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// 1/x from the hardware estimate and two Newton steps (about 1 ulp); x is a
// normal number here
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots);
// d and e2 are loaded four rows at a time, ahead of the recurrence
__device__ __forceinline__ int sturm(int L, const double* __restrict__ d,
                                     const double* __restrict__ e2, double x,
                                     double pivmin) {
  double q = d[0] - x;
  int c = q < 0.0;
  int i = 1;
  for (; i + 4 <= L; i += 4) {
    const double d0 = d[i], d1 = d[i + 1], d2 = d[i + 2], d3 = d[i + 3];
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d0 - x) - f0 * rcp(q);
    c += q < 0.0;
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d1 - x) - f1 * rcp(q);
    c += q < 0.0;
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d2 - x) - f2 * rcp(q);
    c += q < 0.0;
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d3 - x) - f3 * rcp(q);
    c += q < 0.0;
  }
  for (; i < L; ++i) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d[i] - x) - e2[i - 1] * rcp(q);
    c += q < 0.0;
  }
  return c;
}

struct TriSmem {
  double *A, *d, *e, *e2, *hb, *hr, *P, *lam, *red, *red2, *xch;
  int* cnt;
};

__device__ TriSmem tri_layout_r(double* sm, int L, size_t region) {
  TriSmem s;
  s.A = sm;
  double* q = sm + region;
  s.d = q;    q += L;
  s.e = q;    q += L;
  s.e2 = q;   q += L;
  s.hb = q;   q += L;
  s.hr = q;   q += L;
  s.P = q;    q += L;
  s.lam = q;  q += L;
  s.red = q;  q += kTWaves;
  s.red2 = q; q += kTWaves;
  s.xch = q;  q += 4 * kTWaves;
  s.cnt = (int*)q;
  return s;
}

// doubles of the matrix region: A (L x L), later Z (L x k), C (k x k) and,
// for a batch of nb inverse iterations, the U factors (3 L nb), multipliers
// (L nb) and row exchanges (L nb ints, in L nb doubles)
__host__ __device__ inline size_t tri_region(int L, int k, int nb) {
  const size_t a = (size_t)L * L, b = (size_t)L * k + (size_t)k * k + 5 * (size_t)L * nb;
  return a > b ? a : b;
}

__device__ TriSmem tri_layout(double* sm, int L, int k, int nb) {
  return tri_layout_r(sm, L, tri_region(L, k, nb));
}

// Cholesky QR of the L x k block Z (row-major, ld k) in LDS: C = Z^T Z,
// C = R^T R, Z <- Z R^{-1}.  The Cholesky factorisation runs in the first
// wavefront alone (LDS operations of one wavefront complete in order, so it
// needs no barriers); a pivot below 1e-28 (columns enter with unit norm) is
// clamped so a degenerate block still gives finite values.
__device__ void cholqr_lds(int L, int k, double* Z, double* C) {
  const int tid = threadIdx.x;
  // Gram, two output columns per thread
  const int kh = (k + 1) / 2;
  for (int t = tid; t < k * kh; t += kTT) {
    const int a = t / kh, b = 2 * (t % kh);
    if (a > b + 1) continue;
    const bool two = b + 1 < k;
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < L; ++i) {
      const double za = Z[i * k + a];
      s0 += za * Z[i * k + b];
      if (two) s1 += za * Z[i * k + b + 1];
    }
    if (a <= b) C[a * k + b] = s0;
    if (two) C[a * k + b + 1] = s1;
  }
  __syncthreads();
  if (tid < 64) {
    // right-looking on the upper triangle; lanes share the trailing block
    for (int c = 0; c < k; ++c) {
      const double rp = rcp(fmax(C[c * k + c], 1e-28));
      const int n = k - c - 1;
      for (int t = tid; t < n * n; t += 64) {
        const int a = c + 1 + t / n, b = c + 1 + t % n;
        if (a > b) continue;
        C[a * k + b] -= C[c * k + a] * C[c * k + b] * rp;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  // R^T below the diagonal (R_ab = C_ab / sqrt(C_aa)); 1 / R_aa on it
  for (int t = tid; t < k * k; t += kTT) {
    const int a = t / k, b = t % k;
    if (a > b) continue;
    const double ir = rcp(sqrt(fmax(C[a * k + a], 1e-28)));
    if (a < b) C[b * k + a] = C[a * k + b] * ir;
  }
  __syncthreads();
  for (int t = tid; t < k; t += kTT) C[t * k + t] = rcp(sqrt(fmax(C[t * k + t], 1e-28)));
  __syncthreads();
  // Z row i <- Z row i R^{-1}
  for (int i = tid; i < L; i += kTT) {
    double* z = Z + (size_t)i * k;
    for (int c = 0; c < k; ++c) {
      double s = z[c];
      for (int l = 0; l < c; ++l) s -= z[l] * C[c * k + l];
      z[c] = s * C[c * k + c];
    }
  }
  __syncthreads();
}

// One Newton-Schulz step towards the orthogonal polar factor of a block with
// nearly orthonormal columns: Z <- Z (3 I - Z^T Z) / 2.  With Z^T Z = I + E
// the new deviation is O(|E|^2), so after Cholesky QR (|E| ~ 1e-13) one step
// leaves rounding only.  The products run over (row, column) pairs in
// parallel; the new rows are kept in registers across a barrier.
__device__ void polar_step_lds(int L, int k, double* __restrict__ Z,
                               double* __restrict__ C) {
  const int tid = threadIdx.x;
  for (int t = tid; t < k * k; t += kTT) {
    const int a = t / k, b = t % k;
    if (a > b) continue;
    double s = 0.0;
    for (int i = 0; i < L; ++i) s += Z[i * k + a] * Z[i * k + b];
    const double m = (a == b ? 1.5 : 0.0) - 0.5 * s;
    C[a * k + b] = m;
    C[b * k + a] = m;
  }
  __syncthreads();
  // whole rows per pass, so no row is overwritten while it is still read
  constexpr int kPer = 8;                // (row, column) pairs per thread and pass
  const int rows_per = max(1, kTT * kPer / k);
  for (int r0 = 0; r0 < L; r0 += rows_per) {
    const int t0 = r0 * k, t1 = min(L, r0 + rows_per) * k;
    double nz[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kTT + tid;
      nz[u] = 0.0;
      if (t < t1) {
        const int i = t / k, c = t % k;
        double s = 0.0;
        for (int l = 0; l < k; ++l) s += Z[i * k + l] * C[l * k + c];
        nz[u] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = t0 + u * kTT + tid;
      if (t < t1) Z[t] = nz[u];
    }
    __syncthreads();
  }
}

// Inverse iteration for eigenvalue lam on column j of Z (row-major, k
// columns): solves (T - lam I) x = y for the right-hand side y held in the
// column, in place.  The pivoted LU of T - lam I is formed on the first solve
// (FACTOR): row i's U entries go to Uf + i ldu (u0 is replaced by the
// reciprocal of the clamped pivot once the back substitution has used it),
// its multiplier to lf[i ldl] and its row exchange to sw[i ldl]; a later
// solve (!FACTOR) reuses them.  One thread runs it; the operands of kIC
// consecutive rows are read into registers ahead of each stretch of the
// recurrences, and the elimination selects instead of branching.  Returns
// max |x_i| (after any rescaling of the column by 2^-500, which keeps the
// solution finite).
constexpr int kIC = 8;
template <bool FACTOR>
__device__ __forceinline__ double invit_solve(int L, int k, int j, const double* __restrict__ d,
                                              const double* __restrict__ e, double lam,
                                              double ptiny, double* __restrict__ Z,
                                              double* __restrict__ Uf, int ldu,
                                              double* __restrict__ lf, int* __restrict__ sw,
                                              int ldl) {
  double r0 = d[0] - lam;
  double r1 = L > 1 ? e[0] : 0.0;
  double ycur = Z[j];
  // elimination step i (rows i, i + 1) on the factor and the right-hand side
  auto elim = [&](int i, double c, double a1, double b1, double ynext, double lv, int sv) {
    bool swap;
    double l;
    if (FACTOR) {
      // rows i and i + 1 exchange when the subdiagonal entry is larger
      swap = fabs(r0) < fabs(c);
      const double num = swap ? r0 : c;
      const double den = swap ? c : r0;
      l = den != 0.0 ? num * rcp(den) : 0.0;
      double* uf = Uf + (size_t)i * ldu;
      uf[0] = den;
      uf[1] = swap ? a1 : r1;
      uf[2] = swap ? b1 : 0.0;
      lf[(size_t)i * ldl] = l;
      sw[(size_t)i * ldl] = swap;
      const double ra = swap ? r1 : a1;
      const double rb = swap ? a1 : r1;
      r0 = ra - l * rb;
      r1 = swap ? -l * b1 : b1;
    } else {
      swap = sv != 0;
      l = lv;
    }
    const double zi = swap ? ynext : ycur;
    const double ya = swap ? ycur : ynext;
    Z[i * k + j] = zi;
    ycur = ya - l * zi;
  };
  const int nel = L - 1;                       // steps i = 0 .. L - 2
  int i0 = 0;
  for (; i0 + kIC <= nel; i0 += kIC) {
    // row i + 1's operands; Z row i + 1 is read before row i is written
    double cv[kIC], av[kIC], bv[kIC], yv[kIC], lv[kIC];
    int sv[kIC];
#pragma unroll
    for (int u = 0; u < kIC; ++u) {
      const int i = i0 + u;
      yv[u] = Z[(i + 1) * k + j];
      if (FACTOR) {
        cv[u] = e[i];
        av[u] = d[i + 1] - lam;
        bv[u] = e[i + 1];                      // e[L - 1] = 0
        lv[u] = 0.0;
        sv[u] = 0;
      } else {
        cv[u] = av[u] = bv[u] = 0.0;
        lv[u] = lf[(size_t)i * ldl];
        sv[u] = sw[(size_t)i * ldl];
      }
    }
#pragma unroll
    for (int u = 0; u < kIC; ++u) elim(i0 + u, cv[u], av[u], bv[u], yv[u], lv[u], sv[u]);
  }
  for (; i0 < nel; ++i0) {
    const int i = i0;
    if (FACTOR)
      elim(i, e[i], d[i + 1] - lam, e[i + 1], Z[(i + 1) * k + j], 0.0, 0);
    else
      elim(i, 0.0, 0.0, 0.0, Z[(i + 1) * k + j], lf[(size_t)i * ldl], sw[(size_t)i * ldl]);
  }
  if (FACTOR) {
    double* uf = Uf + (size_t)(L - 1) * ldu;
    uf[0] = r0; uf[1] = 0.0; uf[2] = 0.0;
  }
  Z[(L - 1) * k + j] = ycur;
  // back substitution, rescaling if the solution grows past 2^500 (after a
  // rescaling the next stretch starts at the row below, read afresh)
  double z1 = 0.0, z2 = 0.0, zmax = 0.0;
  // row i from its U entries and right-hand side; true if it rescaled
  auto back = [&](int i, double f0, double f1, double f2, double zr) {
    double ri = f0;
    if (FACTOR) {
      const double u0 = fabs(ri) < ptiny ? (ri < 0.0 ? -ptiny : ptiny) : ri;
      ri = rcp(u0);
      Uf[(size_t)i * ldu] = ri;
    }
    double z = (zr - f1 * z1 - f2 * z2) * ri;
    const bool big = fabs(z) > 0x1p500;
    if (big) {
      const double sc = 0x1p-500;
      for (int t = 0; t < L; ++t)
        if (t != i) Z[t * k + j] *= sc;
      z *= sc; z1 *= sc; z2 *= sc; zmax *= sc;
    }
    Z[i * k + j] = z;
    zmax = fmax(zmax, fabs(z));
    z2 = z1;
    z1 = z;
    return big;
  };
  for (int i0 = L - 1; i0 >= 0;) {
    if (i0 + 1 < kIC) {
      const double* uf = Uf + (size_t)i0 * ldu;
      back(i0, uf[0], uf[1], uf[2], Z[i0 * k + j]);
      --i0;
      continue;
    }
    int next = i0 - kIC;
    double f0[kIC], f1[kIC], f2[kIC], zv[kIC];
#pragma unroll
    for (int u = 0; u < kIC; ++u) {
      const double* uf = Uf + (size_t)(i0 - u) * ldu;
      f0[u] = uf[0]; f1[u] = uf[1]; f2[u] = uf[2];
      zv[u] = Z[(i0 - u) * k + j];
    }
#pragma unroll
    for (int u = 0; u < kIC; ++u) {
      if (back(i0 - u, f0[u], f1[u], f2[u], zv[u])) {
        next = i0 - u - 1;
        break;
      }
    }
    i0 = next;
  }
  return zmax;
}

// column j of Z scaled to unit norm (after a first scaling by 1 / zmax, so
// the sum of squares cannot overflow); one thread
__device__ __forceinline__ void invit_normalize(int L, int k, int j, double zmax,
                                                double* __restrict__ Z) {
  const double inv = zmax > 0.0 ? rcp(zmax) : 1.0;
  double ss = 0.0;
#pragma unroll 8
  for (int i = 0; i < L; ++i) {
    const double z = Z[i * k + j] * inv;
    ss += z * z;
  }
  const double sc = inv * rcp(sqrt(ss));
#pragma unroll 8
  for (int i = 0; i < L; ++i) Z[i * k + j] *= sc;
}

// Two steps of inverse iteration for eigenvalue lam on column j of Z (the
// right-hand side on entry, the normalised solution on exit), in one thread;
// lf, sw: L entries each (stride ldl) for the multipliers and row exchanges.
__device__ __forceinline__ void invit_column(int L, int k, int j, const double* __restrict__ d,
                                             const double* __restrict__ e, double lam,
                                             double tnorm, double* __restrict__ Z,
                                             double* __restrict__ Uf, int ldu,
                                             double* __restrict__ lf, int* __restrict__ sw,
                                             int ldl) {
  const double ptiny = fmax(kU * tnorm, DBL_MIN / kU);
  for (int pass = 0; pass < 2; ++pass) {
    const double zmax =
        pass == 0 ? invit_solve<true>(L, k, j, d, e, lam, ptiny, Z, Uf, ldu, lf, sw, ldl)
                  : invit_solve<false>(L, k, j, d, e, lam, ptiny, Z, Uf, ldu, lf, sw, ldl);
    invit_normalize(L, k, j, zmax, Z);
  }
}

// Householder steps j = j0 .. L-3 of the reduction to tridiagonal form, on
// the trailing block held in LDS: element (r, c), r, c >= j0, of the matrix
// being reduced is Ab[(r - j0) * ldb + (c - j0)].  Writes d, e, hb, hr for
// j >= j0 and, once all steps are done, the reflectors v_j as full rows of hh
// (no global store inside the step loop, whose barriers would wait for it).
__device__ void tri_steps(int L, int j0, double* __restrict__ Ab, int ldb,
                          const TriSmem& s, double* __restrict__ hh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto el = [&](int r, int c) -> double& { return Ab[(r - j0) * ldb + (c - j0)]; };
  {
    double sq = 0.0;
    if (j0 + 2 < L)
      for (int c = j0 + 2 + tid; c < L; c += kTT) sq += el(j0, c) * el(j0, c);
    sq = wsum(sq);
    if (lane == 0) s.red2[wave] = sq;
  }
  __syncthreads();
  for (int j = j0; j + 2 < L; ++j) {
    const int n = L - j - 1;            // trailing size
    const int o = j + 1;                // first trailing index
    double sig2 = 0.0;
    for (int w = 0; w < kTWaves; ++w) sig2 += s.red2[w];
    const double* __restrict__ hrow = &el(j, o);   // reflector data of step j
    const double alpha = hrow[0];
    double beta = 0.0, rv = 0.0, mu = alpha;
    if (sig2 > 0.0) {
      mu = sqrt(alpha * alpha + sig2);
      const double v0 = alpha <= 0.0 ? alpha - mu : -sig2 / (alpha + mu);
      beta = 2.0 * v0 * v0 / (sig2 + v0 * v0);
      rv = 1.0 / v0;
    }
    if (tid == 0) {
      s.d[j] = el(j, j);
      s.e[j] = mu;
      s.hb[j] = beta;
      s.hr[j] = rv;
    }
    // p = beta A22 v, lanes of a group of S share a row
    int S = 1;
    while (S < 8 && 2 * S * n <= kTT) S <<= 1;
    const int rowi = tid / S, part = tid % S;
    double acc = 0.0;
    if (rowi < n) {
      const int i = o + rowi;
#pragma unroll 8
      for (int c = part; c < n; c += S) {
        const double h = hrow[c];
        const double a = el(o + c, i);
        acc += a * (c == 0 ? 1.0 : h * rv);
      }
    }
    acc = group_sum(acc, S);
    double pv = 0.0;
    if (rowi < n && part == 0) {
      const double p = beta * acc;
      const double h = hrow[rowi];
      s.P[rowi] = p;
      pv = p * (rowi == 0 ? 1.0 : h * rv);
    }
    pv = wsum(pv);
    if (lane == 0) s.red[wave] = pv;
    __syncthreads();
    double pvt = 0.0;
    for (int w = 0; w < kTWaves; ++w) pvt += s.red[w];
    const double K = 0.5 * beta * pvt;
    // A22 -= v w^T + w v^T; squares of the new row o beyond its subdiagonal
    const int step = kTT / n;
    double sq = 0.0;
    if (tid < step * n) {
      const int b = tid % n;
      const double hbv = hrow[b];
      const double vb = b == 0 ? 1.0 : hbv * rv;
      const double wb = s.P[b] - K * vb;
      auto upd = [&](int a, double ha, double pa, double old) {
        const double va = a == 0 ? 1.0 : ha * rv;
        const double nv = old - (va * wb + (pa - K * va) * vb);
        el(o + a, o + b) = nv;
        if (a == 0 && b >= 2) sq += nv * nv;
      };
      int a = tid / n;
      // eight of this thread's rows at a time: their operands are read before
      // any of them is written (the rows are distinct, row j is not among them)
      for (; a + 7 * step < n; a += 8 * step) {
        double hv[8], pv[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = a + u * step;
          hv[u] = hrow[r];
          pv[u] = s.P[r];
          xv[u] = el(o + r, o + b);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) upd(a + u * step, hv[u], pv[u], xv[u]);
      }
      for (; a < n; a += step) upd(a, hrow[a], s.P[a], el(o + a, o + b));
    }
    sq = wsum(sq);
    if (lane == 0) s.red2[wave] = sq;
    __syncthreads();
  }
  // the reflectors, in one pass once all steps are done: row j of hh is v_j
  // in full (zero before j + 1, one at j + 1), from row j of the block, which
  // no step after j touches
  const int nb = L - j0;
  for (int t = tid; t < nb * L; t += kTT) {
    const int j = j0 + t / L, c = t % L;
    if (j + 2 < L)
      hh[(int64_t)j * L + c] = c == j + 1 ? 1.0 : (c > j + 1 ? el(j, c) * s.hr[j] : 0.0);
  }
  if (tid == 0) {
    if (L >= 2 && L - 2 >= j0) {
      s.d[L - 2] = el(L - 2, L - 2);
      s.e[L - 2] = el(L - 2, L - 1);
    }
    s.d[L - 1] = el(L - 1, L - 1);
    s.e[L - 1] = 0.0;
  }
  __syncthreads();
}

// The k largest eigenvalues of T = tridiag(e, d, e) into s.lam (descending)
// by multisection on Sturm counts; returns ||T|| (Gershgorin).  All threads.
__device__ double tri_eigvals(int L, int k, const TriSmem& s) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double tn = 0.0, glo = INFINITY, ghi = -INFINITY, emax = 0.0;
  for (int i = tid; i < L; i += kTT) {
    const double r = (i > 0 ? fabs(s.e[i - 1]) : 0.0) + (i + 1 < L ? fabs(s.e[i]) : 0.0);
    tn = fmax(tn, fabs(s.d[i]) + r);
    glo = fmin(glo, s.d[i] - r);
    ghi = fmax(ghi, s.d[i] + r);
    s.e2[i] = i + 1 < L ? s.e[i] * s.e[i] : 0.0;
    emax = fmax(emax, s.e2[i]);
  }
  for (int w = 32; w >= 1; w >>= 1) {
    tn = fmax(tn, __shfl_xor(tn, w, 64));
    glo = fmin(glo, __shfl_xor(glo, w, 64));
    ghi = fmax(ghi, __shfl_xor(ghi, w, 64));
    emax = fmax(emax, __shfl_xor(emax, w, 64));
  }
  if (lane == 0) {
    s.xch[wave] = tn;
    s.xch[kTWaves + wave] = glo;
    s.xch[2 * kTWaves + wave] = ghi;
    s.xch[3 * kTWaves + wave] = emax;
  }
  __syncthreads();
  tn = 0.0; glo = INFINITY; ghi = -INFINITY; emax = 0.0;
  for (int w = 0; w < kTWaves; ++w) {
    tn = fmax(tn, s.xch[w]);
    glo = fmin(glo, s.xch[kTWaves + w]);
    ghi = fmax(ghi, s.xch[2 * kTWaves + w]);
    emax = fmax(emax, s.xch[3 * kTWaves + w]);
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax);
  const double widen = 2.0 * L * kU * tn + 2.0 * pivmin;
  glo -= widen;
  ghi += widen;
  // grid point t of the global pass (the same expression wherever it is used)
  auto grid = [&](int t) { return glo + (ghi - glo) * (double)(t + 1) / (double)(kTT + 1); };
  s.cnt[tid] = sturm(L, s.d, s.e2, grid(tid), pivmin);
  __syncthreads();
  {
    int Gp = 1;
    while (Gp < 64 && 2 * Gp * k <= kTT) Gp <<= 1;
    const int grp = tid / Gp, gl = tid % Gp;
    const bool live = grp < k;
    const int idx = L - 1 - (live ? grp : 0);      // ascending index
    // bracket from the global pass: smallest t with cnt[t] > idx
    int lo_t = 0, hi_t = kTT;
    while (lo_t < hi_t) {
      const int mid = (lo_t + hi_t) >> 1;
      if (s.cnt[mid] > idx) hi_t = mid; else lo_t = mid + 1;
    }
    double lo = lo_t == 0 ? glo : grid(lo_t - 1);
    double hi = lo_t == kTT ? ghi : grid(lo_t);
    const int base = (tid & 63) - gl;               // first lane of the group
    const uint64_t gmask = (Gp == 64) ? ~0ull : ((1ull << Gp) - 1ull);
    for (int round = 0; round < 96; ++round) {
      const double mid = 0.5 * (lo + hi);
      const bool done = !live || (hi - lo) <= fmax(4.0 * kU * fmax(fabs(lo), fabs(hi)),
                                                   2.0 * kU * tn) ||
                        mid <= lo || mid >= hi;
      if (!__any(!done)) break;
      const double x = lo + (hi - lo) * (double)(gl + 1) / (double)(Gp + 1);
      const int c = done ? 0 : sturm(L, s.d, s.e2, x, pivmin);
      const uint64_t m = (__ballot(c <= idx) >> base) & gmask;
      if (!done) {
        const int nle = __popcll(m);
        const double nlo = nle > 0 ? lo + (hi - lo) * (double)nle / (double)(Gp + 1) : lo;
        const double nhi = nle < Gp ? lo + (hi - lo) * (double)(nle + 1) / (double)(Gp + 1) : hi;
        lo = nlo;
        hi = nhi;
      }
    }
    if (live && gl == 0) s.lam[grp] = 0.5 * (lo + hi);
  }
  __syncthreads();

  return tn;
}

__global__ __launch_bounds__(kTT) void tri_topk_kernel(
    int L, const double* __restrict__ G, int64_t ldg, int k, double* __restrict__ S,
    double* __restrict__ D, double* __restrict__ W, int64_t ldw,
    double* __restrict__ hh, int nb) {
  extern __shared__ double smem[];
  const TriSmem s = tri_layout(smem, L, k, nb);
  double* A = s.A;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  for (int t = tid; t < L * L; t += kTT) {
    const int i = t / L, c = t % L;
    A[t] = G[(int64_t)i * ldg + c];
  }
  __syncthreads();

  // ---- 1. tridiagonalisation ----------------------------------------------
  tri_steps(L, 0, A, L, s, hh);
  // ---- 2. eigenvalues by multisection ------------------------------------
  const double tn = tri_eigvals(L, k, s);

  // ---- 3. eigenvectors of T ---------------------------------------------
  double* Z = A;                       // L x k
  double* C = A + (size_t)L * k;       // k x k
  double* Uf = C + (size_t)k * k;      // 3 x L x nb rows of U for a batch
  double* lfb = Uf + 3 * (size_t)L * nb;  // L x nb multipliers
  int* swb = (int*)(lfb + (size_t)L * nb);  // L x nb row exchanges
  for (int t = tid; t < L * k; t += kTT) {
    const int i = t / k, j = t % k;
    const uint64_t h = mix64(((uint64_t)(j + 1) << 32) ^ (uint64_t)i);
    Z[t] = (double)(h >> 11) * 0x1.0p-53 - 0.5;
  }
  __syncthreads();
  for (int j0 = 0; j0 < k; j0 += nb) {
    const int j = j0 + tid;
    if (tid < nb && j < k)
      invit_column(L, k, j, s.d, s.e, s.lam[j], tn, Z, Uf + 3 * tid, 3 * nb, lfb + tid,
                   swb + tid, nb);
  }
  __syncthreads();
  cholqr_lds(L, k, Z, C);
  polar_step_lds(L, k, Z, C);
  for (int j = tid; j < k; j += kTT) {
    double rq = 0.0;
    for (int i = 0; i < L; ++i) {
      const double z = Z[i * k + j];
      rq += s.d[i] * z * z;
      if (i + 1 < L) rq += 2.0 * s.e[i] * z * Z[(i + 1) * k + j];
    }
    D[j] = rq;
    S[j] = sqrt(fmax(rq, 0.0));
  }
  for (int t = tid; t < L * k; t += kTT) {
    const int i = t / k, j = t % k;
    W[(int64_t)i * ldw + j] = Z[t];
  }
  __syncthreads();
  // reflector data back into LDS (row j, columns j+1 ..): one copy of the
  // whole square, whose other entries the back-transformation never reads
  for (int t = tid; t < L * L; t += kTT) A[t] = hh[t];
  __syncthreads();

  // ---- 4. back-transformation -------------------------------------------
  const int vlane = tid % kVecLanes;
  for (int base = 0; base < k; base += kTT / kVecLanes) {
    const int col = base + tid / kVecLanes;
    const bool act = col < k;
    double z[kVecRegs];
#pragma unroll
    for (int q = 0; q < kVecRegs; ++q) {
      const int i = vlane + kVecLanes * q;
      z[q] = (act && i < L) ? W[(int64_t)i * ldw + col] : 0.0;
    }
    for (int j = L - 3; j >= 0; --j) {
      const double beta = s.hb[j];
      double v[kVecRegs];
      double dot = 0.0;
#pragma unroll
      for (int q = 0; q < kVecRegs; ++q) {
        const int i = vlane + kVecLanes * q;
        v[q] = i < L ? A[j * L + min(i, L - 1)] : 0.0;
        dot += v[q] * z[q];
      }
      dot = group_sum(dot, kVecLanes) * beta;
#pragma unroll
      for (int q = 0; q < kVecRegs; ++q) z[q] -= dot * v[q];
    }
    if (act) {
#pragma unroll
      for (int q = 0; q < kVecRegs; ++q) {
        const int i = vlane + kVecLanes * q;
        if (i < L) W[(int64_t)i * ldw + col] = z[q];
      }
    }
  }
}

// ---- matrices too large for one workgroup's LDS -----------------------------
// The first j0 = L - Ls Householder steps run on a copy of G in global memory,
// one launch per step; a one-workgroup kernel then finishes the trailing
// Ls x Ls block in LDS.  Eigenpairs: one workgroup per wanted eigenvalue
// finds it by multisection and its vector by inverse iteration; Cholesky QR
// and a Newton-Schulz step with the Gram and panel kernels; a back-
// transformation kernel with each vector in registers.

constexpr int kBigRows = 4;        // trailing rows per workgroup (one per wavefront)
constexpr int kStepPer = 16;       // row entries per lane: rows of up to 64 * 16 = 1024
static_assert(64 * kStepPer >= 64 * kVecLanes, "big_step_kernel rows must cover tri_big_max()");

// Launch j (0 <= j < j0) of the tridiagonalisation.  It first applies the
// rank-2 update of step j-1, A22 -= v w^T + w v^T with w = p - (beta/2)(p^T v) v,
// which the previous launch left pending (it needs p complete), to this
// workgroup's rows, restricted to rows and columns > j.  Every workgroup
// rebuilds the updated row j from the stored row and the vectors of step
// j-1, takes the reflector of step j from it, and forms p = beta A22 v for
// its own rows (whole rows, so p needs no reduction across workgroups) and
// its share of p^T v.  Workgroup 0 records the reflector.  Launch j = j0
// applies the last pending update to rows and columns >= j0 and stops.
// p and the p^T v partials alternate between two buffers by step parity.
// Everything the launch reads from global memory is requested at its start,
// and it has three barriers.
__global__ __launch_bounds__(256) void big_step_kernel(
    int L, int j, int j0, double* __restrict__ Ag, double* __restrict__ hh,
    double* __restrict__ dg, double* __restrict__ eg, double* __restrict__ hbg,
    double* __restrict__ hrg, double* __restrict__ Pbuf, double* __restrict__ pbuf) {
  extern __shared__ double sv[];
  double* vp = sv;            // v of step j-1 on [j, L)
  double* wp = vp + L;        // w of step j-1 on [j, L)
  double* vj = wp + L;        // row j after step j-1, on [j + 1, L) (not scaled)
  __shared__ double redp[4], red[4], redq[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool last = j == j0;
  const int o = last ? j : j + 1;             // first row / column this launch touches
  const int npart_stride = (L + kBigRows - 1) / kBigRows;
  const bool upd = j >= 1;
  const int jp = j - 1;
  // this wavefront's trailing row (stored with the updates up to step j-2)
  const int r = blockIdx.x * kBigRows + wave;
  const int a = o + r;
  const bool has_row = a < L;
  double xs[kStepPer];
  if (has_row) {
    const double* __restrict__ row = Ag + (int64_t)a * L;
#pragma unroll
    for (int u = 0; u < kStepPer; ++u) xs[u] = row[min(o + lane + 64 * u, L - 1)];
  }
  // row j (likewise; step j-1's update of it is applied below), and step
  // j-1's reflector row and p, at columns c = j + tid + 256 u: the thread
  // that forms vp[c], wp[c] also updates row j at c
  constexpr int kRowJ = 1024 / 256;            // entries per thread (L <= 1024)
  double xj[kRowJ], hv[kRowJ], pw[kRowJ];
  double djj = 0.0;
#pragma unroll
  for (int u = 0; u < kRowJ; ++u) {
    const int c = j + tid + 256 * u;
    const bool in = c < L;
    xj[u] = (!last && in) ? Ag[(int64_t)j * L + c] : 0.0;
    hv[u] = (upd && in) ? hh[(int64_t)jp * L + c] : 0.0;
    pw[u] = (upd && in) ? Pbuf[(size_t)(jp & 1) * L + (c - j)] : 0.0;
  }
  if (!last && blockIdx.x == 0 && tid == 0) djj = Ag[(int64_t)j * L + j];
  // p_j of step j-1 (w_j = p_j - K, since v_j = 1), needed by every thread
  const double p0 = upd ? Pbuf[(size_t)(jp & 1) * L] : 0.0;
  double K = 0.0;
  if (upd) {
    const double bp = hbg[jp];
    const double* __restrict__ pp = pbuf + (size_t)(jp & 1) * npart_stride;
    const int nparts = (L - j + kBigRows - 1) / kBigRows;
    double pv = 0.0;
    for (int w = tid; w < nparts; w += 256) pv += pp[w];
    // p^T v: the partials summed by the whole workgroup
    pv = wsum(pv);
    if (lane == 0) redp[wave] = pv;
    __syncthreads();
    const double pvt = (redp[0] + redp[1]) + (redp[2] + redp[3]);
    K = 0.5 * bp * pvt;
#pragma unroll
    for (int u = 0; u < kRowJ; ++u) {
      const int c = j + tid + 256 * u;
      if (c < L) {
        const double v = hv[u];
        pw[u] = pw[u] - K * v;
        vp[c] = v;
        wp[c] = pw[u];
      }
    }
  }
  const int n = L - o;
  double sq = 0.0;
  if (!last) {
    // row j after step j-1 needs v_j = 1 and w_j, which every thread forms
    // itself (the same expressions as vp[j], wp[j]) rather than waiting for LDS
    const double vjj = 1.0;
    const double wjj = upd ? p0 - K * vjj : 0.0;
#pragma unroll
    for (int u = 0; u < kRowJ; ++u) {
      const int c = j + tid + 256 * u;
      if (c >= o && c < L) {
        double x = xj[u];
        if (upd) x -= vjj * pw[u] + wjj * hv[u];
        vj[c] = x;
        if (c > o) sq += x * x;
      }
    }
    if (blockIdx.x == 0 && tid == 0) {
      if (upd) djj -= vjj * wjj + wjj * vjj;
      dg[j] = djj;
    }
  }
  sq = wsum(sq);
  if (lane == 0) red[wave] = sq;
  __syncthreads();                            // vj, vp, wp and the sums are complete
  if (!last) {
    const double sig2 = (red[0] + red[1]) + (red[2] + red[3]);
    const double alpha = vj[o];
    double beta = 0.0, rv = 0.0, mu = alpha;
    if (sig2 > 0.0) {
      mu = sqrt(alpha * alpha + sig2);
      const double v0 = alpha <= 0.0 ? alpha - mu : -sig2 / (alpha + mu);
      beta = 2.0 * v0 * v0 / (sig2 + v0 * v0);
      rv = 1.0 / v0;
    }
    if (blockIdx.x == 0) {
      if (tid == 0) {
        eg[j] = mu;
        hbg[j] = beta;
        hrg[j] = rv;
      }
      for (int c = tid; c < L; c += 256)
        hh[(int64_t)j * L + c] = c < o ? 0.0 : (c == o ? 1.0 : vj[c] * rv);
    }
    // this workgroup's rows: update by step j-1, then p = beta A22 v with
    // v = (1, vj[o+1..] / v0)
    double pr = 0.0;
    if (r < n) {
      double* __restrict__ row = Ag + (int64_t)a * L;
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < kStepPer; ++u) {
        const int c = o + lane + 64 * u;
        if (c < L) {
          double x = xs[u];
          if (upd) {
            x -= vp[a] * wp[c] + wp[a] * vp[c];
            row[c] = x;
          }
          acc += x * (c == o ? 1.0 : vj[c] * rv);
        }
      }
      acc = wsum(acc);
      pr = beta * acc;
      if (lane == 0) Pbuf[(size_t)(j & 1) * L + r] = pr;
    }
    if (lane == 0) redq[wave] = r < n ? pr * (r == 0 ? 1.0 : vj[o + r] * rv) : 0.0;
    __syncthreads();
    if (tid == 0)
      pbuf[(size_t)(j & 1) * npart_stride + blockIdx.x] =
          (redq[0] + redq[1]) + (redq[2] + redq[3]);
  } else if (upd) {
    // the pending update of step j0 - 1 on rows and columns >= j0
    if (has_row) {
      double* __restrict__ row = Ag + (int64_t)a * L;
#pragma unroll
      for (int u = 0; u < kStepPer; ++u) {
        const int c = o + lane + 64 * u;
        if (c < L) row[c] = xs[u] - (vp[a] * wp[c] + wp[a] * vp[c]);
      }
    }
  }
}

// Ag (L x L, ld L) = G (ld ldg): a kernel, so that the sequence can be
// captured as a graph
__global__ __launch_bounds__(256) void copy_square_kernel(int L, const double* __restrict__ G,
                                                          int64_t ldg, double* __restrict__ Ag) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)L * L) return;
  const int64_t r = t / L, c = t % L;
  Ag[t] = G[r * ldg + c];
}

// The trailing block (rows and columns j0 ..) in LDS: the remaining steps.
// Writes d, e, hb, hr for every step.
__global__ __launch_bounds__(kTT) void tri_tail_kernel(
    int L, int j0, const double* __restrict__ Ag, double* __restrict__ hh,
    double* __restrict__ dg, double* __restrict__ eg, double* __restrict__ hbg,
    double* __restrict__ hrg) {
  extern __shared__ double smem[];
  const int Ls = L - j0;
  const TriSmem s = tri_layout_r(smem, L, (size_t)Ls * Ls);
  const int tid = threadIdx.x;
  for (int t = tid; t < Ls * Ls; t += kTT) {
    const int r = t / Ls, c = t % Ls;
    s.A[t] = Ag[(int64_t)(j0 + r) * L + j0 + c];
  }
  __syncthreads();
  tri_steps(L, j0, s.A, Ls, s, hh);
  for (int i = j0 + tid; i < L; i += kTT) {
    dg[i] = s.d[i];
    eg[i] = s.e[i];
    hbg[i] = s.hb[i];
    hrg[i] = s.hr[i];
  }
}

constexpr int kEigT = 256;         // multisection points per round (one per thread)

// Eigenvalue j (the j-th largest) of T = tridiag(e, d, e) by multisection on
// Sturm counts, kEigT points per round, each round narrowing the bracket by
// a factor kEigT + 1; then two inverse-iteration steps for its vector, whose
// column lands in Zg (L x k, row-major): the solves in one thread, the second
// reusing the first one's factorisation, the normalisations by the whole
// workgroup.  One workgroup per eigenvalue, so the k searches and solves run
// side by side on k compute units.
__global__ __launch_bounds__(kEigT) void big_eigvec_kernel(
    int L, int k, const double* __restrict__ dg, const double* __restrict__ eg,
    double* __restrict__ Zg) {
  extern __shared__ double smem[];
  double* d = smem;
  double* e = d + L;
  double* e2 = e + L;                         // e^2; the multipliers after the search
  double* z = e2 + L;
  double* U = z + L;                          // 3 L
  int* sw = (int*)(U + 3 * (size_t)L);        // L row exchanges
  __shared__ double red[4 * (kEigT / 64)];
  __shared__ int cnt[kEigT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int kW = kEigT / 64;
  const int j = blockIdx.x;
  for (int i = tid; i < L; i += kEigT) {
    d[i] = dg[i];
    e[i] = eg[i];
    const uint64_t h = mix64(((uint64_t)(j + 1) << 32) ^ (uint64_t)i);
    z[i] = (double)(h >> 11) * 0x1.0p-53 - 0.5;
  }
  __syncthreads();
  // Gershgorin interval, ||T||, and the pivot floor
  double tn = 0.0, glo = INFINITY, ghi = -INFINITY, emax = 0.0;
  for (int i = tid; i < L; i += kEigT) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < L ? fabs(e[i]) : 0.0);
    tn = fmax(tn, fabs(d[i]) + r);
    glo = fmin(glo, d[i] - r);
    ghi = fmax(ghi, d[i] + r);
    e2[i] = i + 1 < L ? e[i] * e[i] : 0.0;
    emax = fmax(emax, e2[i]);
  }
  for (int w = 32; w >= 1; w >>= 1) {
    tn = fmax(tn, __shfl_xor(tn, w, 64));
    glo = fmin(glo, __shfl_xor(glo, w, 64));
    ghi = fmax(ghi, __shfl_xor(ghi, w, 64));
    emax = fmax(emax, __shfl_xor(emax, w, 64));
  }
  if (lane == 0) {
    red[wave] = tn;
    red[kW + wave] = glo;
    red[2 * kW + wave] = ghi;
    red[3 * kW + wave] = emax;
  }
  __syncthreads();
  tn = 0.0; glo = INFINITY; ghi = -INFINITY; emax = 0.0;
  for (int w = 0; w < kW; ++w) {
    tn = fmax(tn, red[w]);
    glo = fmin(glo, red[kW + w]);
    ghi = fmax(ghi, red[2 * kW + w]);
    emax = fmax(emax, red[3 * kW + w]);
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax);
  const double widen = 2.0 * L * kU * tn + 2.0 * pivmin;
  double lo = glo - widen, hi = ghi + widen;
  const int idx = L - 1 - j;                  // ascending index
  // every thread holds the same bracket: the count of points at or below idx
  // is shared, and the new ends are the same expressions as the points
  for (int round = 0; round < 64; ++round) {
    const double mid = 0.5 * (lo + hi);
    if ((hi - lo) <= fmax(4.0 * kU * fmax(fabs(lo), fabs(hi)), 2.0 * kU * tn) || mid <= lo ||
        mid >= hi)
      break;
    const double x = lo + (hi - lo) * (double)(tid + 1) / (double)(kEigT + 1);
    const int c = sturm(L, d, e2, x, pivmin);
    const uint64_t m = __ballot(c <= idx);
    if (lane == 0) cnt[wave] = __popcll(m);
    __syncthreads();
    int nle = 0;
    for (int w = 0; w < kW; ++w) nle += cnt[w];
    __syncthreads();                          // cnt is rewritten next round
    const double nlo = nle > 0 ? lo + (hi - lo) * (double)nle / (double)(kEigT + 1) : lo;
    const double nhi =
        nle < kEigT ? lo + (hi - lo) * (double)(nle + 1) / (double)(kEigT + 1) : hi;
    lo = nlo;
    hi = nhi;
  }
  // two inverse-iteration steps: the solves in thread 0 (the second reuses
  // the factorisation), each followed by a normalisation by all threads
  const double lam = 0.5 * (lo + hi);
  const double ptiny = fmax(kU * tn, DBL_MIN / kU);
  __syncthreads();                            // e2 is the multipliers' array now
  for (int pass = 0; pass < 2; ++pass) {
    if (tid == 0)
      red[0] = pass == 0 ? invit_solve<true>(L, 1, 0, d, e, lam, ptiny, z, U, 3, e2, sw, 1)
                         : invit_solve<false>(L, 1, 0, d, e, lam, ptiny, z, U, 3, e2, sw, 1);
    __syncthreads();
    const double zmax = red[0];
    const double inv = zmax > 0.0 ? rcp(zmax) : 1.0;
    double ss = 0.0;
    for (int i = tid; i < L; i += kEigT) {
      const double x = z[i] * inv;
      ss += x * x;
    }
    ss = wsum(ss);
    __syncthreads();                          // red[0] is read by everyone
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    double sst = 0.0;
    for (int w = 0; w < kW; ++w) sst += red[w];
    const double sc = inv * rcp(sqrt(sst));
    for (int i = tid; i < L; i += kEigT) z[i] *= sc;
    __syncthreads();
  }
  for (int i = tid; i < L; i += kEigT) Zg[(int64_t)i * k + j] = z[i];
}

// C (k x k, symmetric positive definite) -> R^{-1} (upper triangular, with
// zeros below) for C = R^T R, in one workgroup.  The factorisation runs in
// the first wavefront; each thread then forms one column of R^{-1} by back
// substitution.  Pivots below 1e-28 are clamped (columns enter with unit norm).
__global__ __launch_bounds__(256) void chol_rinv_kernel(int k, const double* __restrict__ Cg,
                                                        double* __restrict__ Rinv) {
  extern __shared__ double smem[];
  double* C = smem;             // upper: Schur rows; lower: R^{-1} transposed
  double* rd = C + (size_t)k * k;
  const int tid = threadIdx.x;
  for (int t = tid; t < k * k; t += 256) C[t] = Cg[t];
  __syncthreads();
  if (tid < 64) {
    for (int c = 0; c < k; ++c) {
      const double rp = rcp(fmax(C[c * k + c], 1e-28));
      const int n = k - c - 1;
      for (int t = tid; t < n * n; t += 64) {
        const int a = c + 1 + t / n, b = c + 1 + t % n;
        if (a > b) continue;
        C[a * k + b] -= C[c * k + a] * C[c * k + b] * rp;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  for (int t = tid; t < k; t += 256) rd[t] = sqrt(fmax(C[t * k + t], 1e-28));
  __syncthreads();
  // column c of R^{-1}: X_cc = 1 / R_cc, X_lc = -(sum_{m=l+1..c} R_lm X_mc) / R_ll,
  // with R_lm = C_lm / R_ll; X_lc is kept at C[c][l] (l <= c, lower part)
  for (int c = tid; c < k; c += 256) {
    C[c * k + c] = 0.0;                    // the diagonal is read only through rd
    const double xcc = 1.0 / rd[c];
    for (int l = c - 1; l >= 0; --l) {
      double acc = C[l * k + c] / rd[l] * xcc;
      for (int m = l + 1; m < c; ++m) acc += C[l * k + m] / rd[l] * C[c * k + m];
      C[c * k + l] = -acc / rd[l];
    }
    C[c * k + c] = xcc;
  }
  __syncthreads();
  for (int t = tid; t < k * k; t += 256) {
    const int a = t / k, b = t % k;
    Rinv[t] = a <= b ? C[b * k + a] : 0.0;
  }
}

// The same for k <= 128 with the matrix in registers (1024 threads, one
// barrier per column; pivots clamped below at 1e-28 as above).
template <int N>
__global__ __launch_bounds__(1024) void chol_rinv_regs_kernel(int k,
                                                             const double* __restrict__ Cg,
                                                             double* __restrict__ Rinv) {
  extern __shared__ double smem[];
  chol_inv_regs<N, N>(k, Cg, k, Rinv, k, smem, 0, nullptr, nullptr, true);
}

void launch_chol_rinv(int k, const double* C, double* Ri, hipStream_t st) {
  const size_t lds3 = sizeof(double) * 3 * (size_t)k;
  if (k <= 32)
    hipLaunchKernelGGL(chol_rinv_regs_kernel<1>, dim3(1), dim3(1024), lds3, st, k, C, Ri);
  else if (k <= 64)
    hipLaunchKernelGGL(chol_rinv_regs_kernel<2>, dim3(1), dim3(1024), lds3, st, k, C, Ri);
  else if (k <= 96)
    hipLaunchKernelGGL(chol_rinv_regs_kernel<3>, dim3(1), dim3(1024), lds3, st, k, C, Ri);
  else if (k <= 128)
    hipLaunchKernelGGL(chol_rinv_regs_kernel<4>, dim3(1), dim3(1024), lds3, st, k, C, Ri);
  else
    hipLaunchKernelGGL(chol_rinv_kernel, dim3(1), dim3(256),
                       sizeof(double) * ((size_t)k * k + k), st, k, C, Ri);
  MC_CHECK_LAUNCH();
}

// M = (3 I - C) / 2 in place (C symmetric k x k)
__global__ void ns_matrix_kernel(int k, double* __restrict__ C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * k) return;
  const int a = t / k, b = t % k;
  C[t] = (a == b ? 1.5 : 0.0) - 0.5 * C[t];
}

constexpr int kBackT = 256;            // back-transformation: 4 vectors per workgroup
constexpr int kBackLds = 7680;         // doubles of staged reflector rows (60 KB)

// Rayleigh quotients on T and W = H_0 ... H_{L-3} Z: one wavefront per
// vector, entries lane + 64 q in registers (q < R).  The reflector rows come
// in chunks of C consecutive rows (one contiguous stretch of hh), staged in
// LDS by the whole workgroup, so the global-memory latency is paid once per
// chunk instead of once per reflector.
template <int R>
__global__ __launch_bounds__(kBackT) void big_back_kernel(
    int L, int k, int C, const double* __restrict__ Zg, const double* __restrict__ hh,
    const double* __restrict__ hbg, const double* __restrict__ dg,
    const double* __restrict__ eg, double* __restrict__ S, double* __restrict__ D,
    double* __restrict__ W, int64_t ldw) {
  extern __shared__ double hs[];               // C x L
  __shared__ double bs[kBackLds / 64];
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (kBackT / 64) + (threadIdx.x >> 6);
  const bool act = col < k;                    // whole wavefronts; all of them stage
  double z[R];
  double rq = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = lane + 64 * q;
    const bool in = act && i < L;
    const int ic = min(i, L - 1);
    const double zi = in ? Zg[(int64_t)ic * k + col] : 0.0;
    const double zp = (in && i + 1 < L) ? Zg[(int64_t)(ic + 1) * k + col] : 0.0;
    z[q] = zi;
    rq += zi * (dg[ic] * zi + 2.0 * eg[ic] * zp);
  }
  rq = wsum(rq);
  if (act && lane == 0) {
    D[col] = rq;
    S[col] = sqrt(fmax(rq, 0.0));
  }
  for (int jh = L - 3; jh >= 0; jh -= C) {
    const int jl = max(jh - C + 1, 0);
    const int nr = jh - jl + 1;
    __syncthreads();                           // the previous chunk is consumed
    const double* __restrict__ src = hh + (int64_t)jl * L;
#pragma unroll 8
    for (int t = threadIdx.x; t < nr * L; t += kBackT) hs[t] = src[t];
    for (int t = threadIdx.x; t < nr; t += kBackT) bs[t] = hbg[jl + t];
    __syncthreads();
    if (act) {
      for (int j = jh; j >= jl; --j) {
        // the stored v_j holds its zeros, so no masks; four partial sums
        // shorten the dependent chain
        const double* hr = hs + (size_t)(j - jl) * L;
        double v[R];
        double dp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = lane + 64 * q;
          v[q] = i < L ? hr[min(i, L - 1)] : 0.0;
          dp[q & 3] += v[q] * z[q];
        }
        const double dot = wsum((dp[0] + dp[1]) + (dp[2] + dp[3])) * bs[j - jl];
#pragma unroll
        for (int q = 0; q < R; ++q) z[q] -= dot * v[q];
      }
    }
  }
  if (act) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int i = lane + 64 * q;
      if (i < L) W[(int64_t)i * ldw + col] = z[q];
    }
  }
}

}  // namespace

size_t tri_lds_bytes(int L, int k, int nb) {
  return sizeof(double) * (tri_region(L, k, nb) + 7 * (size_t)L + 6 * kTWaves) +
         sizeof(int) * kTT;
}

// inverse iterations run side by side (as many as LDS holds, at least one)
int tri_batch(int L, int k, size_t lds_bytes) {
  int nb = k;
  while (nb > 1 && tri_lds_bytes(L, k, nb) > lds_bytes) --nb;
  return nb;
}

bool tri_fits(int L, int k, size_t lds_bytes) {
  return L >= 1 && k >= 1 && k <= L && L <= kVecLanes * kVecRegs &&
         tri_lds_bytes(L, k, 1) <= lds_bytes;
}

const void* tri_kernel_ptr() { return (const void*)tri_topk_kernel; }

void tri_set_lds_attributes(size_t lim) {
  for (const void* f : {(const void*)tri_tail_kernel, (const void*)chol_rinv_kernel})
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) !=
        hipSuccess)
      (void)hipGetLastError();
}

int tri_big_max() { return kVecLanes * 64; }
int tri_big_kmax() { return 140; }       // chol_rinv_kernel keeps k x k in LDS

// trailing block solved in LDS by the tail kernel
static int tail_block(int L, size_t lds_bytes) {
  const size_t fixed = sizeof(double) * (7 * (size_t)L + 6 * kTWaves) + sizeof(int) * kTT;
  int Ls = 1;
  while (Ls + 1 <= L && fixed + sizeof(double) * (size_t)(Ls + 1) * (Ls + 1) <= lds_bytes)
    ++Ls;
  return Ls;
}

size_t TriBigWork::doubles(int L, int k) {
  const size_t nparts = (size_t)(L + kBigRows - 1) / kBigRows;
  const size_t splits = (size_t)gram_splits(L, k, k, 1);
  return 2 * (size_t)L * L + 6 * (size_t)L + 2 * nparts + 2 * (size_t)L * k +
         3 * (size_t)k * k + splits * k * k;
}

void launch_tri_big(int L, const double* G, int64_t ldg, int k, double* S, double* D,
                    double* W, int64_t ldw, double* ws, size_t ws_doubles,
                    size_t lds_bytes, hipStream_t st) {
  MC_REQUIRE(L <= tri_big_max() && k >= 1 && k <= L && k <= tri_big_kmax(), kEINVAL,
             "eigensolve size out of range");
  MC_REQUIRE(TriBigWork::doubles(L, k) <= ws_doubles, kEINVAL, "eigensolver workspace");
  const int nparts = (L + kBigRows - 1) / kBigRows;
  double* Ag = ws;
  double* hh = Ag + (size_t)L * L;
  double* dg = hh + (size_t)L * L;
  double* eg = dg + L;
  double* hbg = eg + L;
  double* hrg = hbg + L;
  double* Pg = hrg + L;                      // p of two consecutive steps
  double* part = Pg + 2 * (size_t)L;         // their p^T v partials
  double* Zg = part + 2 * (size_t)nparts;
  double* Z2 = Zg + (size_t)L * k;
  double* C = Z2 + (size_t)L * k;
  double* Ri = C + (size_t)k * k;
  double* gpart = Ri + (size_t)k * k;
  const int64_t gcap = gram_splits(L, k, k, 1) * (int64_t)k * k;
  hipLaunchKernelGGL(copy_square_kernel, dim3((unsigned)(((int64_t)L * L + 255) / 256)),
                     dim3(256), 0, st, L, G, ldg, Ag);
  MC_CHECK_LAUNCH();
  const int Ls = tail_block(L, lds_bytes);
  const int j0 = L - Ls;
  const size_t step_lds = 3 * sizeof(double) * (size_t)L;
  for (int j = 0; j <= j0; ++j) {
    if (j == j0 && j0 == 0) break;             // nothing pending
    const int o = j == j0 ? j : j + 1;
    const int nb = (L - o + kBigRows - 1) / kBigRows;
    hipLaunchKernelGGL(big_step_kernel, dim3((unsigned)nb), dim3(256), step_lds, st, L, j,
                       j0, Ag, hh, dg, eg, hbg, hrg, Pg, part);
    MC_CHECK_LAUNCH();
  }
  const size_t tail_bytes = sizeof(double) * ((size_t)Ls * Ls + 7 * (size_t)L + 6 * kTWaves) +
                            sizeof(int) * kTT;
  hipLaunchKernelGGL(tri_tail_kernel, dim3(1), dim3(kTT), tail_bytes, st, L, j0, Ag, hh,
                     dg, eg, hbg, hrg);
  MC_CHECK_LAUNCH();
  hipLaunchKernelGGL(big_eigvec_kernel, dim3(k), dim3(kEigT),
                     sizeof(double) * 7 * (size_t)L + sizeof(int) * (size_t)L, st, L, k, dg, eg,
                     Zg);
  MC_CHECK_LAUNCH();
  // Cholesky QR, then one Newton-Schulz step
  launch_gram<double, double>(L, k, k, Zg, k, Zg, k, C, k, 1, gpart, gcap, st);
  launch_chol_rinv(k, C, Ri, st);
  launch_panel_gemm<double, double>(L, k, k, Zg, k, Ri, k, 1.0, nullptr, 0.0, nullptr, 0,
                                    Z2, k, st);
  launch_gram<double, double>(L, k, k, Z2, k, Z2, k, C, k, 1, gpart, gcap, st);
  hipLaunchKernelGGL(ns_matrix_kernel, dim3((k * k + 255) / 256), dim3(256), 0, st, k, C);
  MC_CHECK_LAUNCH();
  launch_panel_gemm<double, double>(L, k, k, Z2, k, C, k, 1.0, nullptr, 0.0, nullptr, 0, Zg,
                                    k, st);
  const dim3 grid((unsigned)((k + kBackT / 64 - 1) / (kBackT / 64)));
  const int rows = std::max(1, std::min(kBackLds / L, kBackLds / 64));   // per chunk
  const size_t back_lds = sizeof(double) * (size_t)rows * L;
  if (L <= 512)
    hipLaunchKernelGGL(big_back_kernel<8>, grid, dim3(kBackT), back_lds, st, L, k, rows, Zg,
                       hh, hbg, dg, eg, S, D, W, ldw);
  else
    hipLaunchKernelGGL(big_back_kernel<16>, grid, dim3(kBackT), back_lds, st, L, k, rows, Zg,
                       hh, hbg, dg, eg, S, D, W, ldw);
  MC_CHECK_LAUNCH();
}

void launch_tri_topk(int L, const double* G, int64_t ldg, int k, double* S, double* D,
                     double* W, int64_t ldw, double* hh, size_t lds_bytes,
                     hipStream_t st) {
  const int nb = tri_batch(L, k, lds_bytes);
  hipLaunchKernelGGL(tri_topk_kernel, dim3(1), dim3(kTT), tri_lds_bytes(L, k, nb), st, L,
                     G, ldg, k, S, D, W, ldw, hh, nb);
  MC_CHECK_LAUNCH();
}

}  // namespace mcsvt
