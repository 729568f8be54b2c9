// Top-k eigenpairs of the symmetric Gram matrix of eigSVD (Alg. 3 step 2 and
// Alg. 5 steps 9-10) inside one workgroup, for L small enough that the whole
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
//      with the vector held in registers.
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

// doubles of the matrix region: A (L x L), later Z (L x k), C (k x k) and
// the U factors of a batch of nb inverse iterations (3 L nb)
__host__ __device__ inline size_t tri_region(int L, int k, int nb) {
  const size_t a = (size_t)L * L, b = (size_t)L * k + (size_t)k * k + 3 * (size_t)L * nb;
  return a > b ? a : b;
}

__device__ TriSmem tri_layout(double* sm, int L, int k, int nb) {
  TriSmem s;
  s.A = sm;
  double* q = sm + tri_region(L, k, nb);
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

// Two steps of inverse iteration for eigenvalue lam on column j of Z (the
// right-hand side on entry, the normalised solution on exit).  The rows of
// the U factor of the pivoted LU of T - lam I (3 values per row) go to Uf
// with stride ldu between rows and unit stride between columns of a batch.
__device__ void invit_column(int L, int k, int j, const double* d, const double* e,
                             double lam, double tnorm, double* Z, double* Uf, int ldu) {
  const double ptiny = fmax(kU * tnorm, DBL_MIN / kU);
  for (int pass = 0; pass < 2; ++pass) {
    double r0 = d[0] - lam;
    double r1 = L > 1 ? e[0] : 0.0;
    double ycur = Z[j];
    for (int i = 0; i + 1 < L; ++i) {
      const double c = e[i];
      const double a1 = d[i + 1] - lam;
      const double b1 = e[i + 1];            // e[L - 1] = 0
      const double ynext = Z[(i + 1) * k + j];
      double u0, u1, u2;
      if (fabs(r0) >= fabs(c)) {
        const double l = r0 != 0.0 ? c * rcp(r0) : 0.0;
        u0 = r0; u1 = r1; u2 = 0.0;
        r0 = a1 - l * r1;
        r1 = b1;
        Z[i * k + j] = ycur;
        ycur = ynext - l * ycur;
      } else {
        const double l = r0 * rcp(c);
        u0 = c; u1 = a1; u2 = b1;
        r0 = r1 - l * a1;
        r1 = -l * b1;
        Z[i * k + j] = ynext;
        ycur = ycur - l * ynext;
      }
      double* u = Uf + (size_t)i * ldu;
      u[0] = u0; u[1] = u1; u[2] = u2;
    }
    {
      double* u = Uf + (size_t)(L - 1) * ldu;
      u[0] = r0; u[1] = 0.0; u[2] = 0.0;
    }
    Z[(L - 1) * k + j] = ycur;
    // back substitution, rescaling if the solution grows past 2^500
    double z1 = 0.0, z2 = 0.0, zmax = 0.0;
    for (int i = L - 1; i >= 0; --i) {
      const double* u = Uf + (size_t)i * ldu;
      double u0 = u[0];
      if (fabs(u0) < ptiny) u0 = u0 < 0.0 ? -ptiny : ptiny;
      double z = (Z[i * k + j] - u[1] * z1 - u[2] * z2) * rcp(u0);
      if (fabs(z) > 0x1p500) {
        const double sc = 0x1p-500;
        for (int t = 0; t < L; ++t)
          if (t != i) Z[t * k + j] *= sc;
        z *= sc; z1 *= sc; z2 *= sc; zmax *= sc;
      }
      Z[i * k + j] = z;
      zmax = fmax(zmax, fabs(z));
      z2 = z1;
      z1 = z;
    }
    const double inv = zmax > 0.0 ? rcp(zmax) : 1.0;
    double ss = 0.0;
    for (int i = 0; i < L; ++i) {
      const double z = Z[i * k + j] * inv;
      ss += z * z;
    }
    const double sc = inv * rcp(sqrt(ss));
    for (int i = 0; i < L; ++i) Z[i * k + j] *= sc;
  }
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
  {
    double sq = 0.0;
    for (int c = 2 + tid; c < L; c += kTT) sq += A[c] * A[c];
    sq = wsum(sq);
    if (lane == 0) s.red2[wave] = sq;
  }
  __syncthreads();
  for (int j = 0; j + 2 < L; ++j) {
    const int n = L - j - 1;            // trailing size
    const int o = j + 1;                // first trailing index
    double sig2 = 0.0;
    for (int w = 0; w < kTWaves; ++w) sig2 += s.red2[w];
    const double alpha = A[j * L + o];
    double beta = 0.0, rv = 0.0, mu = alpha;
    if (sig2 > 0.0) {
      mu = sqrt(alpha * alpha + sig2);
      const double v0 = alpha <= 0.0 ? alpha - mu : -sig2 / (alpha + mu);
      beta = 2.0 * v0 * v0 / (sig2 + v0 * v0);
      rv = 1.0 / v0;
    }
    if (tid == 0) {
      s.d[j] = A[j * L + j];
      s.e[j] = mu;
      s.hb[j] = beta;
      s.hr[j] = rv;
    }
    for (int t = tid; t < n; t += kTT) hh[(int64_t)j * L + o + t] = A[j * L + o + t];
    // p = beta A22 v, lanes of a group of S share a row
    int S = 1;
    while (S < 8 && 2 * S * n <= kTT) S <<= 1;
    const int rowi = tid / S, part = tid % S;
    double acc = 0.0;
    if (rowi < n) {
      const int i = o + rowi;
      const double* __restrict__ hrow = A + j * L + o;      // reflector data
#pragma unroll 4
      for (int c = part; c < n; c += S) {
        const double h = hrow[c];
        const double a = A[(o + c) * L + i];
        acc += a * (c == 0 ? 1.0 : h * rv);
      }
    }
    acc = group_sum(acc, S);
    double pv = 0.0;
    if (rowi < n && part == 0) {
      const double p = beta * acc;
      const double h = A[j * L + o + rowi];
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
      const double hb = A[j * L + o + b];
      const double vb = b == 0 ? 1.0 : hb * rv;
      const double wb = s.P[b] - K * vb;
#pragma unroll 2
      for (int a = tid / n; a < n; a += step) {
        const double ha = A[j * L + o + a];
        const double pa = s.P[a];
        double* x = A + (o + a) * L + o + b;
        const double old = *x;
        const double va = a == 0 ? 1.0 : ha * rv;
        const double nv = old - (va * wb + (pa - K * va) * vb);
        *x = nv;
        if (a == 0 && b >= 2) sq += nv * nv;
      }
    }
    sq = wsum(sq);
    if (lane == 0) s.red2[wave] = sq;
    __syncthreads();
  }
  if (tid == 0) {
    if (L >= 2) {
      s.d[L - 2] = A[(L - 2) * L + L - 2];
      s.e[L - 2] = A[(L - 2) * L + L - 1];
    }
    s.d[L - 1] = A[(L - 1) * L + L - 1];
    s.e[L - 1] = 0.0;
  }
  __syncthreads();

  // ---- 2. eigenvalues by multisection ------------------------------------
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

  // ---- 3. eigenvectors of T ---------------------------------------------
  double* Z = A;                       // L x k
  double* C = A + (size_t)L * k;       // k x k
  double* Uf = C + (size_t)k * k;      // 3 x L x nb rows of U for a batch
  for (int t = tid; t < L * k; t += kTT) {
    const int i = t / k, j = t % k;
    const uint64_t h = mix64(((uint64_t)(j + 1) << 32) ^ (uint64_t)i);
    Z[t] = (double)(h >> 11) * 0x1.0p-53 - 0.5;
  }
  __syncthreads();
  for (int j0 = 0; j0 < k; j0 += nb) {
    const int j = j0 + tid;
    if (tid < nb && j < k)
      invit_column(L, k, j, s.d, s.e, s.lam[j], tn, Z, Uf + 3 * tid, 3 * nb);
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
  // reflector data back into LDS (row j, columns j+1 ..)
  for (int j = 0; j + 2 < L; ++j)
    for (int t = tid; t < L - j - 1; t += kTT)
      A[j * L + j + 1 + t] = hh[(int64_t)j * L + j + 1 + t];
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
      const double rv = s.hr[j];
      double v[kVecRegs];
      double dot = 0.0;
#pragma unroll
      for (int q = 0; q < kVecRegs; ++q) {
        const int i = vlane + kVecLanes * q;
        const double h = A[j * L + min(i, L - 1)];
        v[q] = i == j + 1 ? 1.0 : (i > j + 1 && i < L ? h * rv : 0.0);
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

void launch_tri_topk(int L, const double* G, int64_t ldg, int k, double* S, double* D,
                     double* W, int64_t ldw, double* hh, size_t lds_bytes,
                     hipStream_t st) {
  const int nb = tri_batch(L, k, lds_bytes);
  hipLaunchKernelGGL(tri_topk_kernel, dim3(1), dim3(kTT), tri_lds_bytes(L, k, nb), st, L,
                     G, ldg, k, S, D, W, ldw, hh, nb);
  MC_CHECK_LAUNCH();
}

}  // namespace mcsvt
