// Symmetric eigensolver for the small Gram matrix of eigSVD (Alg. 3),
// and the top-k selection of Alg. 5.
//
// Two-sided block Jacobi in FP64.  The L x L matrix is padded to Lp (a
// multiple of 32) with a decoupled negative diagonal and cut into nb = Lp/16
// blocks.  A sweep visits all block pairs by the round-robin ("circle")
// ordering: nb - 1 rounds of nb/2 disjoint pairs.  In a round,
//   1. each pair's 32 x 32 principal submatrix is diagonalised in LDS by
//      cyclic Jacobi (one workgroup per pair), giving an orthogonal J;
//   2. every 32 x 32 tile (I, K) of A is replaced by J_I^T A_IK J_K and every
//      row tile of V by V_{:,K} J_K (tiles are disjoint, so in place).
// A rotation is applied only when |a_pq| > max(tol_rel sqrt(|a_pp a_qq|),
// tol_abs); the solve stops after a sweep in which no rotation was applied.
#include "kernels.hpp"

namespace mcsvt {

namespace {

constexpr int BS = 16;        // block size
constexpr int SP = 2 * BS;    // subproblem size (32)

__device__ __forceinline__ void pair_of(int nb, int r, int t, int& bi, int& bj) {
  // circle method: position 0 fixed, the others rotate by r
  auto pos = [&](int j) { return j == 0 ? 0 : 1 + ((j - 1 + r) % (nb - 1)); };
  bi = pos(t);
  bj = pos(nb - 1 - t);
  if (bi > bj) { int x = bi; bi = bj; bj = x; }
}

__device__ __forceinline__ void inner_pair(int rr, int t, int& p, int& q) {
  auto pos = [&](int j) { return j == 0 ? 0 : 1 + ((j - 1 + rr) % (SP - 1)); };
  p = pos(t);
  q = pos(SP - 1 - t);
  if (p > q) { const int x = p; p = q; q = x; }
}

__device__ __forceinline__ int sub_index(int bi, int bj, int a) {
  return a < BS ? bi * BS + a : bj * BS + (a - BS);
}

// Whole eigenproblem in one workgroup (L <= single-workgroup limit).
// Cyclic Jacobi with the round-robin ordering of all L indices (a dummy index
// pads odd L) on the upper triangle of A in LDS.  A round: (1) the rotations
// of its L/2 disjoint pairs are computed and logged (c, s) to global memory,
// (2) every 2 x 2 block (pair i rows, pair j columns, i <= j) of A is
// replaced by R_i^T A_ij R_j in place, the diagonal blocks set exactly to
// diag(a_pp - t a_pq, a_qq + t a_pq).  After convergence the eigenvalues are
// ranked, and the eigenvectors of the k largest are formed by applying the
// logged rounds in reverse order to the k unit vectors e_j (V = R_1 ... R_N,
// so V e_j = R_1 (... (R_N e_j))): only k columns are ever rotated.
constexpr int kSingleMaxPairs = 96;
constexpr int kSingleThreads = 512;
constexpr int kSingleMaxSweeps = 40;

__device__ __forceinline__ int rr_pos(int j, int rr, int n2) {
  if (j == 0) return 0;
  int x = j - 1 + rr;            // < 2 (n2 - 1)
  if (x >= n2 - 1) x -= n2 - 1;
  return 1 + x;
}

// Tiny eigenproblems (L <= kTinyL) in one wavefront: cyclic Jacobi with the
// round-robin ordering of the L indices (a dummy pads odd L), A and the
// eigenvector matrix V in LDS.  A round computes the rotations of its
// disjoint pairs, then applies them to the rows of A, then to the columns of
// A and V (A <- J^T A J, V <- V J).  One wavefront's LDS operations complete
// in order, so the rounds need wavefront fences, not barriers.  A rotation is
// applied only when |a_pq| > max(4e-15 sqrt(|a_pp a_qq|), 1e-14 ||G||_F);
// the solve stops after a sweep without rotations (at most 40 sweeps).
constexpr int kTinyL = 16;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64) void jac_tiny_kernel(
    int L, const double* __restrict__ G, int64_t ldg, int k, double* __restrict__ S_out,
    double* __restrict__ D_out, double* __restrict__ W_out, int64_t ldw) {
  __shared__ double A[kTinyL][kTinyL + 1];
  __shared__ double V[kTinyL][kTinyL + 1];
  __shared__ double Cs[kTinyL / 2], Sn[kTinyL / 2];
  __shared__ int Pp[kTinyL / 2], Qq[kTinyL / 2], idx[kTinyL];
  const int lane = threadIdx.x;
  double f2 = 0.0;
  for (int t = lane; t < L * L; t += 64) {
    const int i = t / L, j = t % L;
    const double g = G[(int64_t)i * ldg + j];
    A[i][j] = g;
    V[i][j] = i == j ? 1.0 : 0.0;
    f2 += g * g;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) f2 += __shfl_xor(f2, o, 64);
  const double tol_abs = 1e-14 * sqrt(f2);
  wave_sync();
  const int n2 = L + (L & 1), np = n2 / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rotated = false;
    for (int rr = 0; rr < n2 - 1; ++rr) {
      double c = 1.0, sn = 0.0;
      if (lane < np) {
        int p = rr_pos(lane, rr, n2), q = rr_pos(n2 - 1 - lane, rr, n2);
        if (p > q) { const int x = p; p = q; q = x; }
        if (q < L) {
          const double app = A[p][p], aqq = A[q][q], apq = A[p][q];
          if (fabs(apq) > fmax(4e-15 * sqrt(fabs(app * aqq)), tol_abs)) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
          }
        }
        Cs[lane] = c;
        Sn[lane] = sn;
        Pp[lane] = p;
        Qq[lane] = q;
      }
      const bool any = __any(sn != 0.0);
      wave_sync();
      if (!any) continue;                      // uniform
      rotated = true;
      for (int t = lane; t < np * L; t += 64) {  // rows p, q of A
        const int i = t / L, j = t % L;
        const int p = Pp[i], q = Qq[i];
        const double ci = Cs[i], si = Sn[i];
        if (q < L && si != 0.0) {
          const double ap = A[p][j], aq = A[q][j];
          A[p][j] = ci * ap - si * aq;
          A[q][j] = si * ap + ci * aq;
        }
      }
      wave_sync();
      for (int t = lane; t < np * L; t += 64) {  // columns p, q of A and V
        const int i = t / L, j = t % L;
        const int p = Pp[i], q = Qq[i];
        const double ci = Cs[i], si = Sn[i];
        if (q < L && si != 0.0) {
          const double ap = A[j][p], aq = A[j][q];
          A[j][p] = ci * ap - si * aq;
          A[j][q] = si * ap + ci * aq;
          const double vp = V[j][p], vq = V[j][q];
          V[j][p] = ci * vp - si * vq;
          V[j][q] = si * vp + ci * vq;
        }
      }
      wave_sync();
    }
    if (!rotated) break;
  }
  // the k largest: rank by (value descending, index ascending)
  if (lane < L) {
    const double dj = A[lane][lane];
    int rank = 0;
    for (int i = 0; i < L; ++i) rank += (A[i][i] > dj) || (A[i][i] == dj && i < lane);
    if (rank < k) {
      idx[rank] = lane;
      if (D_out) D_out[rank] = dj;
      S_out[rank] = sqrt(fmax(dj, 0.0));
    }
  }
  wave_sync();
  for (int t = lane; t < L * k; t += 64) {
    const int i = t / k, c = t % k;
    W_out[(int64_t)i * ldw + c] = V[i][idx[c]];
  }
}

__global__ __launch_bounds__(kSingleThreads) void jac_topk_kernel(
    int L, const double* __restrict__ G, int64_t ldg, int k,
    double* __restrict__ S_out, double* __restrict__ D_out,
    double* __restrict__ W_out, int64_t ldw, double2* __restrict__ cs_log,
    int* __restrict__ rr_log, double tol_rel, double tol_abs_fac,
    int* __restrict__ sweeps_out) {
  extern __shared__ double lds[];
  const int ld = L + 1;
  double* A = lds;                 // upper triangle: A[min * ld + max]
  __shared__ int P[kSingleMaxPairs], Q[kSingleMaxPairs];
  __shared__ double Cc[kSingleMaxPairs], Ss[kSingleMaxPairs];
  __shared__ double D0[kSingleMaxPairs], D1[kSingleMaxPairs];
  __shared__ double red[kSingleThreads];
  __shared__ double dsh[2 * kSingleMaxPairs];
  __shared__ int idx[2 * kSingleMaxPairs];
  const int tid = threadIdx.x;
  const int tx = tid % 32, ty = tid / 32;          // 32 x 16 thread grid
  const int n2 = L + (L & 1);
  const int np = n2 / 2;
  double ss = 0.0;
  for (int t = tid; t < L * L; t += kSingleThreads) {
    const int i = t / L, j = t % L;
    if (i > j) continue;
    const double a = (i == j) ? G[(int64_t)i * ldg + i]
                              : 0.5 * (G[(int64_t)i * ldg + j] + G[(int64_t)j * ldg + i]);
    A[i * ld + j] = a;
    ss += (i == j) ? a * a : 2.0 * a * a;
  }
  red[tid] = ss;
  __syncthreads();
  for (int w = kSingleThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double tol_abs = tol_abs_fac * sqrt(red[0]);
  const double tol_abs2 = tol_abs * tol_abs, tol_rel2 = tol_rel * tol_rel;
  int nlog = 0, sweep = 0;
  for (; sweep < kSingleMaxSweeps; ++sweep) {
    int swept = 0;
    for (int rr = 0; rr < n2 - 1; ++rr) {
      int mine = 0;
      if (tid < np) {
        int p = rr_pos(tid, rr, n2), q = rr_pos(n2 - 1 - tid, rr, n2);
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0, d0 = 0.0, d1 = 0.0;
        if (q < L) {
          const double apq = A[p * ld + q], app = A[p * ld + p], aqq = A[q * ld + q];
          if (apq * apq > fmax(tol_rel2 * fabs(app * aqq), tol_abs2)) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double tt =
                (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            d0 = app - tt * apq;
            d1 = aqq + tt * apq;
            mine = 1;
          }
        }
        P[tid] = p;
        Q[tid] = q;
        Cc[tid] = c;
        Ss[tid] = s;
        D0[tid] = d0;
        D1[tid] = d1;
        cs_log[(int64_t)nlog * np + tid] = make_double2(c, s);
      }
      if (!__syncthreads_or(mine)) continue;
      swept = 1;
      if (tid == 0) rr_log[nlog] = rr;
      ++nlog;
      for (int ti = ty; ti < np; ti += kSingleThreads / 32) {
        const int p1 = P[ti], q1 = Q[ti];
        const double c1 = Cc[ti], s1 = Ss[ti];
        for (int tj = tx; tj < np; tj += 32) {
          if (tj < ti) continue;
          const double s2 = Ss[tj];
          if (s1 == 0.0 && s2 == 0.0) continue;
          if (ti == tj) {
            A[p1 * ld + p1] = D0[ti];
            A[q1 * ld + q1] = D1[ti];
            A[p1 * ld + q1] = 0.0;
            continue;
          }
          const int p2 = P[tj], q2 = Q[tj];
          const double c2 = Cc[tj];
          const bool vq1 = q1 < L, vq2 = q2 < L;
          // upper-triangle addresses of the four entries
          const int ia = p1 < p2 ? p1 * ld + p2 : p2 * ld + p1;
          const int ib = p1 < q2 ? p1 * ld + q2 : q2 * ld + p1;
          const int ic = q1 < p2 ? q1 * ld + p2 : p2 * ld + q1;
          const int id = q1 < q2 ? q1 * ld + q2 : q2 * ld + q1;
          double a = A[ia];
          double b = vq2 ? A[ib] : 0.0;
          double c = vq1 ? A[ic] : 0.0;
          double d = (vq1 && vq2) ? A[id] : 0.0;
          const double a1 = c1 * a - s1 * c, b1 = c1 * b - s1 * d;
          const double c1r = s1 * a + c1 * c, d1r = s1 * b + c1 * d;
          A[ia] = c2 * a1 - s2 * b1;
          if (vq2) A[ib] = s2 * a1 + c2 * b1;
          if (vq1) A[ic] = c2 * c1r - s2 * d1r;
          if (vq1 && vq2) A[id] = s2 * c1r + c2 * d1r;
        }
      }
      __syncthreads();
    }
    if (!swept) break;
  }
  if (tid == 0 && sweeps_out) *sweeps_out = sweep + 1;
  // eigenvalues: rank by (value descending, index ascending)
  for (int j = tid; j < L; j += kSingleThreads) dsh[j] = A[j * ld + j];
  __syncthreads();
  for (int j = tid; j < L; j += kSingleThreads) {
    const double dj = dsh[j];
    int rank = 0;
    for (int i = 0; i < L; ++i) rank += (dsh[i] > dj) || (dsh[i] == dj && i < j);
    if (D_out) D_out[rank] = dj;
    if (rank < k) {
      idx[rank] = j;
      S_out[rank] = sqrt(fmax(dj, 0.0));
    }
  }
  __syncthreads();
  // eigenvectors of the k largest: replay the logged rounds in reverse on
  // Z = [e_idx[0] .. e_idx[k-1]] (L x k, row stride k, in A's space)
  double* Z = lds;
  for (int t = tid; t < L * k; t += kSingleThreads) {
    const int i = t / k, c = t % k;
    Z[t] = (i == idx[c]) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int r = nlog - 1; r >= 0; --r) {
    const int rr = rr_log[r];
    const double2* cs = cs_log + (int64_t)r * np;
    for (int t = ty; t < np; t += kSingleThreads / 32) {
      const double2 v = cs[t];
      if (v.y == 0.0) continue;
      int p = rr_pos(t, rr, n2), q = rr_pos(n2 - 1 - t, rr, n2);
      if (p > q) { const int x = p; p = q; q = x; }
      for (int c = tx; c < k; c += 32) {
        const double zp = Z[p * k + c], zq = Z[q * k + c];
        Z[p * k + c] = v.x * zp + v.y * zq;
        Z[q * k + c] = -v.y * zp + v.x * zq;
      }
    }
    __syncthreads();
  }
  for (int t = tid; t < L * k; t += kSingleThreads)
    W_out[(int64_t)(t / k) * ldw + (t % k)] = Z[t];
}

__global__ void jac_init_kernel(int L, int Lp, const double* __restrict__ G,
                                int64_t ldg, double* __restrict__ A,
                                double* __restrict__ V, double pad) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)Lp * Lp) return;
  const int i = (int)(t / Lp), j = (int)(t % Lp);
  double a;
  if (i < L && j < L) {
    // symmetrise exactly
    const double x = G[(int64_t)i * ldg + j], y = G[(int64_t)j * ldg + i];
    a = (i == j) ? x : 0.5 * (x + y);
  } else {
    a = (i == j) ? pad : 0.0;
  }
  A[t] = a;
  V[t] = (i == j) ? 1.0 : 0.0;
}

// One workgroup (256 threads = 16 x 16 over the 16 x 16 pair blocks) per
// block pair: cyclic Jacobi on the 32 x 32 principal submatrix in LDS, two
// phases per round as in the one-workgroup solver; J accumulates the
// rotations.
__global__ __launch_bounds__(256) void jac_solve_kernel(
    int Lp, int nb, int round, double* __restrict__ A,
    double* __restrict__ Jbuf, double* __restrict__ Sbuf,
    int* __restrict__ rot_flag, double tol_rel, double tol_abs) {
  __shared__ double S[SP][SP + 1];
  __shared__ double J[SP][SP + 1];
  __shared__ int P[SP / 2], Q[SP / 2];
  __shared__ double Cc[SP / 2], Ss[SP / 2], D0[SP / 2], D1[SP / 2];
  const int pair = blockIdx.x;
  int bi, bj;
  pair_of(nb, round, pair, bi, bj);
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  for (int t = tid; t < SP * SP; t += 256) {
    const int a = t / SP, b = t % SP;
    S[a][b] = A[(int64_t)sub_index(bi, bj, a) * Lp + sub_index(bi, bj, b)];
    J[a][b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  int any = 0;
  for (int sweep = 0; sweep < 20; ++sweep) {
    int swept = 0;
    for (int rr = 0; rr < SP - 1; ++rr) {
      int mine = 0;
      if (tid < SP / 2) {
        int p, q;
        inner_pair(rr, tid, p, q);
        const double apq = S[p][q], app = S[p][p], aqq = S[q][q];
        double c = 1.0, s = 0.0, d0 = 0.0, d1 = 0.0;
        if (fabs(apq) > fmax(tol_rel * sqrt(fabs(app * aqq)), tol_abs)) {
          const double theta = (aqq - app) / (2.0 * apq);
          const double tt =
              (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          d0 = app - tt * apq;
          d1 = aqq + tt * apq;
          mine = 1;
        }
        P[tid] = p;
        Q[tid] = q;
        Cc[tid] = c;
        Ss[tid] = s;
        D0[tid] = d0;
        D1[tid] = d1;
      }
      if (!__syncthreads_or(mine)) continue;
      swept = 1;
      {
        const int ti = ty, tj = tx;      // one 2 x 2 block of S per thread
        const double s1 = Ss[ti], s2 = Ss[tj];
        if (tj >= ti && (s1 != 0.0 || s2 != 0.0)) {
          const int p1 = P[ti], q1 = Q[ti];
          if (ti == tj) {
            S[p1][p1] = D0[ti];
            S[q1][q1] = D1[ti];
            S[p1][q1] = 0.0;
            S[q1][p1] = 0.0;
          } else {
            const int p2 = P[tj], q2 = Q[tj];
            const double c1 = Cc[ti], c2 = Cc[tj];
            double a = S[p1][p2], b = S[p1][q2], c = S[q1][p2], d = S[q1][q2];
            const double a1 = c1 * a - s1 * c, b1 = c1 * b - s1 * d;
            const double c1r = s1 * a + c1 * c, d1r = s1 * b + c1 * d;
            a = c2 * a1 - s2 * b1;
            b = s2 * a1 + c2 * b1;
            c = c2 * c1r - s2 * d1r;
            d = s2 * c1r + c2 * d1r;
            S[p1][p2] = a; S[p2][p1] = a;
            S[p1][q2] = b; S[q2][p1] = b;
            S[q1][p2] = c; S[p2][q1] = c;
            S[q1][q2] = d; S[q2][q1] = d;
          }
        }
      }
      for (int w = tid; w < SP * (SP / 2); w += 256) {   // J <- J R
        const int j = w / (SP / 2), t = w % (SP / 2);
        const double s = Ss[t];
        if (s != 0.0) {
          const int p = P[t], q = Q[t];
          const double c = Cc[t];
          const double a = J[j][p], b = J[j][q];
          J[j][p] = c * a - s * b;
          J[j][q] = s * a + c * b;
        }
      }
      __syncthreads();
    }
    any |= swept;
    if (!swept) break;
  }
  double* Jo = Jbuf + (int64_t)pair * SP * SP;
  double* So = Sbuf + (int64_t)pair * SP * SP;
  for (int t = tid; t < SP * SP; t += 256) {
    const int a = t / SP, b = t % SP;
    Jo[t] = J[a][b];
    So[t] = S[a][b];
  }
  if (tid == 0 && any) atomicAdd(rot_flag, 1);
}

// grid.x = npair * npair (upper tiles only used), grid.y = 0: A tiles;
// a second launch handles V.
__global__ __launch_bounds__(256) void jac_apply_a_kernel(
    int Lp, int nb, int round, double* __restrict__ A,
    const double* __restrict__ Jbuf, const double* __restrict__ Sbuf,
    const int* __restrict__ rot_flag) {
  const int npair = nb / 2;
  const int I = blockIdx.x % npair, K = blockIdx.x / npair;
  if (I > K) return;
  if (*rot_flag == 0) return;   // nothing rotated in this round so far
  if (I == K) {
    // the pair's own block: the subproblem solver's (symmetrised) result
    int ai, aj;
    pair_of(nb, round, I, ai, aj);
    const double* Sg = Sbuf + (int64_t)I * SP * SP;
    for (int t = threadIdx.x; t < SP * SP; t += 256) {
      const int a = t / SP, b = t % SP;
      A[(int64_t)sub_index(ai, aj, a) * Lp + sub_index(ai, aj, b)] = Sg[t];
    }
    return;
  }
  __shared__ double T[SP][SP + 1];
  __shared__ double U[SP][SP + 1];
  __shared__ double JI[SP][SP + 1];
  __shared__ double JK[SP][SP + 1];
  int ai, aj, ki, kj;
  pair_of(nb, round, I, ai, aj);
  pair_of(nb, round, K, ki, kj);
  const double* JIg = Jbuf + (int64_t)I * SP * SP;
  const double* JKg = Jbuf + (int64_t)K * SP * SP;
  for (int t = threadIdx.x; t < SP * SP; t += 256) {
    const int a = t / SP, b = t % SP;
    T[a][b] = A[(int64_t)sub_index(ai, aj, a) * Lp + sub_index(ki, kj, b)];
    JI[a][b] = JIg[t];
    JK[a][b] = JKg[t];
  }
  __syncthreads();
  // U = T JK
  for (int t = threadIdx.x; t < SP * SP; t += 256) {
    const int a = t / SP, b = t % SP;
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < SP; ++c) s += T[a][c] * JK[c][b];
    U[a][b] = s;
  }
  __syncthreads();
  // T = JI^T U
  for (int t = threadIdx.x; t < SP * SP; t += 256) {
    const int a = t / SP, b = t % SP;
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < SP; ++c) s += JI[c][a] * U[c][b];
    T[a][b] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SP * SP; t += 256) {
    const int a = t / SP, b = t % SP;
    const int gi = sub_index(ai, aj, a), gj = sub_index(ki, kj, b);
    A[(int64_t)gi * Lp + gj] = T[a][b];
    A[(int64_t)gj * Lp + gi] = T[a][b];
  }
}

// V[r0:r0+32, K-cols] = V[r0:r0+32, K-cols] J_K
__global__ __launch_bounds__(256) void jac_apply_v_kernel(
    int Lp, int nb, int round, double* __restrict__ V,
    const double* __restrict__ Jbuf, const int* __restrict__ rot_flag) {
  if (*rot_flag == 0) return;
  const int K = blockIdx.y;
  const int r0 = blockIdx.x * SP;
  __shared__ double T[SP][SP + 1];
  __shared__ double JK[SP][SP + 1];
  int ki, kj;
  pair_of(nb, round, K, ki, kj);
  const double* JKg = Jbuf + (int64_t)K * SP * SP;
  for (int t = threadIdx.x; t < SP * SP; t += 256) {
    const int a = t / SP, b = t % SP;
    T[a][b] = V[(int64_t)(r0 + a) * Lp + sub_index(ki, kj, b)];
    JK[a][b] = JKg[t];
  }
  __syncthreads();
  double out[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int t = threadIdx.x + u * 256;
    const int a = t / SP, b = t % SP;
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < SP; ++c) s += T[a][c] * JK[c][b];
    out[u] = s;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int t = threadIdx.x + u * 256;
    const int a = t / SP, b = t % SP;
    V[(int64_t)(r0 + a) * Lp + sub_index(ki, kj, b)] = out[u];
  }
}

__global__ void frob_kernel(int L, const double* __restrict__ G, int64_t ldg,
                            double* __restrict__ out) {
  __shared__ double sh[1024];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < (int64_t)L * L; t += 1024) {
    const double v = G[(t / L) * ldg + (t % L)];
    acc += v * v;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(sh[0]);
}

// top-k of the L eigenvalues (descending): S = sqrt(max(d, 0)),
// Wk (L x k, row-major) = the matching eigenvectors.
__global__ void select_topk_kernel(int L, int Lp, int k,
                                   const double* __restrict__ A,
                                   const double* __restrict__ V,
                                   double* __restrict__ S, double* __restrict__ D,
                                   double* __restrict__ Wk, int64_t ldw) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
  const double dj = A[(int64_t)j * Lp + j];
  int rank = 0;
  for (int i = 0; i < L; ++i) {
    const double di = A[(int64_t)i * Lp + i];
    rank += (di > dj) || (di == dj && i < j);
  }
  if (D) D[rank] = dj;
  if (rank >= k) return;
  S[rank] = sqrt(fmax(dj, 0.0));
  for (int i = 0; i < L; ++i) Wk[(int64_t)i * ldw + rank] = V[(int64_t)i * Lp + j];
}

}  // namespace

void EigSolver::reserve(int L, hipStream_t st) {
  const int Lp = (int)round_up(std::max(L, 1), SP);   // >= L for both paths
  const int nb = Lp / BS;
  A.reserve((size_t)Lp * Lp, st);
  V.reserve((size_t)Lp * Lp, st);
  J.reserve((size_t)(nb / 2) * SP * SP, st);
  Sd.reserve((size_t)(nb / 2) * SP * SP, st);
  {
    // rotation log of the one-workgroup solver: every round of every sweep
    const int n2 = L + (L & 1);
    const size_t rounds = (size_t)kSingleMaxSweeps * std::max(n2 - 1, 1);
    cslog.reserve(2 * rounds * std::max(n2 / 2, 1), st);
    rrlog.reserve(rounds, st);
  }
  flags.reserve(kMaxSweeps * 64 + 8, st);
  scal.reserve(4, st);
  // tridiagonal path: reflector rows (allocated here, outside any stream
  // capture)
  hh.reserve((size_t)L * L, st);
  {
    // the multi-launch path serves every width up to tri_big_max()
    const int Lb = std::min(L, tri_big_max());
    big.reserve(TriBigWork::doubles(Lb, std::min(Lb, tri_big_kmax())), st);
  }
  if (!hflags) MC_HIP(hipHostMalloc((void**)&hflags, sizeof(int) * 64));
}

EigSolver::~EigSolver() {
  if (hflags) (void)hipHostFree(hflags);
}

namespace {
constexpr size_t kStaticLdsReserve = 12288;   // static LDS of jac_topk_kernel

// Largest dynamic LDS one workgroup may use (queried once; gfx950 allows more
// than the 64 KB default once the kernel attribute is raised).
size_t query_lds_limit() {
  int dev = 0, v = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) !=
          hipSuccess || v <= 0) {
    (void)hipGetLastError();
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
        hipSuccess) {
      (void)hipGetLastError();
      v = 65536;
    }
  }
  size_t lim = (size_t)v;
  tri_set_lds_attributes(lim);
  if (hipFuncSetAttribute((const void*)jac_topk_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(lim - kStaticLdsReserve)) != hipSuccess ||
      hipFuncSetAttribute(tri_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lim) != hipSuccess) {
    (void)hipGetLastError();
    lim = 65536;
  }
  return lim;
}

// queried once per process (thread-safe initialisation)
size_t lds_limit() {
  static const size_t lim = query_lds_limit();
  return lim;
}
}  // namespace

int EigSolver::single_max() {
  // dynamic LDS holds A (L x (L + 1)); the kernel's own arrays take the rest
  const size_t lim = lds_limit() - kStaticLdsReserve;
  int L = 1;
  while (L + 1 <= 2 * kSingleMaxPairs &&
         (size_t)(L + 1) * (L + 2) * sizeof(double) <= lim)
    ++L;
  return L;
}

bool EigSolver::device_only(int L, int k) {
  return tri_fits(L, k, lds_limit()) || (L <= tri_big_max() && k <= tri_big_kmax()) ||
         L <= single_max();
}

void EigSolver::solve_topk(int L, const double* G, int64_t ldg, int k, double* S,
                           double* D, double* Wk, int64_t ldw, hipStream_t st) {
  if (L <= kTinyL) {
    hipLaunchKernelGGL(jac_tiny_kernel, dim3(1), dim3(64), 0, st, L, G, ldg, k, S, D, Wk,
                       ldw);
    MC_CHECK_LAUNCH();
    this->L = L;
    this->Lp = L;
    sweeps = 0;      // known on the device only
    return;
  }
  if (tri_fits(L, k, lds_limit())) {
    reserve(L, st);
    this->L = L;
    this->Lp = L;
    launch_tri_topk(L, G, ldg, k, S, D, Wk, ldw, hh.p, lds_limit(), st);
    sweeps = 0;      // no sweeps: a direct method
    return;
  }
  if (L <= tri_big_max() && k <= tri_big_kmax()) {
    reserve(L, st);
    this->L = L;
    this->Lp = L;
    launch_tri_big(L, G, ldg, k, S, D, Wk, ldw, big.p, big.n, lds_limit(), st);
    sweeps = 0;
    return;
  }
  if (L <= single_max()) {
    reserve(L, st);
    this->L = L;
    this->Lp = L;
    const size_t bytes = (size_t)L * (L + 1) * sizeof(double);
    hipLaunchKernelGGL(jac_topk_kernel, dim3(1), dim3(kSingleThreads), bytes, st, L,
                       G, ldg, k, S, D, Wk, ldw, (double2*)cslog.p, rrlog.p,
                       4e-15, 1e-14, flags.p);
    MC_CHECK_LAUNCH();
    sweeps = -1;     // known on the device only
    return;
  }
  solve(L, G, ldg, st);
  select_topk(k, S, D, Wk, ldw, st);
}

int EigSolver::solve(int L, const double* G, int64_t ldg, hipStream_t st) {
  reserve(L, st);
  // rotations below ~LAPACK-level accuracy (1e-14 ||G||_F) resolve only the
  // round-off of the Gram product itself
  const double tol_rel = 4e-15;
  const double tol_abs_fac = 1e-14;
  this->L = L;
  const int Lp = (int)round_up(std::max(L, 1), SP);
  const int nb = Lp / BS;
  const int npair = nb / 2;
  this->Lp = Lp;
  hipLaunchKernelGGL(frob_kernel, dim3(1), dim3(1024), 0, st, L, G, ldg, scal.p);
  MC_CHECK_LAUNCH();
  double hnorm = 0.0;
  MC_HIP(hipMemcpyAsync(&hnorm, scal.p, sizeof(double), hipMemcpyDeviceToHost, st));
  MC_HIP(hipStreamSynchronize(st));
  const double tol_abs = tol_abs_fac * hnorm;
  const int64_t tot = (int64_t)Lp * Lp;
  const double pad = -(1.0 + 2.0 * hnorm);
  hipLaunchKernelGGL(jac_init_kernel, dim3((unsigned)ceil_div(tot, 256)),
                     dim3(256), 0, st, L, Lp, G, ldg, A.p, V.p, pad);
  MC_CHECK_LAUNCH();
  const int rounds = nb - 1;
  MC_HIP(hipMemsetAsync(flags.p, 0, sizeof(int) * (kMaxSweeps * 64 + 8), st));
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    int* sflag = flags.p + sweep * 64;
    for (int r = 0; r < rounds; ++r) {
      // counts the pairs that rotated in this round of this sweep
      int* rflag = sflag + 1 + (r % 63);
      hipLaunchKernelGGL(jac_solve_kernel, dim3(npair), dim3(256), 0, st, Lp, nb,
                         r, A.p, J.p, Sd.p, rflag, tol_rel, tol_abs);
      MC_CHECK_LAUNCH();
      hipLaunchKernelGGL(jac_apply_a_kernel, dim3(npair * npair), dim3(256), 0,
                         st, Lp, nb, r, A.p, J.p, Sd.p, rflag);
      MC_CHECK_LAUNCH();
      hipLaunchKernelGGL(jac_apply_v_kernel, dim3(Lp / SP, npair), dim3(256), 0,
                         st, Lp, nb, r, V.p, J.p, rflag);
      MC_CHECK_LAUNCH();
    }
    if (sweep >= 1 || nb == 2) {
      MC_HIP(hipMemcpyAsync(hflags, sflag, sizeof(int) * 64, hipMemcpyDeviceToHost, st));
      MC_HIP(hipStreamSynchronize(st));
      int tot_rot = 0;
      for (int r = 0; r < std::min(rounds, 63); ++r) tot_rot += hflags[1 + r];
      if (tot_rot == 0) { ++sweep; break; }
      if (nb == 2) { ++sweep; break; }   // one exact solve diagonalises it
    }
  }
  sweeps = sweep;
  return sweep;
}

int EigSolver::device_sweeps(hipStream_t st) {
  if (sweeps >= 0) return sweeps;
  MC_HIP(hipMemcpyAsync(hflags, flags.p, sizeof(int), hipMemcpyDeviceToHost, st));
  MC_HIP(hipStreamSynchronize(st));
  return hflags[0];
}

void EigSolver::select_topk(int k, double* S, double* D, double* Wk, int64_t ldw,
                            hipStream_t st) {
  hipLaunchKernelGGL(select_topk_kernel, dim3((unsigned)ceil_div(L, 128)),
                     dim3(128), 0, st, L, Lp, k, A.p, V.p, S, D, Wk, ldw);
  MC_CHECK_LAUNCH();
}

}  // namespace mcsvt
