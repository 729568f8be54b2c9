// Symmetric eigensolver for the small Gram matrix of eigSVD (Alg. 3 step 2),
// and the top-k selection of Alg. 5 steps 9-10.
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

// 64 threads (one wavefront) per pair
__global__ __launch_bounds__(64) void jac_solve_kernel(
    int Lp, int nb, int round, double* __restrict__ A,
    double* __restrict__ Jbuf, double* __restrict__ Sbuf,
    int* __restrict__ rot_flag, double tol_rel, double tol_abs) {
  __shared__ double S[SP][SP + 1];
  __shared__ double J[SP][SP + 1];
  __shared__ double cs[SP / 2][2];
  __shared__ double dnew[SP / 2][2];
  __shared__ int any;
  const int pair = blockIdx.x;
  int bi, bj;
  pair_of(nb, round, pair, bi, bj);
  const int tid = threadIdx.x;
  for (int t = tid; t < SP * SP; t += 64) {
    const int a = t / SP, b = t % SP;
    S[a][b] = A[(int64_t)sub_index(bi, bj, a) * Lp + sub_index(bi, bj, b)];
    J[a][b] = (a == b) ? 1.0 : 0.0;
  }
  if (tid == 0) any = 0;
  __syncthreads();
  for (int sweep = 0; sweep < 20; ++sweep) {
    int swept = 0;
    for (int rr = 0; rr < SP - 1; ++rr) {
      int mine = 0;
      if (tid < SP / 2) {
        const int t = tid;
        int p, q;
        inner_pair(rr, t, p, q);
        const double apq = S[p][q], app = S[p][p], aqq = S[q][q];
        double c = 1.0, s = 0.0, tt = 0.0;
        if (fabs(apq) > fmax(tol_rel * sqrt(fabs(app * aqq)), tol_abs)) {
          const double theta = (aqq - app) / (2.0 * apq);
          tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          mine = 1;
        }
        cs[t][0] = c;
        cs[t][1] = s;
        dnew[t][0] = app - tt * apq;
        dnew[t][1] = aqq + tt * apq;
      }
      const int round_rot = __syncthreads_or(mine);
      if (!round_rot) continue;
      swept = 1;
      // rows: a'_pj = c a_pj - s a_qj ; a'_qj = s a_pj + c a_qj
      for (int w = tid; w < (SP / 2) * SP; w += 64) {
        const int t = w / SP, j = w % SP;
        int p, q;
        inner_pair(rr, t, p, q);
        const double c = cs[t][0], s = cs[t][1];
        if (s != 0.0) {
          const double a = S[p][j], b = S[q][j];
          S[p][j] = c * a - s * b;
          S[q][j] = s * a + c * b;
        }
      }
      __syncthreads();
      // cols of S and J: x'_jp = c x_jp - s x_jq ; x'_jq = s x_jp + c x_jq
      for (int w = tid; w < (SP / 2) * SP; w += 64) {
        const int t = w / SP, j = w % SP;
        int p, q;
        inner_pair(rr, t, p, q);
        const double c = cs[t][0], s = cs[t][1];
        if (s != 0.0) {
          double a = S[j][p], b = S[j][q];
          S[j][p] = c * a - s * b;
          S[j][q] = s * a + c * b;
          a = J[j][p];
          b = J[j][q];
          J[j][p] = c * a - s * b;
          J[j][q] = s * a + c * b;
        }
      }
      __syncthreads();
      if (tid < SP / 2) {
        const int t = tid;
        int p, q;
        inner_pair(rr, t, p, q);
        if (cs[t][1] != 0.0) {
          S[p][q] = 0.0;
          S[q][p] = 0.0;
          S[p][p] = dnew[t][0];
          S[q][q] = dnew[t][1];
        }
      }
      __syncthreads();
    }
    if (swept && tid == 0) any = 1;
    if (!swept) break;
  }
  __syncthreads();
  double* Jo = Jbuf + (int64_t)pair * SP * SP;
  double* So = Sbuf + (int64_t)pair * SP * SP;
  for (int t = tid; t < SP * SP; t += 64) {
    const int a = t / SP, b = t % SP;
    Jo[t] = J[a][b];
    So[t] = (a == b) ? S[a][a] : 0.5 * (S[a][b] + S[b][a]);
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
  const int Lp = (int)round_up(std::max(L, 1), SP);
  const int nb = Lp / BS;
  A.reserve((size_t)Lp * Lp, st);
  V.reserve((size_t)Lp * Lp, st);
  J.reserve((size_t)(nb / 2) * SP * SP, st);
  Sd.reserve((size_t)(nb / 2) * SP * SP, st);
  flags.reserve(kMaxSweeps * 64 + 8, st);
  scal.reserve(4, st);
  if (!hflags) MC_HIP(hipHostMalloc((void**)&hflags, sizeof(int) * 64));
}

EigSolver::~EigSolver() {
  if (hflags) (void)hipHostFree(hflags);
}

int EigSolver::solve(int L, const double* G, int64_t ldg, hipStream_t st) {
  reserve(L, st);
  const int Lp = (int)round_up(std::max(L, 1), SP);
  const int nb = Lp / BS;
  const int npair = nb / 2;
  this->L = L;
  this->Lp = Lp;
  hipLaunchKernelGGL(frob_kernel, dim3(1), dim3(1024), 0, st, L, G, ldg, scal.p);
  MC_CHECK_LAUNCH();
  double hnorm = 0.0;
  MC_HIP(hipMemcpyAsync(&hnorm, scal.p, sizeof(double), hipMemcpyDeviceToHost, st));
  const int64_t tot = (int64_t)Lp * Lp;
  MC_HIP(hipStreamSynchronize(st));
  const double pad = -(1.0 + 2.0 * hnorm);
  hipLaunchKernelGGL(jac_init_kernel, dim3((unsigned)ceil_div(tot, 256)),
                     dim3(256), 0, st, L, Lp, G, ldg, A.p, V.p, pad);
  MC_CHECK_LAUNCH();
  const int rounds = nb - 1;
  MC_HIP(hipMemsetAsync(flags.p, 0, sizeof(int) * (kMaxSweeps * 64 + 8), st));
  const double tol_rel = 4e-15;
  const double tol_abs = 4e-16 * hnorm;
  int sweep = 0;
  for (; sweep < kMaxSweeps; ++sweep) {
    int* sflag = flags.p + sweep * 64;
    for (int r = 0; r < rounds; ++r) {
      int* rflag = sflag + 1 + (r % 63);
      // rflag counts pairs that rotated in this round (shared across sweeps
      // of the same round slot, so offset by sweep)
      hipLaunchKernelGGL(jac_solve_kernel, dim3(npair), dim3(64), 0, st, Lp, nb,
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

void EigSolver::select_topk(int k, double* S, double* D, double* Wk, int64_t ldw,
                            hipStream_t st) {
  hipLaunchKernelGGL(select_topk_kernel, dim3((unsigned)ceil_div(L, 128)),
                     dim3(128), 0, st, L, Lp, k, A.p, V.p, S, D, Wk, ldw);
  MC_CHECK_LAUNCH();
}

}  // namespace mcsvt
