// Counter-based Gaussian test matrices Omega (Alg. 5, Alg. 1).
//
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): counter c0..c3, key
// k0, k1; a round maps (c0, c1, c2, c3) to
//   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
// with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key is bumped by
// (0x9E3779B9, 0xBB67AE85) between the ten rounds.  Box-Muller turns the two
// 53-bit uniforms of one counter into the two normals of an element pair.
//
// Element e of the row-major (rows x cols) matrix uses pair t = e / 2 with
// counter (t mod 2^32, t div 2^32, step, attempt) and key = seed; the even
// element takes the cosine branch, the odd one the sine branch.
#include "kernels.hpp"

namespace mcsvt {

namespace {

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1,
                                             uint32_t& c2, uint32_t& c3,
                                             uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  c0 = hi1 ^ c1 ^ k0;
  c1 = lo1;
  c2 = hi0 ^ c3 ^ k1;
  c3 = lo0;
}

__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo) {
  const uint64_t z = (((uint64_t)hi << 32) | lo) >> 11;
  return ((double)z + 0.5) * 0x1.0p-53;
}

template <class T>
__global__ void gaussian_kernel(T* __restrict__ out, int64_t rows, int64_t cols,
                                int64_t ld, uint64_t seed, uint32_t step_arg,
                                uint32_t attempt_arg, const uint32_t* __restrict__ ctr) {
  // (step, attempt) from device memory when given, so a captured graph can
  // be replayed for any call of the stream
  const uint32_t step = ctr ? ctr[0] : step_arg;
  const uint32_t attempt = ctr ? ctr[1] : attempt_arg;
  const int64_t count = rows * cols;
  const int64_t npair = (count + 1) / 2;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < npair;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c0 = (uint32_t)t, c1 = (uint32_t)((uint64_t)t >> 32);
    uint32_t c2 = step, c3 = attempt;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      if (r > 0) {
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
      }
      philox_round(c0, c1, c2, c3, k0, k1);
    }
    const double u1 = unit53(c0, c1);
    const double u2 = unit53(c2, c3);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 2.0 * 3.141592653589793 * u2;
    const int64_t e0 = 2 * t;
    const int64_t e1 = e0 + 1;
    out[(e0 / cols) * ld + (e0 % cols)] = (T)(rad * cos(ang));
    if (e1 < count) out[(e1 / cols) * ld + (e1 % cols)] = (T)(rad * sin(ang));
  }
}

}  // namespace

template <class T>
void launch_gaussian(T* out, int64_t rows, int64_t cols, int64_t ld,
                     uint64_t seed, uint32_t step, uint32_t attempt,
                     hipStream_t st) {
  const int64_t npair = (rows * cols + 1) / 2;
  if (npair == 0) return;
  const int threads = 256;
  const int64_t grid = std::min<int64_t>(ceil_div(npair, threads), kMaxGrid);
  hipLaunchKernelGGL(gaussian_kernel<T>, dim3((unsigned)grid), dim3(threads), 0,
                     st, out, rows, cols, ld, seed, step, attempt, nullptr);
  MC_CHECK_LAUNCH();
}

template <class T>
void launch_gaussian_ctr(T* out, int64_t rows, int64_t cols, int64_t ld,
                         uint64_t seed, const uint32_t* d_ctr, hipStream_t st) {
  const int64_t npair = (rows * cols + 1) / 2;
  if (npair == 0) return;
  const int threads = 256;
  const int64_t grid = std::min<int64_t>(ceil_div(npair, threads), kMaxGrid);
  hipLaunchKernelGGL(gaussian_kernel<T>, dim3((unsigned)grid), dim3(threads), 0,
                     st, out, rows, cols, ld, seed, 0u, 0u, d_ctr);
  MC_CHECK_LAUNCH();
}
template void launch_gaussian_ctr<double>(double*, int64_t, int64_t, int64_t,
                                          uint64_t, const uint32_t*, hipStream_t);
template void launch_gaussian_ctr<float>(float*, int64_t, int64_t, int64_t,
                                         uint64_t, const uint32_t*, hipStream_t);

template void launch_gaussian<double>(double*, int64_t, int64_t, int64_t,
                                      uint64_t, uint32_t, uint32_t, hipStream_t);
template void launch_gaussian<float>(float*, int64_t, int64_t, int64_t,
                                     uint64_t, uint32_t, uint32_t, hipStream_t);

}  // namespace mcsvt
