// Allocation-free Gram product: mc_k_gram_noalloc (include/mcsvt_kernels.h).
//
// The split partial sums of the matrix-core Gram live in a file-scope device
// array instead of a buffer the library allocates.  Host code never passes
// that array's name to a kernel or a copy: it takes the array's device
// address with hipGetSymbolAddress, once per device, and passes that.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mcsvt_kernels.h"
#include "kernels.hpp"

namespace {

// 16 MiB of FP64 partial sums per device, held until the process ends
constexpr int64_t kScratchDoubles = int64_t(1) << 21;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there, with that device current).
double* scratch_on_current_device() {
  int dev = -1;
  MC_HIP(hipGetDevice(&dev));
  MC_REQUIRE(dev >= 0 && dev < kMaxDevices, mcsvt::kEDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw mcsvt::Error(mcsvt::kEDEVICE,
                         std::string("hipGetSymbolAddress(scratch) failed: ") +
                             hipGetErrorString(e));
    g_addr[dev] = static_cast<double*>(p);
  }
  return g_addr[dev];
}

}  // namespace

extern "C" mc_status mc_k_gram_noalloc(int64_t N, int32_t p, int32_t q, const double* A,
                                       int64_t lda, const double* B, int64_t ldb,
                                       int32_t sym, void* stream, double* C,
                                       int64_t ldc) {
  try {
    MC_REQUIRE(N >= 1 && p >= 1 && q >= 1 && A && C && (sym || B), mcsvt::kEINVAL,
               "bad sizes or NULL argument");
    MC_REQUIRE(!sym || p == q, mcsvt::kEINVAL, "sym needs p == q");
    MC_REQUIRE(lda >= p && ldc >= q && (sym || ldb >= q), mcsvt::kEINVAL,
               "leading dimension smaller than the row width");
    MC_REQUIRE((int64_t)p * q <= kScratchDoubles, mcsvt::kERANGE,
               "p * q exceeds the 2^21 doubles (16 MiB) of the allocation-free "
               "scratch array");
    double* part = scratch_on_current_device();
    const double* pB = sym ? A : B;
    const int64_t ldB = sym ? lda : ldb;
    // the split count shrinks until the partials fit the array; every partial
    // element the reduction reads is written first, so nothing is cleared
    mcsvt::launch_gram<double, double>(N, p, q, A, lda, pB, ldB, C, ldc, sym, part,
                                       kScratchDoubles, (hipStream_t)stream);
    return MC_OK;
  } catch (const mcsvt::Error& e) {
    mcsvt_set_thread_error(e.what());
    return (mc_status)e.status;
  } catch (const std::exception& e) {
    mcsvt_set_thread_error(e.what());
    return MC_EDEVICE;
  }
}
