// Shared host/device utilities of the mcsvt library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace mcsvt {

// Status codes mirror mc_status in include/mcsvt.h.
enum Status : int {
  kOK = 0, kEINVAL = 1, kEDUP = 2, kERANGE = 3, kENOMEM = 4, kEDEVICE = 5,
  kENUMERIC = 6, kEDONE = 7, kENOTCONV = 8
};

struct Error : std::runtime_error {
  int status;
  Error(int st, const std::string& msg) : std::runtime_error(msg), status(st) {}
};

[[noreturn]] void throw_hip(hipError_t e, const char* expr, const char* file,
                            int line);

#define MC_HIP(expr)                                                   \
  do {                                                                 \
    hipError_t mc_e_ = (expr);                                         \
    if (mc_e_ != hipSuccess) ::mcsvt::throw_hip(mc_e_, #expr, __FILE__, \
                                                __LINE__);             \
  } while (0)

#define MC_CHECK_LAUNCH() MC_HIP(hipGetLastError())

#define MC_REQUIRE(cond, st, msg) \
  do {                            \
    if (!(cond)) throw ::mcsvt::Error((st), (msg)); \
  } while (0)

// thread-local message returned by mc_svt_last_error(NULL)
}  // namespace mcsvt
void mcsvt_set_thread_error(const char* msg);
namespace mcsvt {

// ---- device memory through the (optional) allocator hooks ---------------
void* dev_alloc(size_t bytes, hipStream_t stream);
void dev_free(void* p, size_t bytes, hipStream_t stream);

// Owning device buffer; grows on demand, never shrinks.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t stream = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) dev_free(p, n * sizeof(T), stream);
    p = nullptr;
    n = 0;
  }
  // Ensure capacity for `count` elements (contents are NOT preserved).
  T* reserve(size_t count, hipStream_t s) {
    if (count <= n && p) return p;
    {
      // buffers grow only outside stream capture (callers size them first)
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (s && hipStreamIsCapturing(s, &cs) == hipSuccess &&
          cs != hipStreamCaptureStatusNone)
        throw Error(kEDEVICE, "device buffer growth inside a stream capture");
    }
    release();
    stream = s;
    size_t want = count ? count : 1;
    p = static_cast<T*>(dev_alloc(want * sizeof(T), s));
    n = want;
    return p;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// bfloat16 storage (1 sign, 8 exponent, 7 mantissa bits): the upper half of
// an IEEE binary32; conversion from float rounds to nearest, ties to even.
struct bf16_t {
  uint16_t bits;
  __host__ __device__ bf16_t() : bits(0) {}
  __host__ __device__ explicit bf16_t(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
      bits = (uint16_t)((u >> 16) | 0x0040u);     // quiet NaN
    } else {
      u += 0x7FFFu + ((u >> 16) & 1u);
      bits = (uint16_t)(u >> 16);
    }
  }
  __host__ __device__ explicit bf16_t(double d) : bf16_t((float)d) {}
  __host__ __device__ operator float() const {
    const uint32_t u = (uint32_t)bits << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
  }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Grid size cap for 1-D grid-stride kernels.
constexpr int kMaxGrid = 65535 * 4;

}  // namespace mcsvt
