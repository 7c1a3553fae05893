// Shared host/device helpers of the LABFM HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/labfm.h"

namespace labfm {

// Records a thread-local error message (read back by labfm_last_error).
void set_error(const char* fmt, ...);
void clear_error();

// Evaluates a HIP call; on failure records the message and returns
// LABFM_ERR_HIP from the enclosing function.
#define LABFM_HIP(call)                                                          \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::labfm::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                         __FILE__, __LINE__);                                    \
      return LABFM_ERR_HIP;                                                      \
    }                                                                            \
  } while (0)

#define LABFM_REQUIRE(cond, ...)                                                 \
  do {                                                                           \
    if (!(cond)) {                                                               \
      ::labfm::set_error(__VA_ARGS__);                                           \
      return LABFM_ERR_ARG;                                                      \
    }                                                                            \
  } while (0)

// Checks the launch that was just enqueued.
#define LABFM_LAUNCHED() LABFM_HIP(hipGetLastError())

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Rounds a byte count up to a multiple of 256 (the alignment of every part
// of a caller workspace).
inline size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Checks a caller workspace (device pointer and size in bytes) against what
// a call needs.
#define LABFM_WORKSPACE(ptr, have, need, what)                                    \
  LABFM_REQUIRE((ptr) != nullptr && (have) >= (need),                            \
                "%s: a workspace of %zu bytes is required (got %zu bytes at %p)", \
                what, static_cast<size_t>(need), static_cast<size_t>(have),      \
                static_cast<const void*>(ptr))

inline unsigned blocks_for(int64_t work, int per_block) {
  return static_cast<unsigned>((work + per_block - 1) / per_block);
}

// Largest LABFM order the library builds weights for, and the matching
// number of moments n = (m^2 + 3m)/2.
constexpr int kMaxOrder = 10;
constexpr int kMoments = LABFM_NUM_MOM32;  // rows of the float32-weight first moments
constexpr int kMaxMoments = (kMaxOrder * kMaxOrder + 3 * kMaxOrder) / 2;

__host__ __device__ constexpr int moments_of(int m) { return (m * m + 3 * m) / 2; }

// Row stride of the float32 weight copy: nnz rounded up to 32 elements, so
// every operator's row starts on a 128-byte boundary (labfm_w32_stride).
__host__ __device__ constexpr long long w32_stride(long long nnz) { return (nnz + 31) / 32 * 32; }

// Device-side minimum-image difference on one axis.
__device__ __forceinline__ double wrap_axis(double d, double L, int periodic) {
  if (periodic) {
    const double half = 0.5 * L;
    if (d > half) {
      d = d - L;
    } else if (d < -half) {
      d = d + L;
    }
  }
  return d;
}

// Wave-level (64-lane) butterfly sum of a double over lane groups of width
// `width` (a power of two <= 64): every lane of a group ends with the group
// total.
template <int width>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = width / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
  return v;
}

}  // namespace labfm
