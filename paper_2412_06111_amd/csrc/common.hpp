// Shared host/device helpers of the TTNN engine: status plumbing, dtype tags and
// the mixed-radix index maps that turn a box-local linear index into a DRM row.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/ttnn.h"

namespace ttnn {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);          // thread-local message
const char* last_error();

struct Error {
  ttnn_status status;
  std::string msg;
};

#define TTNN_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::ttnn::Error{TTNN_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define TTNN_REQUIRE(cond, code, msg)                                             \
  do {                                                                            \
    if (!(cond)) throw ::ttnn::Error{code, msg};                                  \
  } while (0)

// ---------------------------------------------------------------- dtypes
inline size_t dtype_size(int dt) {
  return dt == TTNN_F64 ? 8 : dt == TTNN_F32 ? 4 : 2;
}

// bf16 storage is the raw upper half of the fp32 bit pattern
__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

template <typename T> __device__ inline double to_f64(T v);
template <> __device__ inline double to_f64<double>(double v) { return v; }
template <> __device__ inline double to_f64<float>(float v) { return static_cast<double>(v); }
template <> __device__ inline double to_f64<uint16_t>(uint16_t v) {
  return static_cast<double>(bf16_bits_to_f32(v));
}

// ---------------------------------------------------------------- index maps
constexpr int kMaxPos = TTNN_MAX_ORDER + 1;

// Decodes a linear index over `n` positions (first fastest, extents ext[]) and
// returns sum_p (off[p] + i_p) * stride[p].
struct IndexMap {
  int32_t n = 0;
  int64_t ext[kMaxPos] = {};
  int64_t off[kMaxPos] = {};
  int64_t stride[kMaxPos] = {};

  __host__ __device__ inline int64_t operator()(int64_t idx) const {
    int64_t row = 0;
    for (int p = 0; p < n; ++p) {
      const int64_t e = ext[p];
      const int64_t i = idx % e;
      idx /= e;
      row += (off[p] + i) * stride[p];
    }
    return row;
  }
  void push(int64_t e, int64_t o, int64_t s) {
    ext[n] = e;
    off[n] = o;
    stride[n] = s;
    ++n;
  }
  int64_t count() const {
    int64_t c = 1;
    for (int p = 0; p < n; ++p) c *= ext[p];
    return c;
  }
};

}  // namespace ttnn
