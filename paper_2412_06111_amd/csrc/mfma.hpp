// MFMA policies for gfx950 (CDNA4), one per storage dtype.  Every policy uses a
// 16 x 16 output block with K values spread over the four 16-lane groups:
//   A fragment: lane l holds A[l % 16][KPL*(l/16) + e], e < KPL
//   B fragment: lane l holds B[KPL*(l/16) + e][l % 16]
//   C fragment: lane l holds C[crow(l, v)][l % 16], v < 4
// (bf16 16x16x32 and f32 16x16x4: crow = 4*(l/16) + v; f64 16x16x4: crow = 4*v + l/16.)
#pragma once

#include "common.hpp"

namespace ttnn {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <int DT> struct Pol;

template <> struct Pol<TTNN_BF16> {
  using T = uint16_t;            // storage: bf16 bit pattern
  using Acc = float;
  using Frag = bf16x8_t;
  using CFrag = f32x4_t;
  static constexpr int KPL = 8, KSTEP = 32, ESZ = 2;
  __device__ static inline CFrag mfma(Frag a, Frag b, CFrag c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int crow(int l, int v) { return 4 * (l >> 4) + v; }
  // 8 consecutive elements (16-byte aligned)
  __device__ static inline Frag load8(const T* p) {
    return __builtin_bit_cast(Frag, *reinterpret_cast<const u16x8_t*>(p));
  }
  __device__ static inline T from_acc(float x) {
    const uint32_t b = __float_as_uint(x);
    return static_cast<uint16_t>((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
  }
};

template <> struct Pol<TTNN_F32> {
  using T = float;
  using Acc = float;
  using Frag = float;
  using CFrag = f32x4_t;
  static constexpr int KPL = 1, KSTEP = 4, ESZ = 4;
  __device__ static inline CFrag mfma(Frag a, Frag b, CFrag c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int crow(int l, int v) { return 4 * (l >> 4) + v; }
  __device__ static inline T from_acc(float x) { return x; }
};

template <> struct Pol<TTNN_F64> {
  using T = double;
  using Acc = double;
  using Frag = double;
  using CFrag = f64x4_t;
  static constexpr int KPL = 1, KSTEP = 4, ESZ = 8;
  __device__ static inline CFrag mfma(Frag a, Frag b, CFrag c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int crow(int l, int v) { return 4 * v + (l >> 4); }
  __device__ static inline T from_acc(double x) { return x; }
};

}  // namespace ttnn
