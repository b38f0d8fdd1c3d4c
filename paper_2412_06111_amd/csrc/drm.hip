// Seeded Gaussian DRMs (Sec. 4, eq. "sketch"; Gaussian maps of Lemma 4 and
// Theorem 2).  One thread per entry:
//   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) on counter
//   (lo32 row, hi32 row, col, 2 node + kind) with key (lo32 seed, hi32 seed);
//   u1 = (a + 1) 2^-53 in (0,1], u2 = b 2^-53 in [0,1) from the 53 high bits of
//   the 64-bit words (x1:x0) and (x3:x2);  z = sqrt(-2 ln u1) cos(2 pi u2).
// ln and cos(2 pi .) are fixed sequences of correctly rounded binary64 operations
// (atanh series for ln after an exact split u = f 2^e; Taylor series for cos / sin
// after exact reduction of the argument to [0, 1/4]), compiled without FMA
// contraction, so the FP64 value is reproducible bit for bit on any IEEE machine.
// FP32 copy = round-to-nearest(z); BF16 copy = round-to-nearest-even of the FP32
// bit pattern to its upper half.
#include "kernels.hpp"

#pragma clang fp contract(off)

namespace ttnn {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;   // double nearest sqrt(2)
constexpr double kLn2 = 0x1.62e42fefa39efp-1;     // double nearest ln 2
constexpr double kTwoPi = 0x1.921fb54442d18p+2;   // double nearest 2 pi
constexpr double kTwoM53 = 0x1p-53;

struct Series {
  double ln[24];    // ln[k] = 1/k for odd k in [3, 23]
  double cosc[11];  // a_0 = 1, a_k = -a_{k-1} / ((2k-1)(2k))
  double sinc[11];  // b_0 = 1, b_k = -b_{k-1} / ((2k)(2k+1))
};

constexpr Series make_series() {
  Series s{};
  for (int k = 3; k <= 23; k += 2) s.ln[k] = 1.0 / static_cast<double>(k);
  s.cosc[0] = 1.0;
  s.sinc[0] = 1.0;
  for (int k = 1; k <= 10; ++k) {
    s.cosc[k] = -s.cosc[k - 1] / static_cast<double>((2 * k - 1) * (2 * k));
    s.sinc[k] = -s.sinc[k - 1] / static_cast<double>((2 * k) * (2 * k + 1));
  }
  return s;
}

__constant__ Series kSeries = make_series();

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint32_t hi0 = __umulhi(kPhiloxM0, c[0]);
    const uint32_t lo0 = kPhiloxM0 * c[0];
    const uint32_t hi1 = __umulhi(kPhiloxM1, c[2]);
    const uint32_t lo1 = kPhiloxM1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// ln(u), u in (0, 1]: u = f 2^e exactly from the bits, f in [1, 2), halved when
// above sqrt(2); ln f = 2 atanh(s), s = (f-1)/(f+1), |s| <= 0.1716.
__device__ inline double ln_fixed(double u) {
  const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(u));
  const int ebiased = static_cast<int>((bits >> 52) & 0x7ff);
  double e = static_cast<double>(ebiased - 1023);
  double f = __longlong_as_double(static_cast<long long>((bits & 0x000fffffffffffffull) |
                                                        0x3ff0000000000000ull));
  if (f > kSqrt2) {
    f = f * 0.5;
    e = e + 1.0;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double w = s * s;
  double P = kSeries.ln[23];
#pragma unroll
  for (int k = 21; k >= 3; k -= 2) P = kSeries.ln[k] + w * P;
  const double lnf = 2.0 * (s + s * (w * P));
  return e * kLn2 + lnf;
}

__device__ inline double horner(double y, const double* c) {
  double acc = c[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) acc = c[k] + y * acc;
  return acc;
}

// cos(2 pi v), v in [0, 1)
__device__ inline double cos2pi_fixed(double v) {
  if (v >= 0.5) v = 1.0 - v;
  double sg = 1.0;
  if (v > 0.25) {
    v = 0.5 - v;
    sg = -1.0;
  }
  double c;
  if (v <= 0.125) {
    const double x = kTwoPi * v;
    c = horner(x * x, kSeries.cosc);
  } else {
    const double x = kTwoPi * (0.25 - v);
    c = x * horner(x * x, kSeries.sinc);
  }
  return sg * c;
}

__device__ inline double gaussian(uint64_t seed, uint32_t tag, uint64_t row, uint32_t col) {
  uint32_t c[4] = {static_cast<uint32_t>(row), static_cast<uint32_t>(row >> 32), col, tag};
  philox4x32_10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  const uint64_t a = ((static_cast<uint64_t>(c[1]) << 32) | c[0]) >> 11;
  const uint64_t b = ((static_cast<uint64_t>(c[3]) << 32) | c[2]) >> 11;
  const double u1 = static_cast<double>(a + 1) * kTwoM53;
  const double u2 = static_cast<double>(b) * kTwoM53;
  return __builtin_sqrt(-2.0 * ln_fixed(u1)) * cos2pi_fixed(u2);
}

__global__ void drm_kernel(int64_t rows, int cols, uint64_t seed, uint32_t tag, double* __restrict__ o64,
                           float* __restrict__ o32, uint16_t* __restrict__ o16) {
  const int64_t total = rows * cols;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  // (row, column) of idx, advanced by the grid stride with one carry test instead of a
  // 64-bit division per entry (the generator is bound by its integer and FP64 work)
  int64_t row = idx / cols;
  int col = static_cast<int>(idx - row * cols);
  const int64_t srow = stride / cols;
  const int scol = static_cast<int>(stride - srow * cols);
  for (; idx < total; idx += stride) {
    const double z = gaussian(seed, tag, static_cast<uint64_t>(row), static_cast<uint32_t>(col));
    // a plan of lower precision uses one matrix everywhere: the rounded copy, whose
    // values the FP64 array then holds exactly
    double m = z;
    if (o32 || o16) {
      const float f = static_cast<float>(z);
      m = static_cast<double>(f);
      if (o32) o32[idx] = f;
      if (o16) {
        const uint32_t b = __float_as_uint(f);
        const uint16_t h = static_cast<uint16_t>((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
        o16[idx] = h;
        m = static_cast<double>(bf16_bits_to_f32(h));
      }
    }
    o64[idx] = m;
    col += scol;
    row += srow;
    if (col >= cols) {
      col -= cols;
      ++row;
    }
  }
}

}  // namespace

__global__ void eye_kernel(int64_t n, double* o64, float* o32, uint16_t* o16) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n * n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const bool diag = e / n == e % n;
    o64[e] = diag ? 1.0 : 0.0;
    if (o32) o32[e] = diag ? 1.0f : 0.0f;
    if (o16) o16[e] = diag ? static_cast<uint16_t>(0x3F80) : static_cast<uint16_t>(0);   // BF16 1.0
  }
}

void launch_eye(int64_t n, double* o64, float* o32, uint16_t* o16, hipStream_t stream) {
  if (n <= 0) return;
  const int64_t want = (n * n + 255) / 256;
  const int blocks = static_cast<int>(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(eye_kernel, dim3(blocks), dim3(256), 0, stream, n, o64, o32, o16);
}

void launch_drm(int64_t rows, int cols, uint64_t seed, uint32_t tag, double* o64, float* o32,
                uint16_t* o16, hipStream_t stream) {
  const int64_t total = rows * cols;
  if (total <= 0) return;
  const int threads = 256;
  const int64_t want = (total + threads - 1) / threads;
  const int blocks = static_cast<int>(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(drm_kernel, dim3(blocks), dim3(threads), 0, stream, rows, cols, seed, tag, o64,
                     o32, o16);
}

}  // namespace ttnn
