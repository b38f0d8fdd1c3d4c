// Right sketch of a whole tensor on MFMA: R_t = T^{(t)} X_t (eq. sketch) when the
// modes before t are contiguous and long, i.e. with T viewed as H[L][n][Q]
// (l fastest) and X_t rows indexed by l + L q:
//   out(i, j) = sum_{l, q} H[l + L (i + n q)] Xt[j][l + L q].
// The contraction index runs along memory, so the tensor feeds MFMA A fragments
// straight from global memory (16 bytes a lane) and the transposed DRM copy Xt
// (r x m, contraction index contiguous) feeds B fragments the same way; no LDS.
// A workgroup (4 waves) owns 128 output rows and one contiguous chunk of the
// contraction; chunk partials are summed in a fixed order by the generic reduce.
//
// Each lane loads V = 16 / sizeof(T) consecutive contraction values; a 16 x 16 x K
// MFMA step takes KPL of them per lane group, so one load feeds V / KPL MFMAs.  The
// pairing of A and B values is the same in every MFMA, so the sum runs over the
// whole K range whatever the order.
#include <algorithm>

#include "kernels.hpp"
#include "mfma.hpp"

namespace ttnn {
namespace {

constexpr int kRows = 128;     // output rows per workgroup
constexpr int kWaves = 4;      // each wave: 2 row blocks of 16

template <int DT, int NCB>
__global__ __launch_bounds__(256) void right_mfma_kernel(const void* __restrict__ Hv, int64_t L, int64_t n, int64_t Q,
                                                         const void* __restrict__ Xtv, int64_t m, int r,
                                                         int64_t kchunk, double* __restrict__ part) {
  using P = Pol<DT>;
  using T = typename P::T;
  using Frag = typename P::Frag;
  using CFrag = typename P::CFrag;
  constexpr int V = 16 / P::ESZ;            // values per 16-byte load
  constexpr int KPL = P::KPL;
  constexpr int SUB = V / KPL;              // MFMAs per load
  constexpr int KG = 4 * V;                 // contraction values per step (4 lane groups)
  typedef T vec_t __attribute__((ext_vector_type(V)));

  const T* H = static_cast<const T*>(Hv);
  const T* Xt = static_cast<const T*>(Xtv);
  const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kRows;
  const int64_t K = L * Q;
  const int64_t c = blockIdx.y;
  const int64_t k_begin = c * kchunk;
  const int64_t k_end = k_begin + kchunk < K ? k_begin + kchunk : K;

  // rows of this lane's A loads (two row blocks per wave), clamped for loading
  int64_t irow[2];
  bool rvalid[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    irow[b] = row0 + 32 * wave + 16 * b + l16;
    rvalid[b] = irow[b] < n;
  }
  int jcol[NCB];
  bool cvalid[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    jcol[cb] = 16 * cb + l16;
    cvalid[cb] = jcol[cb] < r;
  }

  CFrag acc[2][NCB];
  const CFrag zero = {};
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[b][cb] = zero;

#pragma unroll 2
  for (int64_t k = k_begin; k < k_end; k += KG) {
    const int64_t kk = k + V * lg;          // this lane group's first value
    const int64_t q = kk / L, l = kk - q * L;
    vec_t a[2], bx[NCB];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (rvalid[b]) a[b] = *reinterpret_cast<const vec_t*>(H + l + L * (irow[b] + n * q));
      else a[b] = vec_t{};
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      if (cvalid[cb]) bx[cb] = *reinterpret_cast<const vec_t*>(Xt + static_cast<int64_t>(jcol[cb]) * m + kk);
      else bx[cb] = vec_t{};
    }
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        Frag af;
        if constexpr (KPL == 8) af = __builtin_bit_cast(Frag, a[b]);
        else af = a[b][s];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          Frag bf;
          if constexpr (KPL == 8) bf = __builtin_bit_cast(Frag, bx[cb]);
          else bf = bx[cb][s];
          acc[b][cb] = P::mfma(af, bf, acc[b][cb]);
        }
      }
    }
  }

  // partial of chunk c: part[(c n + i) r + j]
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = row0 + 32 * wave + 16 * b + P::crow(lane, v);
      if (i >= n) continue;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int j = 16 * cb + l16;
        if (j < r) part[(c * n + i) * r + j] = static_cast<double>(acc[b][cb][v]);
      }
    }
}

template <int DT>
void launch_dt(const void* H, int64_t L, int64_t n, int64_t Q, const void* Xt, int64_t m, int r, int64_t kchunk,
               int64_t nch, double* part, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kRows - 1) / kRows), static_cast<unsigned>(nch));
  const int ncb = (r + 15) / 16;
  if (ncb <= 1) hipLaunchKernelGGL((right_mfma_kernel<DT, 1>), grid, dim3(256), 0, st, H, L, n, Q, Xt, m, r, kchunk, part);
  else if (ncb == 2)
    hipLaunchKernelGGL((right_mfma_kernel<DT, 2>), grid, dim3(256), 0, st, H, L, n, Q, Xt, m, r, kchunk, part);
  else if (ncb == 3)
    hipLaunchKernelGGL((right_mfma_kernel<DT, 3>), grid, dim3(256), 0, st, H, L, n, Q, Xt, m, r, kchunk, part);
  else hipLaunchKernelGGL((right_mfma_kernel<DT, 4>), grid, dim3(256), 0, st, H, L, n, Q, Xt, m, r, kchunk, part);
}

}  // namespace

bool right_mfma_eligible(int64_t L, int64_t n, int64_t Q, int r, int dt) {
  (void)n;
  (void)Q;
  const int64_t kg = dt == TTNN_BF16 ? 32 : dt == TTNN_F32 ? 16 : 8;
  return L % kg == 0 && L >= 64 && r >= 1 && r <= 64;
}

int launch_right_mfma(const void* H, int dt, int64_t L, int64_t n, int64_t Q, const void* Xt, int64_t m, int r,
                      double* part, size_t part_elems, hipStream_t st) {
  const int64_t K = L * Q;
  const int64_t kg = dt == TTNN_BF16 ? 32 : dt == TTNN_F32 ? 16 : 8;
  const int64_t row_blocks = (n + kRows - 1) / kRows;
  // enough workgroups to fill the chip twice, chunks of at least 1024 values, and
  // partials within the scratch
  int64_t nch = (2048 + row_blocks - 1) / row_blocks;
  nch = std::min<int64_t>(nch, (K + 1023) / 1024);
  nch = std::min<int64_t>(nch, static_cast<int64_t>(part_elems / static_cast<size_t>(n * r)));
  nch = std::max<int64_t>(nch, 1);
  int64_t kchunk = (K + nch - 1) / nch;
  kchunk = (kchunk + kg - 1) / kg * kg;
  nch = (K + kchunk - 1) / kchunk;
  if (dt == TTNN_BF16) launch_dt<TTNN_BF16>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  else if (dt == TTNN_F32) launch_dt<TTNN_F32>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  else launch_dt<TTNN_F64>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  return static_cast<int>(nch);
}

}  // namespace ttnn
