// Mode product of a whole tensor at a group that does not start at mode 1, on MFMA:
// with T viewed as H[L][n][Q] (l fastest) and the group's map Y (n x k, row-major),
//   out[l + L (j + k q)] = sum_{i < n} H[l + L i + L n q] Y[i][j],
// the first contraction of an STTNN chain when the visiting order (Sec. 5) contracts a
// later group before the first one.  Output FP64: the chain's intermediates are FP64.
//
// The rows rho = l + L q of the product run along memory within each l-run, and the
// contraction index i steps by L, so the kernel computes the transpose
// C^T[j][rho] = sum_i Y[i][j] H(rho, i): in a 16 x 16 x 4 MFMA the tensor is the B
// operand (lane -> row rho), the map the A operand (lane -> column j), and each
// output fragment holds 16 consecutive rows of one column, so the stores of a lane
// group are contiguous.  A workgroup (4 waves) owns 128 rows and the whole
// contraction, taken in steps of KS values: for each value the 128 rows are loaded as
// 16-byte row vectors (whole vectors inside one l-run: L a multiple of V) into an LDS
// tile [i][rho], the KS rows of Y into a second tile [i][j]; the next step's loads
// are in flight while the waves multiply.  No contraction split: the rows number
// N / n, far more than the machine's workgroups, and each output is written once.
#include "kernels.hpp"
#include "mfma.hpp"

namespace ttnn {
namespace {

constexpr int kMidRows = 128;   // rows rho per workgroup: 4 waves x 2 blocks of 16

template <int DT, int NCB>
__global__ __launch_bounds__(256) void mid_mfma_kernel(const void* __restrict__ Hv, int64_t L, int64_t n, int64_t Q,
                                                       const void* __restrict__ Yv, int k, double* __restrict__ out) {
  using P = Pol<DT>;
  using T = typename P::T;
  static_assert(P::KPL == 1, "FP32 / FP64 fragments: one value a lane");
  constexpr int V = 16 / P::ESZ;               // rows per 16-byte vector
  constexpr int RV = kMidRows / V;             // vectors per contraction value
  constexpr int IPR = 256 / RV;                // contraction values per staging round
  constexpr int ROUNDS = 4;
  constexpr int KS = IPR * ROUNDS;             // contraction values per step (f32 32, f64 16)
  constexpr int PITCH = kMidRows + V;          // LDS pitch of a value's rows (one vector of pad)
  constexpr int NJ = 16 * NCB;                 // map columns staged (padded)
  constexpr int PITCHY = NJ + 1;
  constexpr int YPT = (KS * NJ + 255) / 256;   // map values a thread stages per step
  typedef T vec_t __attribute__((ext_vector_type(V)));
  __shared__ __align__(16) T As[2][KS * PITCH];
  __shared__ T Ys[2][KS * PITCHY];

  const T* H = static_cast<const T*>(Hv);
  const T* Y = static_cast<const T*>(Yv);
  const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t M = L * Q;
  const int64_t rho0 = static_cast<int64_t>(blockIdx.x) * kMidRows;

  // this thread's row vector (fixed over the contraction) and its first value
  const int vr = (tid % RV) * V, vi = tid / RV;
  const int64_t rho = rho0 + vr;
  const bool row_live = rho < M;              // V | L and V | rho: the vector stays in one run
  const int64_t qv = rho / L;
  const T* hrow = H + (rho - qv * L) + L * n * qv;

  vec_t ra0[ROUNDS], ra1[ROUNDS];
  T ry0[YPT], ry1[YPT];
  auto gload = [&](int64_t i0, vec_t* ra, T* ry) {
#pragma unroll
    for (int u = 0; u < ROUNDS; ++u) {
      const int64_t i = i0 + vi + IPR * u;
      ra[u] = (row_live && i < n) ? *reinterpret_cast<const vec_t*>(hrow + L * i) : vec_t{};
    }
#pragma unroll
    for (int u = 0; u < YPT; ++u) {
      const int e = tid + 256 * u, ii = e / NJ, j = e % NJ;
      const int64_t i = i0 + ii;
      ry[u] = (ii < KS && j < k && i < n) ? Y[i * k + j] : T(0);
    }
  };
  auto lstore = [&](int buf, const vec_t* ra, const T* ry) {
#pragma unroll
    for (int u = 0; u < ROUNDS; ++u)
      *reinterpret_cast<vec_t*>(&As[buf][(vi + IPR * u) * PITCH + vr]) = ra[u];
#pragma unroll
    for (int u = 0; u < YPT; ++u) {
      const int e = tid + 256 * u, ii = e / NJ, j = e % NJ;
      if (ii < KS) Ys[buf][ii * PITCHY + j] = ry[u];
    }
  };

  typename P::CFrag acc[2][NCB];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[b][cb] = typename P::CFrag{};
  const bool live0 = rho0 + 32 * wave < M, live1 = rho0 + 32 * wave + 16 < M;   // wave-uniform

  auto compute = [&](int buf) {
#pragma unroll
    for (int s = 0; s < KS / 4; ++s) {
      const int i = 4 * s + lg;
      const T b0 = As[buf][i * PITCH + 32 * wave + l16];
      const T b1 = As[buf][i * PITCH + 32 * wave + 16 + l16];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const T a = Ys[buf][i * PITCHY + 16 * cb + l16];
        if (live0) acc[0][cb] = P::mfma(a, b0, acc[0][cb]);
        if (live1) acc[1][cb] = P::mfma(a, b1, acc[1][cb]);
      }
    }
  };

  // step s is staged in LDS buffer s % 2; its loads were issued two steps earlier
  gload(0, ra0, ry0);
  gload(KS, ra1, ry1);
  lstore(0, ra0, ry0);
  __syncthreads();
  for (int64_t i0 = 0; i0 < n; i0 += 2 * KS) {
    gload(i0 + 2 * KS, ra0, ry0);
    compute(0);
    lstore(1, ra1, ry1);
    __syncthreads();
    if (i0 + KS >= n) break;
    gload(i0 + 3 * KS, ra1, ry1);
    compute(1);
    lstore(0, ra0, ry0);
    __syncthreads();
  }

  // C^T[j][rho]: lane -> row rho0 + 32 wave + 16 b + l16, column 16 cb + crow(lane, v)
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int64_t r = rho0 + 32 * wave + 16 * b + l16;
    if (r >= M) continue;
    const int64_t q = r / L;
    double* o = out + (r - q * L) + L * static_cast<int64_t>(k) * q;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 16 * cb + P::crow(lane, v);
        if (j < k) o[L * j] = static_cast<double>(acc[b][cb][v]);
      }
  }
}

template <int DT>
void launch_mid_dt(const void* H, int64_t L, int64_t n, int64_t Q, const void* Y, int k, double* out, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((L * Q + kMidRows - 1) / kMidRows));
  switch ((k + 15) / 16) {
    case 1: hipLaunchKernelGGL((mid_mfma_kernel<DT, 1>), grid, dim3(256), 0, st, H, L, n, Q, Y, k, out); break;
    case 2: hipLaunchKernelGGL((mid_mfma_kernel<DT, 2>), grid, dim3(256), 0, st, H, L, n, Q, Y, k, out); break;
    case 3: hipLaunchKernelGGL((mid_mfma_kernel<DT, 3>), grid, dim3(256), 0, st, H, L, n, Q, Y, k, out); break;
    case 4: hipLaunchKernelGGL((mid_mfma_kernel<DT, 4>), grid, dim3(256), 0, st, H, L, n, Q, Y, k, out); break;
    case 5: hipLaunchKernelGGL((mid_mfma_kernel<DT, 5>), grid, dim3(256), 0, st, H, L, n, Q, Y, k, out); break;
    case 6: hipLaunchKernelGGL((mid_mfma_kernel<DT, 6>), grid, dim3(256), 0, st, H, L, n, Q, Y, k, out); break;
    case 7: hipLaunchKernelGGL((mid_mfma_kernel<DT, 7>), grid, dim3(256), 0, st, H, L, n, Q, Y, k, out); break;
    default: hipLaunchKernelGGL((mid_mfma_kernel<DT, 8>), grid, dim3(256), 0, st, H, L, n, Q, Y, k, out); break;
  }
}

}  // namespace

bool mid_mfma_eligible(int64_t L, int64_t n, int64_t Q, int k, int dt) {
  if (dt != TTNN_F32 && dt != TTNN_F64) return false;
  const int64_t v = dt == TTNN_F32 ? 4 : 2;
  // whole row vectors in one l-run, at most 128 columns, enough rows to fill the machine
  return L > 1 && L % v == 0 && n >= 1 && Q >= 1 && k >= 1 && k <= 128 && L * Q >= 256 * kMidRows &&
         L * Q <= (int64_t(1) << 37);
}

void launch_mid_mfma(const void* H, int dt, int64_t L, int64_t n, int64_t Q, const void* Y, int k, double* out,
                     hipStream_t st) {
  TTNN_REQUIRE(mid_mfma_eligible(L, n, Q, k, dt), TTNN_E_INVALID, "mode product shape not covered by the MFMA form");
  if (dt == TTNN_F32) launch_mid_dt<TTNN_F32>(H, L, n, Q, Y, k, out, st);
  else launch_mid_dt<TTNN_F64>(H, L, n, Q, Y, k, out, st);
  TTNN_HIP(hipGetLastError());
}

}  // namespace ttnn
