// Right sketch of a whole tensor on MFMA: R_t = T^{(t)} X_t (eq. sketch) when the
// modes before t are contiguous and long, i.e. with T viewed as H[L][n][Q]
// (l fastest) and X_t rows indexed by l + L q:
//   out(i, j) = sum_{l, q} H[l + L (i + n q)] Xt[j][l + L q].
// The contraction index runs along memory in both the tensor and the transposed DRM
// copy Xt (r x m).  A workgroup (4 waves) owns 128 output rows and one contiguous
// chunk of the contraction, taken in steps of 128 bytes of every row: the step's
// rows are loaded with eight lanes per row (full cache lines, 16 bytes a lane) into a
// padded LDS tile, from which the waves read their MFMA fragments while the next
// step's loads are in flight.  Chunk partials are summed in a fixed order by the
// generic reduce.
//
// A fragment load gives a lane V = 16 / sizeof(T) consecutive contraction values; a
// 16 x 16 x K MFMA step takes KPL of them per lane group, so one load feeds V / KPL
// MFMAs.  The pairing of A and B values is the same in every MFMA, so the sum runs
// over the whole K range whatever the order.
//
// Row-contiguous form (IF, L = 1: nodes that start at mode 1, FP32 / FP64): there the
// contraction index q is the slow one and the rows i run along memory, so a step
// stages, for each of its KS contraction values, the workgroup's 128 rows as 16-byte
// row vectors into an LDS tile laid out [k][row]; a lane then gathers its V
// contraction values of one row from V tile rows.  In both forms, when n is not a
// multiple of the 128 rows of a workgroup (SK), row blocks wholly past n skip their
// MFMAs (a wave-uniform test).
//
// Few rows (SN, n <= 32, contiguous form): a 128-row tile would hold a quarter of real
// rows or less, so each step would move a fraction of the bytes it is sized for and the
// pass would be bound by the bytes in flight.  The tile is then 32 rows by four steps'
// worth of contraction values; each wave takes one quarter of every staged step for
// both row blocks, and the four waves' sums are added in wave order through LDS.
//
// Odd l-runs (S1, FP64, L odd): a lane's two consecutive contraction values may lie in
// two l-runs, so the tensor operand is loaded as two 8-byte values, the second one
// stepping to the next run when the first ends one.
//
// The contiguous form needs whole 16-byte vectors inside one l-run (L a multiple of
// V); when L Q is not a multiple of the step (KT) the last step is masked vector by
// vector.  The row-contiguous form needs whole row vectors (n a multiple of V) and
// whole steps (Q a multiple of the step).
#include <algorithm>
#include <atomic>

#include "kernels.hpp"
#include "mfma.hpp"

namespace ttnn {
namespace {

constexpr int kRows = 128;     // output rows per workgroup (4 waves x 2 row blocks of 16)
constexpr int kRowsFew = 32;   // at most this many rows: the few-rows tile (one row block pair)

template <int DT, int NCB, bool IF = false, bool SK = false, bool KT = false, bool SN = false, bool S1 = false>
__global__ __launch_bounds__(256) void right_mfma_kernel(const void* __restrict__ Hv, int64_t L, int64_t n, int64_t Q,
                                                         const void* __restrict__ Xtv, int64_t m, int r,
                                                         int64_t kchunk, double* __restrict__ part) {
  using P = Pol<DT>;
  using T = typename P::T;
  using Frag = typename P::Frag;
  using CFrag = typename P::CFrag;
  constexpr int V = 16 / P::ESZ;            // values per 16-byte load
  constexpr int KPL = P::KPL;
  constexpr int SUB = V / KPL;              // MFMAs per fragment load
  constexpr int KG = 4 * V;                 // contraction values per fragment step (4 lane groups)
  constexpr int KS = 2 * KG;                // contraction values per staged step: 128 bytes of a row
  constexpr int CPR = KS / V;               // 16-byte chunks of a row per step (8)
  constexpr int PITCH = KS + V;             // LDS row pitch: one 16-byte pad (rows on distinct banks)
  constexpr int NJ = 16 * NCB;              // DRM rows staged (output columns, padded)
  constexpr int RPR = 256 / CPR;            // rows per staging round (32)
  constexpr int AR = kRows / RPR;           // staging rounds of the tensor tile
  constexpr int BRN = (NJ + RPR - 1) / RPR; // staging rounds of the DRM tile
  constexpr int ROWS = SN ? 32 : kRows;     // output rows per workgroup
  constexpr int KSX = SN ? 4 * KS : KS;     // contraction values per staged step
  constexpr int CPRX = KSX / V;
  constexpr int PITCHX = KSX + V;
  constexpr int RPRX = 256 / CPRX;
  constexpr int ARX = ROWS / RPRX;
  constexpr int BRNX = (NJ + RPRX - 1) / RPRX;
  static_assert(!(IF && SN), "one tile form at a time");
  static_assert(!S1 || (DT == TTNN_F64 && !IF), "odd l-runs: FP64 contiguous form");
  constexpr int RV = kRows / V;             // IF: row vectors per contraction value
  constexpr int PITCHT = kRows + V;         // IF: LDS pitch of a contraction value's rows
  constexpr int ASZ = IF ? KS * PITCHT : ROWS * PITCHX;
  static_assert(!IF || (KPL == 1 && KS * RV == 256 * AR), "row-contiguous form: FP32 / FP64 tiles");
  typedef T vec_t __attribute__((ext_vector_type(V)));
  __shared__ __align__(16) T As[2][ASZ];
  __shared__ __align__(16) T Bs[2][NJ * PITCHX];

  const T* H = static_cast<const T*>(Hv);
  const T* Xt = static_cast<const T*>(Xtv);
  const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kRows;
  const int64_t K = L * Q;
  const int64_t c = blockIdx.y;
  const int64_t k_begin = c * kchunk;
  const int64_t k_end = k_begin + kchunk < K ? k_begin + kchunk : K;

  // staging map: thread -> row tid / CPR (+ RPR per round), chunk tid % CPR
  const int sr = tid / CPRX, sc = (tid % CPRX) * V;
  vec_t ra0[ARX], rb0[BRNX], ra1[ARX], rb1[BRNX];   // two steps of loads in flight
  auto gload = [&](int64_t k, vec_t* ra, vec_t* rb) {
    const int64_t kk = k + sc;
    const bool live = (KT ? kk : k) < k_end;
    const int64_t q = kk / L, l = kk - q * L;
    if constexpr (IF) {
      // H[i + n q]: thread -> row vector tid % RV of contraction values tid / RV (+ 256 / RV a round)
#pragma unroll
      for (int u = 0; u < AR; ++u) {
        const int e = tid + 256 * u;
        const int64_t qq = k + e / RV, row = row0 + static_cast<int64_t>(e % RV) * V;
        ra[u] = (live && row < n) ? *reinterpret_cast<const vec_t*>(H + row + n * qq) : vec_t{};
      }
    } else {
      if constexpr (S1) {
        // value kk at (l, q), value kk + 1 at (l + 1, q) or at (0, q + 1)
        const int64_t l1 = l + 1 == L ? 0 : l + 1, q1 = l + 1 == L ? q + 1 : q;
#pragma unroll
        for (int u = 0; u < ARX; ++u) {
          const int64_t row = row0 + sr + RPRX * u;
          vec_t v{};
          if (live && row < n) {
            v[0] = H[l + L * (row + n * q)];
            v[1] = H[l1 + L * (row + n * q1)];
          }
          ra[u] = v;
        }
      } else {
#pragma unroll
        for (int u = 0; u < ARX; ++u) {
          const int64_t row = row0 + sr + RPRX * u;
          ra[u] = (live && row < n) ? *reinterpret_cast<const vec_t*>(H + l + L * (row + n * q)) : vec_t{};
        }
      }
    }
#pragma unroll
    for (int u = 0; u < BRNX; ++u) {
      const int j = sr + RPRX * u;
      rb[u] = (live && j < r) ? *reinterpret_cast<const vec_t*>(Xt + static_cast<int64_t>(j) * m + kk) : vec_t{};
    }
  };
  auto lstore = [&](int buf, const vec_t* ra, const vec_t* rb) {
    if constexpr (IF) {
#pragma unroll
      for (int u = 0; u < AR; ++u) {
        const int e = tid + 256 * u;
        *reinterpret_cast<vec_t*>(&As[buf][(e / RV) * PITCHT + (e % RV) * V]) = ra[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < ARX; ++u) *reinterpret_cast<vec_t*>(&As[buf][(sr + RPRX * u) * PITCHX + sc]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < BRNX; ++u)
      if (sr + RPRX * u < NJ) *reinterpret_cast<vec_t*>(&Bs[buf][(sr + RPRX * u) * PITCHX + sc]) = rb[u];
  };

  CFrag acc[2][NCB];
  const CFrag zero = {};
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[b][cb] = zero;

  auto compute = [&](int buf) {
#pragma unroll
    for (int h = 0; h < KS / KG; ++h) {
      const int kl = (SN ? KS * wave : 0) + h * KG + V * lg;
      constexpr int WROWS = SN ? 0 : 32;      // rows a wave owns (SN: all 32, every wave)
      vec_t a[2], bx[NCB];
      if constexpr (IF) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int s = 0; s < V; ++s) a[b][s] = As[buf][(kl + s) * PITCHT + 32 * wave + 16 * b + l16];
      } else {
#pragma unroll
        for (int b = 0; b < 2; ++b)
          a[b] = *reinterpret_cast<const vec_t*>(&As[buf][(WROWS * wave + 16 * b + l16) * PITCHX + kl]);
      }
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        bx[cb] = *reinterpret_cast<const vec_t*>(&Bs[buf][(16 * cb + l16) * PITCHX + kl]);
#pragma unroll
      for (int s = 0; s < SUB; ++s) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if constexpr (IF || SK) {
            if (row0 + WROWS * wave + 16 * b >= n) continue;   // wave-uniform: rows past n
          }
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
  };

  // step s is staged in LDS buffer s % 2 and its loads were issued two steps earlier
  gload(k_begin, ra0, rb0);
  gload(k_begin + KSX, ra1, rb1);
  lstore(0, ra0, rb0);
  __syncthreads();
  for (int64_t k = k_begin; k < k_end; k += 2 * KSX) {
    gload(k + 2 * KSX, ra0, rb0);            // step s + 2
    compute(0);                              // step s
    lstore(1, ra1, rb1);                     // step s + 1 (buffer 1 was read before the last barrier)
    __syncthreads();
    if (k + KSX >= k_end) break;
    gload(k + 3 * KSX, ra1, rb1);            // step s + 3
    compute(1);                              // step s + 1
    lstore(0, ra0, rb0);                     // step s + 2
    __syncthreads();
  }

  // partial of chunk c: part[(c n + i) r + j]
  if constexpr (SN) {
    // every wave holds its quarters' sums for all 32 rows: add them in wave order
    // through LDS (the A tile is free after the loop's last barrier), one column block
    // at a time; thread t delivers entries t and t + 256 of the block's 2 x 4 x 64
    double* red = reinterpret_cast<double*>(&As[0][0]);
    static_assert(2 * ASZ * sizeof(T) >= 4 * 512 * sizeof(double), "reduction fits the A tile");
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave * 8 + b * 4 + v) * 64 + lane] = static_cast<double>(acc[b][cb][v]);
      __syncthreads();
#pragma unroll
      for (int e0 = 0; e0 < 512; e0 += 256) {
        const int e = e0 + tid, b = e >> 8, v = (e >> 6) & 3, ln = e & 63;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) sum += red[(w * 8 + b * 4 + v) * 64 + ln];
        const int64_t i = row0 + 16 * b + P::crow(ln, v);
        const int j = 16 * cb + (ln & 15);
        if (i < n && j < r) part[(c * n + i) * r + j] = sum;
      }
      __syncthreads();
    }
    return;
  }
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

template <int DT, bool IF, bool SK, bool KT = false, bool SN = false, bool S1 = false>
void launch_form(const void* H, int64_t L, int64_t n, int64_t Q, const void* Xt, int64_t m, int r, int64_t kchunk,
                 int64_t nch, double* part, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n + kRows - 1) / kRows), static_cast<unsigned>(nch));
  const int ncb = (r + 15) / 16;
  if (ncb <= 1)
    hipLaunchKernelGGL((right_mfma_kernel<DT, 1, IF, SK, KT, SN, S1>), grid, dim3(256), 0, st, H, L, n, Q, Xt, m, r, kchunk,
                       part);
  else if (ncb == 2)
    hipLaunchKernelGGL((right_mfma_kernel<DT, 2, IF, SK, KT, SN, S1>), grid, dim3(256), 0, st, H, L, n, Q, Xt, m, r, kchunk,
                       part);
  else if (ncb == 3)
    hipLaunchKernelGGL((right_mfma_kernel<DT, 3, IF, SK, KT, SN, S1>), grid, dim3(256), 0, st, H, L, n, Q, Xt, m, r, kchunk,
                       part);
  else
    hipLaunchKernelGGL((right_mfma_kernel<DT, 4, IF, SK, KT, SN, S1>), grid, dim3(256), 0, st, H, L, n, Q, Xt, m, r, kchunk,
                       part);
}

template <int DT>
void launch_dt(bool rowc, const void* H, int64_t L, int64_t n, int64_t Q, const void* Xt, int64_t m, int r,
               int64_t kchunk, int64_t nch, double* part, hipStream_t st) {
  const bool sk = n % kRows != 0;
  if constexpr (DT != TTNN_BF16) {
    if (rowc) {
      launch_form<DT, true, true>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
      return;
    }
  }
  constexpr int64_t KS = 2 * 4 * (16 / Pol<DT>::ESZ);   // the kernel's staged step
  if constexpr (DT == TTNN_F64) {
    if (L % 2 != 0) {                                  // odd l-runs: 8-byte tensor loads
      const bool kt = (L * Q) % (n <= kRowsFew ? 4 * KS : KS) != 0;
      if (n <= kRowsFew && kt) launch_form<DT, false, true, true, true, true>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
      else if (n <= kRowsFew) launch_form<DT, false, true, false, true, true>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
      else launch_form<DT, false, true, true, false, true>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
      return;
    }
  }
  if (n <= kRowsFew) {                                 // few rows: 32-row tiles of 4 steps
    if ((L * Q) % (4 * KS) != 0) launch_form<DT, false, true, true, true>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
    else launch_form<DT, false, true, false, true>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  } else if ((L * Q) % KS != 0) {
    launch_form<DT, false, true, true>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  } else if (sk) {
    launch_form<DT, false, true>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  } else {
    launch_form<DT, false, false>(H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  }
}

// compute units of the current device (queried once per device; threads that race
// on the first query store the same value)
int compute_units() {
  static std::atomic<int> cus[64];
  int dev = 0;
  TTNN_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return 256;
  int c = cus[dev].load(std::memory_order_relaxed);
  if (c == 0) {
    int n = 0;
    TTNN_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    c = n > 0 ? n : 256;
    cus[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

}  // namespace

bool right_mfma_eligible(int64_t L, int64_t n, int64_t Q, int r, int dt) {
  const int64_t ks = dt == TTNN_BF16 ? 64 : dt == TTNN_F32 ? 32 : 16;   // staged step: 128 bytes of a row
  const int64_t v = 16 / (dt == TTNN_BF16 ? 2 : dt == TTNN_F32 ? 4 : 8);   // values per 16-byte vector
  if (r < 1 || r > 64 || n < 1 || Q < 1) return false;
  // contiguous form: whole vectors inside one l-run
  if (L >= v && L % v == 0 && L * Q >= 16) return true;
  // FP64 with odd l-runs: two 8-byte tensor loads a vector, whole DRM vectors
  if (dt == TTNN_F64 && L > 1 && L % 2 == 1 && (L * Q) % 2 == 0 && L * Q >= 16) return true;
  // row-contiguous form: whole row vectors, whole steps
  return L == 1 && dt != TTNN_BF16 && n % v == 0 && Q % ks == 0 && Q >= 64;
}

RightMfmaSplit right_mfma_split(int64_t L, int64_t n, int64_t Q, int r, int dt, size_t part_elems, int cus) {
  TTNN_REQUIRE(right_mfma_eligible(L, n, Q, r, dt), TTNN_E_INVALID, "right sketch shape not covered by the MFMA form");
  // every chunk writes an n x r partial: the scratch must hold at least one
  TTNN_REQUIRE(part_elems >= static_cast<size_t>(n) * static_cast<size_t>(r), TTNN_E_INVALID,
               "partial buffer smaller than one chunk of the right sketch");
  const int64_t K = L * Q;
  const bool few = L != 1 && n <= kRowsFew;
  const int64_t kg = (dt == TTNN_BF16 ? 64 : dt == TTNN_F32 ? 32 : 16) * (few ? 4 : 1);   // staged step
  const int64_t row_blocks = (n + kRows - 1) / kRows;
  // enough workgroups to fill the chip twice, chunks of at least 1024 values, and
  // partials within the scratch
  int64_t nch = (2048 + row_blocks - 1) / row_blocks;
  nch = std::min<int64_t>(nch, (K + 1023) / 1024);
  nch = std::min<int64_t>(nch, static_cast<int64_t>(part_elems / static_cast<size_t>(n * r)));
  // and at most one round of resident workgroups (three a compute unit, by LDS): a
  // second, partial round would stream with a fraction of the machine
  nch = std::min<int64_t>(nch, std::max<int64_t>(1, 3 * static_cast<int64_t>(cus) / row_blocks));
  nch = std::max<int64_t>(nch, 1);
  int64_t kchunk = (K + nch - 1) / nch;
  kchunk = (kchunk + kg - 1) / kg * kg;
  nch = (K + kchunk - 1) / kchunk;
  return RightMfmaSplit{nch, kchunk};
}

int launch_right_mfma(const void* H, int dt, int64_t L, int64_t n, int64_t Q, const void* Xt, int64_t m, int r,
                      double* part, size_t part_elems, hipStream_t st) {
  const RightMfmaSplit sp = right_mfma_split(L, n, Q, r, dt, part_elems, compute_units());
  const int64_t nch = sp.nch, kchunk = sp.kchunk;
  const bool rowc = L == 1;
  if (dt == TTNN_BF16) launch_dt<TTNN_BF16>(rowc, H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  else if (dt == TTNN_F32) launch_dt<TTNN_F32>(rowc, H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  else launch_dt<TTNN_F64>(rowc, H, L, n, Q, Xt, m, r, kchunk, nch, part, st);
  return static_cast<int>(nch);
}

}  // namespace ttnn
