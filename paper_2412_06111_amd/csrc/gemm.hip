// Generic contraction kernels of the engine (any tree, any box, any dtype).
//
// One LDS-tiled FP64 kernel covers both contractions the method needs on a
// 3-index view H[L][n][Q] of a (partially contracted) tensor:
//   RIGHT  R(i, j)    = sum_{l,q} H[l, i, q] X[row(l, q), j]   (right sketch T^{t} X_t,
//                                                           Sec. 4; STTNN on T_{S_t}, Sec. 5)
//   LEFT   Z(l, j, q) = sum_i     H[l, i, q] Y[row(i), j]      (mode product with Y_s^T,
//                                                           Def. 1 / Sec. 5 contractions)
// The contraction is split in chunks; each chunk writes an FP64 partial that a
// second kernel sums in a fixed order, so the result does not depend on timing.
// This path is the reference engine for arbitrary shapes; the fused kernels for
// the large dense trees live in separate files.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>

#include "kernels.hpp"
#include "mfma.hpp"

namespace ttnn {
namespace {

constexpr int BR = 64;   // output rows per block
constexpr int BJ = 32;   // output columns per block
constexpr int BK = 16;   // contraction step

template <typename T> __device__ inline double ld(const T* p, int64_t i) { return to_f64(p[i]); }
__device__ inline float ldf(const float* p, int64_t i) { return p[i]; }
__device__ inline float ldf(const uint16_t* p, int64_t i) { return bf16_bits_to_f32(p[i]); }

// The tile's inner product on the 16x16x4 MFMA of the compute type CT: FP32 for FP32 /
// BF16 operands (FP32 accumulation within the chunk; the chunk partial is written in
// the output type and chunks are summed in FP64 by the reduction), FP64 when either
// operand is FP64.  Each of the 4 waves owns 16 rows and both 16-column blocks.  A VALU
// form (four rows by two columns a thread) reads six LDS words per eight FMAs and is
// bound by LDS bandwidth; an MFMA reads one word a lane per 1024 FMAs (FP32) or 512
// (FP64), and the FP64 MFMA's peak equals the FP64 vector units'.
template <typename CT> __device__ inline CT ldc(const float* p, int64_t i) { return static_cast<CT>(p[i]); }
template <typename CT> __device__ inline CT ldc(const uint16_t* p, int64_t i) {
  return static_cast<CT>(bf16_bits_to_f32(p[i]));
}
template <typename CT> __device__ inline CT ldc(const double* p, int64_t i) { return static_cast<CT>(p[i]); }

template <bool RIGHT, typename TH, typename TD, typename TO, typename CT = float>
__device__ __forceinline__ void gemm_tile_mfma(const TH* __restrict__ H, int64_t L, int64_t n, int64_t Q,
                                               const TD* __restrict__ D, int64_t sDr, int64_t sDc, int ncols,
                                               const IndexMap& amap, const IndexMap& bmap, const HMap& hm,
                                               int64_t kchunk, TO* __restrict__ out, const OutLayout& ol,
                                               int64_t row0, int64_t c, int j0) {
  // operand and DRM entries of step s + 1 are loaded into registers (and the DRM rows
  // of step s + 2 computed) while step s is multiplied out of LDS
  using P = Pol<std::is_same_v<CT, double> ? TTNN_F64 : TTNN_F32>;
  constexpr int NA = BR * BK / 256, NB = BK * BJ / 256;
  __shared__ CT As[BK][BR + 4];
  __shared__ CT Bs[BK][BJ + 4];
  __shared__ int64_t drow[2][BK];

  const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int wave = tid >> 6;
  const int64_t rows_total = RIGHT ? n : L * Q;
  const int64_t K = RIGHT ? L * Q : n;
  const int64_t k_begin = c * kchunk;
  const int64_t k_end = (k_begin + kchunk < K) ? k_begin + kchunk : K;
  const bool kk_contig = RIGHT ? (L > 1) : (L == 1);
  typename P::CFrag acc[BJ / 16];
#pragma unroll
  for (int cb = 0; cb < BJ / 16; ++cb) acc[cb] = typename P::CFrag{};

  auto drm_row = [&](int64_t kk) -> int64_t {
    if (kk >= k_end) return -1;
    return RIGHT ? amap(kk % L) + bmap(kk / L) : amap(kk);
  };
  auto a_pos = [&](int e, int& kk, int& rr) {
    if (kk_contig) {
      kk = e % BK;
      rr = e / BK;
    } else {
      rr = e % BR;
      kk = e / BR;
    }
  };
  CT ra[NA], rb[NB];
  auto fetch = [&](int64_t kb, int buf) {
#pragma unroll
    for (int s = 0; s < NA; ++s) {
      int kk, rr;
      a_pos(tid + 256 * s, kk, rr);
      const int64_t kg = kb + kk;
      const int64_t rg = row0 + rr;
      CT v = 0;
      if (kg < k_end && rg < rows_total) {
        const int64_t m = RIGHT ? kg : rg;
        const int64_t i = RIGHT ? rg : kg;
        const int64_t l = m % L;
        const int64_t q = m / L;
        v = ldc<CT>(H, hm(l, i, q, L, n));
      }
      ra[s] = v;
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const int e = tid + 256 * s;
      const int jj = e % BJ;
      const int kk = e / BJ;
      const int64_t r = drow[buf][kk];
      rb[s] = (r >= 0 && j0 + jj < ncols) ? ldc<CT>(D, r * sDr + static_cast<int64_t>(j0 + jj) * sDc) : CT(0);
    }
  };

  if (tid < BK) {
    drow[0][tid] = drm_row(k_begin + tid);
    drow[1][tid] = drm_row(k_begin + BK + tid);
  }
  __syncthreads();
  if (k_begin < k_end) fetch(k_begin, 0);
  int buf = 0;
  for (int64_t kb = k_begin; kb < k_end; kb += BK) {
#pragma unroll
    for (int s = 0; s < NA; ++s) {
      int kk, rr;
      a_pos(tid + 256 * s, kk, rr);
      As[kk][rr] = ra[s];
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const int e = tid + 256 * s;
      Bs[e / BJ][e % BJ] = rb[s];
    }
    __syncthreads();
    // drow[buf] is free again (its step is staged): it takes the rows of step s + 2
    if (kb + BK < k_end) fetch(kb + BK, buf ^ 1);
    if (tid < BK) drow[buf][tid] = drm_row(kb + 2 * BK + tid);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const CT a = As[4 * s + lg][16 * wave + l16];
#pragma unroll
      for (int cb = 0; cb < BJ / 16; ++cb) acc[cb] = P::mfma(a, Bs[4 * s + lg][16 * cb + l16], acc[cb]);
    }
    __syncthreads();
    buf ^= 1;
  }

  // lane holds C[16 wave + crow(lane, v)][16 cb + l16]
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = row0 + 16 * wave + P::crow(lane, v);
    if (row >= rows_total) continue;
#pragma unroll
    for (int cb = 0; cb < BJ / 16; ++cb) {
      const int j = j0 + 16 * cb + l16;
      if (j >= ncols) continue;
      const int64_t o = c * ol.cs + (row % ol.Lo) * ol.s0 + static_cast<int64_t>(j) * ol.s1 +
                        (row / ol.Lo) * ol.s2;
      out[o] = static_cast<TO>(acc[cb][v]);
    }
  }
}

// FP32 / BF16 operands take the FP32 MFMA tile, anything with FP64 the FP64 MFMA tile.
template <bool RIGHT, typename TH, typename TD, typename TO>
__device__ __forceinline__ void gemm_tile(const TH* __restrict__ H, int64_t L, int64_t n, int64_t Q,
                                          const TD* __restrict__ D, int64_t sDr, int64_t sDc, int ncols,
                                          const IndexMap& amap, const IndexMap& bmap, const HMap& hm,
                                          int64_t kchunk, TO* __restrict__ out, const OutLayout& ol, int64_t row0,
                                          int64_t c, int j0) {
  if constexpr (!std::is_same_v<TH, double> && !std::is_same_v<TD, double>)
    gemm_tile_mfma<RIGHT, TH, TD, TO, float>(H, L, n, Q, D, sDr, sDc, ncols, amap, bmap, hm, kchunk, out, ol, row0,
                                             c, j0);
  else
    gemm_tile_mfma<RIGHT, TH, TD, TO, double>(H, L, n, Q, D, sDr, sDc, ncols, amap, bmap, hm, kchunk, out, ol, row0,
                                              c, j0);
}

template <bool RIGHT, typename TH, typename TD, typename TO>
__global__ __launch_bounds__(256) void hm_gemm(const TH* __restrict__ H, int64_t L, int64_t n, int64_t Q,
                                               const TD* __restrict__ D, int64_t sDr, int64_t sDc,
                                               int ncols, IndexMap amap, IndexMap bmap, HMap hm, int64_t kchunk,
                                               TO* __restrict__ out, OutLayout ol) {
  gemm_tile<RIGHT, TH, TD, TO>(H, L, n, Q, D, sDr, sDc, ncols, amap, bmap, hm, kchunk, out, ol,
                               static_cast<int64_t>(blockIdx.x) * BR, blockIdx.y, blockIdx.z * BJ);
}

// Copy a descriptor from global memory into LDS (8-byte words) after locating, by
// binary search on first_block, the task that owns this workgroup.
template <typename Task>
__device__ inline int64_t load_task(const Task* __restrict__ tasks, int ntasks, Task* t, int64_t b) {
  __shared__ int idx;
  if (threadIdx.x == 0) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (tasks[mid].first_block <= b) lo = mid;
      else hi = mid - 1;
    }
    idx = lo;
  }
  __syncthreads();
  static_assert(sizeof(Task) % 8 == 0, "task size");
  const uint64_t* src = reinterpret_cast<const uint64_t*>(tasks + idx);
  uint64_t* dst = reinterpret_cast<uint64_t*>(t);
  for (int w = threadIdx.x; w < static_cast<int>(sizeof(Task) / 8); w += blockDim.x) dst[w] = src[w];
  __syncthreads();
  return b - t->first_block;
}

// Every workgroup serves one tile of one task; tasks of one launch may belong to
// different updates (of different plans) and have different sizes.
// Tile b of a batched contraction launch (its task found by binary search).
template <bool RIGHT, typename TH, typename TD, typename TO>
__device__ __forceinline__ void gemm_task_tile(const GemmTask* __restrict__ tasks, int ntasks, int64_t b) {
  __shared__ __align__(16) char tbuf[sizeof(GemmTask)];      // raw storage: IndexMap has initialisers
  GemmTask& t = *reinterpret_cast<GemmTask*>(tbuf);
  int64_t rel = load_task(tasks, ntasks, &t, b);
  const int64_t rb = rel % t.row_blocks;
  rel /= t.row_blocks;
  const int64_t c = rel % t.nch;
  const int cb = static_cast<int>(rel / t.nch);
  gemm_tile<RIGHT, TH, TD, TO>(static_cast<const TH*>(t.H), t.L, t.n, t.Q, static_cast<const TD*>(t.D), t.sDr,
                               t.sDc, t.ncols, t.amap, t.bmap, t.hm, t.kchunk, static_cast<TO*>(t.out), t.ol,
                               rb * BR, c, cb * BJ);
}

template <bool RIGHT, typename TH, typename TD, typename TO>
__global__ __launch_bounds__(256) void hm_gemm_batched(const GemmTask* __restrict__ tasks, int ntasks) {
  gemm_task_tile<RIGHT, TH, TD, TO>(tasks, ntasks, static_cast<int64_t>(blockIdx.x));
}

template <bool RIGHT, typename TH, typename TD>
void gemm_dispatch_out(const GemmArgs& a, dim3 grid, int64_t kchunk, hipStream_t st) {
  if (a.out_f32)
    hipLaunchKernelGGL((hm_gemm<RIGHT, TH, TD, float>), grid, dim3(256), 0, st,
                       static_cast<const TH*>(a.H), a.L, a.n, a.Q, static_cast<const TD*>(a.D), a.sDr,
                       a.sDc, a.ncols, a.amap, a.bmap, a.hm, kchunk, static_cast<float*>(a.out), a.ol);
  else
    hipLaunchKernelGGL((hm_gemm<RIGHT, TH, TD, double>), grid, dim3(256), 0, st,
                       static_cast<const TH*>(a.H), a.L, a.n, a.Q, static_cast<const TD*>(a.D), a.sDr,
                       a.sDc, a.ncols, a.amap, a.bmap, a.hm, kchunk, static_cast<double*>(a.out), a.ol);
}

template <bool RIGHT, typename TH>
void gemm_dispatch_d(const GemmArgs& a, dim3 grid, int64_t kchunk, hipStream_t st) {
  switch (a.td) {
    case TTNN_F64: gemm_dispatch_out<RIGHT, TH, double>(a, grid, kchunk, st); break;
    case TTNN_F32: gemm_dispatch_out<RIGHT, TH, float>(a, grid, kchunk, st); break;
    default: gemm_dispatch_out<RIGHT, TH, uint16_t>(a, grid, kchunk, st); break;
  }
}

template <bool RIGHT>
void gemm_dispatch_h(const GemmArgs& a, dim3 grid, int64_t kchunk, hipStream_t st) {
  switch (a.th) {
    case TTNN_F64: gemm_dispatch_d<RIGHT, double>(a, grid, kchunk, st); break;
    case TTNN_F32: gemm_dispatch_d<RIGHT, float>(a, grid, kchunk, st); break;
    default: gemm_dispatch_d<RIGHT, uint16_t>(a, grid, kchunk, st); break;
  }
}

template <bool RIGHT, typename TH, typename TD>
void batched_dispatch_d(bool out_f32, const GemmTask* tasks, int nt, int64_t blocks, hipStream_t st) {
  if (out_f32)
    hipLaunchKernelGGL((hm_gemm_batched<RIGHT, TH, TD, float>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                       st, tasks, nt);
  else
    hipLaunchKernelGGL((hm_gemm_batched<RIGHT, TH, TD, double>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                       st, tasks, nt);
}
template <bool RIGHT, typename TH>
void batched_dispatch_h(int td, bool out_f32, const GemmTask* tasks, int nt, int64_t blocks, hipStream_t st) {
  switch (td) {
    case TTNN_F64: batched_dispatch_d<RIGHT, TH, double>(out_f32, tasks, nt, blocks, st); break;
    case TTNN_F32: batched_dispatch_d<RIGHT, TH, float>(out_f32, tasks, nt, blocks, st); break;
    default: batched_dispatch_d<RIGHT, TH, uint16_t>(out_f32, tasks, nt, blocks, st); break;
  }
}
template <bool RIGHT>
void batched_dispatch(int th, int td, bool out_f32, const GemmTask* tasks, int nt, int64_t blocks, hipStream_t st) {
  switch (th) {
    case TTNN_F64: batched_dispatch_h<RIGHT, double>(td, out_f32, tasks, nt, blocks, st); break;
    case TTNN_F32: batched_dispatch_h<RIGHT, float>(td, out_f32, tasks, nt, blocks, st); break;
    default: batched_dispatch_h<RIGHT, uint16_t>(td, out_f32, tasks, nt, blocks, st); break;
  }
}

// part[c * stride + e] summed over c in [c0, c1) in the order of c: the loads go out
// eight at a time with no dependence between them, the additions stay in order, so the
// sum is bitwise that of the plain loop.
__device__ __forceinline__ double sum_chunks(const double* __restrict__ part, int c0, int c1, int64_t stride,
                                             int64_t e) {
  double s = 0.0;
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = part[(c + i) * stride + e];
#pragma unroll
    for (int i = 0; i < 8; ++i) s += v[i];
  }
  for (; c < c1; ++c) s += part[c * stride + e];
  return s;
}

__device__ inline void reduce_range(const double* __restrict__ part, int nchunks, int64_t rows, int ncols, int mode,
                                    double alpha, const IndexMap& rmap, int64_t ldr, double* __restrict__ dst,
                                    int64_t L, int64_t kdim, int64_t start, int64_t step, int64_t stride) {
  const int64_t total = rows * ncols;
  for (int64_t e = start; e < total; e += step) {
    const int64_t row = e / ncols;
    const int j = static_cast<int>(e - row * ncols);
    const double s = sum_chunks(part, 0, nchunks, stride, e);
    if (mode == 0) {
      dst[rmap(row) + ldr * j] += alpha * s;
    } else {
      const int64_t o = (row % L) + L * (j + kdim * (row / L));
      if (mode == 1) dst[o] += alpha * s;
      else dst[o] = s;
    }
  }
}

__device__ __forceinline__ void reduce_task_tile(const ReduceTask* __restrict__ tasks, int ntasks, int64_t b) {
  __shared__ __align__(16) char tbuf[sizeof(ReduceTask)];
  ReduceTask& t = *reinterpret_cast<ReduceTask*>(tbuf);
  const int64_t rel = load_task(tasks, ntasks, &t, b);
  reduce_range(t.part, t.nchunks, t.rows, t.ncols, t.mode, t.alpha, t.rmap, t.ldr, t.dst, t.L, t.kdim,
               rel * 256 + threadIdx.x, t.nblocks * 256, t.cstride ? t.cstride : t.rows * t.ncols);
}

__global__ __launch_bounds__(256) void reduce_batched_kernel(const ReduceTask* __restrict__ tasks, int ntasks) {
  reduce_task_tile(tasks, ntasks, static_cast<int64_t>(blockIdx.x));
}

constexpr int kFold = 32;

// Fold groups of kFold consecutive chunks into each group's first slot (see
// fold_chunks_kernel); workgroup -> (task, element block, group).
__device__ __forceinline__ void fold_task_tile(const ReduceTask* __restrict__ tasks, int ntasks, int64_t b) {
  __shared__ __align__(16) char tbuf[sizeof(ReduceTask)];
  ReduceTask& t = *reinterpret_cast<ReduceTask*>(tbuf);
  const int64_t rel = load_task(tasks, ntasks, &t, b);
  const int64_t E = t.rows * t.ncols;
  const int64_t eblocks = (E + 255) / 256;
  const int64_t e = (rel % eblocks) * 256 + threadIdx.x;
  const int g = static_cast<int>(rel / eblocks);
  if (e >= E) return;
  const int c0 = g * kFold, c1 = c0 + kFold < t.nchunks ? c0 + kFold : t.nchunks;
  t.part[c0 * E + e] = sum_chunks(t.part, c0, c1, E, e);
}

__global__ __launch_bounds__(256) void fold_batched_kernel(const ReduceTask* __restrict__ tasks, int ntasks) {
  fold_task_tile(tasks, ntasks, static_cast<int64_t>(blockIdx.x));
}

// ---------------------------------------------------------------- persistent ingest
// One launch for a whole batched round of box updates: the workgroups sweep, phase by
// phase, every tile of every task list of the round (a level's contractions of all
// kinds, then its chunk folds, then its reductions, level after level) and meet at a
// grid-wide barrier between phases.  The tiles are those of the per-level launches, so
// results are bitwise the same.  Launched cooperatively (every workgroup resident), so
// each barrier ends; the wait is still bounded, and a wait that ran out marks the
// round's plans (their sticky numerical status).
struct IngestSeg {
  int64_t tasks;        // byte offset of the task table from the program
  int64_t blocks;
  int32_t kind, ntasks;
};
struct IngestPhase {
  IngestSeg seg[kIngestSegs];
  int32_t nseg, pad_;
};
struct IngestProgram {
  uint32_t counter;     // barrier arrivals (zero as staged)
  int32_t nphases, nsticky, pad_;
  int* sticky[kIngestPlans];
  IngestPhase ph[kIngestPhases];
};

__device__ inline bool grid_barrier(uint32_t* counter, uint32_t target) {
  __shared__ int ok;
  __syncthreads();                                     // the workgroup's writes are done
  if (threadIdx.x == 0) {
    __threadfence();                                   // ... and visible device-wide
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t spins = 0;
    ok = 1;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > (1u << 24)) {                      // ~1 s: cannot happen with resident workgroups
        ok = 0;
        break;
      }
    }
    __threadfence();                                   // later reads see the other workgroups' writes
  }
  __syncthreads();
  return ok != 0;
}

template <typename TC>
__global__ __launch_bounds__(256) void ingest_kernel(char* base) {
  IngestProgram* prog = reinterpret_cast<IngestProgram*>(base);
  uint32_t* counter = &prog->counter;
  const int nph = prog->nphases;
  for (int p = 0; p < nph; ++p) {
    const IngestPhase& P = prog->ph[p];
    int64_t total = 0;
    for (int s = 0; s < P.nseg; ++s) total += P.seg[s].blocks;
    for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
      int s = 0;
      int64_t rel = b;
      while (rel >= P.seg[s].blocks) rel -= P.seg[s++].blocks;
      const IngestSeg& g = P.seg[s];
      const void* tasks = base + g.tasks;
      switch (g.kind) {
        case kSegRightRaw:
          gemm_task_tile<true, TC, TC, double>(static_cast<const GemmTask*>(tasks), g.ntasks, rel);
          break;
        case kSegLeftRaw:
          gemm_task_tile<false, TC, TC, double>(static_cast<const GemmTask*>(tasks), g.ntasks, rel);
          break;
        case kSegRightF64:
          gemm_task_tile<true, double, double, double>(static_cast<const GemmTask*>(tasks), g.ntasks, rel);
          break;
        case kSegLeftF64:
          gemm_task_tile<false, double, double, double>(static_cast<const GemmTask*>(tasks), g.ntasks, rel);
          break;
        case kSegFold:
          fold_task_tile(static_cast<const ReduceTask*>(tasks), g.ntasks, rel);
          break;
        default:
          reduce_task_tile(static_cast<const ReduceTask*>(tasks), g.ntasks, rel);
          break;
      }
    }
    if (p + 1 < nph && !grid_barrier(counter, static_cast<uint32_t>(p + 1) * gridDim.x)) {
      if (threadIdx.x == 0)
        for (int i = 0; i < prog->nsticky; ++i) atomicOr(prog->sticky[i], 1);
      return;
    }
  }
}

__global__ void reduce_kernel(const double* __restrict__ part, int nchunks, int64_t rows, int ncols, int mode,
                              double alpha, IndexMap rmap, int64_t ldr, double* __restrict__ dst, int64_t L,
                              int64_t kdim, int64_t stride) {
  reduce_range(part, nchunks, rows, ncols, mode, alpha, rmap, ldr, dst, L, kdim,
               static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x,
               static_cast<int64_t>(gridDim.x) * blockDim.x, stride);
}

// Many chunks, few elements: fold each group of kFold consecutive chunks into the
// group's first chunk slot (in place, fixed order), so that the final pass sums
// ceil(nchunks / kFold) values per element.  Element e of group g is read and
// written by one thread only.
__global__ void fold_chunks_kernel(double* __restrict__ part, int nchunks, int64_t E) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (e >= E) return;
  const int c0 = g * kFold, c1 = c0 + kFold < nchunks ? c0 + kFold : nchunks;
  part[c0 * E + e] = sum_chunks(part, c0, c1, E, e);
}

__global__ void zero_kernel(double* p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}
__global__ void axpy_kernel(double* y, const double* x, double alpha, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] += alpha * x[i];
}
__global__ void copy_kernel(double* y, const double* x, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = x[i];
}
__global__ void f64_to_f32_kernel(float* y, const double* x, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = static_cast<float>(x[i]);
}
__global__ void zero_int_kernel(int* p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}
__global__ void finite_kernel(const double* p, int64_t n, int* flag) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (!isfinite(p[i])) *flag = 1;
}

// Block b of a list launch serves segment `seg` (blocks are dealt to segments in
// proportion to their length, at most kSegBlocks each).
constexpr int kSegBlocks = 512;
__device__ inline int seg_of(const SegList& s, int b, int* first) {
  int acc = 0;
  for (int i = 0; i < s.count; ++i) {
    int64_t nb = (s.n[i] + 255) / 256;
    if (nb > kSegBlocks) nb = kSegBlocks;
    if (nb < 1) nb = 1;
    if (b < acc + nb) {
      *first = acc;
      return i;
    }
    acc += static_cast<int>(nb);
  }
  *first = acc;
  return -1;
}
__global__ void zero_list_kernel(SegList s) {
  int first = 0;
  const int i = seg_of(s, blockIdx.x, &first);
  if (i < 0) return;
  int64_t nb = (s.n[i] + 255) / 256;
  nb = nb > kSegBlocks ? kSegBlocks : (nb < 1 ? 1 : nb);
  for (int64_t e = static_cast<int64_t>(blockIdx.x - first) * 256 + threadIdx.x; e < s.n[i]; e += nb * 256)
    s.p[i][e] = 0.0;
}
__global__ void finite_list_kernel(SegList s, int* flag) {
  int first = 0;
  const int i = seg_of(s, blockIdx.x, &first);
  if (i < 0) return;
  int64_t nb = (s.n[i] + 255) / 256;
  nb = nb > kSegBlocks ? kSegBlocks : (nb < 1 ? 1 : nb);
  for (int64_t e = static_cast<int64_t>(blockIdx.x - first) * 256 + threadIdx.x; e < s.n[i]; e += nb * 256)
    if (!isfinite(s.p[i][e])) *flag = 1;
}

inline bool fold_pays(int nchunks, int64_t E) { return nchunks > 2 * kFold && E < (int64_t(1) << 20); }

inline int grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return static_cast<int>(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

int pick_chunks(int64_t rows, int ncols, int64_t K, size_t partial_cap) {
  const int64_t row_blocks = (rows + BR - 1) / BR;
  const int64_t col_blocks = (ncols + BJ - 1) / BJ;
  const int64_t blocks = row_blocks * col_blocks;
  int64_t want = 2048 / (blocks > 0 ? blocks : 1);
  const int64_t by_len = (K + 127) / 128;              // at least ~128 terms per chunk
  if (want > by_len) want = by_len;
  const int64_t cap = static_cast<int64_t>(partial_cap / static_cast<size_t>(rows * ncols));
  if (want > cap) want = cap;
  if (want > 65535) want = 65535;
  return static_cast<int>(want < 1 ? 1 : want);
}

int gemm_chunks(const GemmArgs& a, int64_t* kchunk_out) {
  const int64_t rows = a.right ? a.n : a.L * a.Q;
  const int64_t K = a.right ? a.L * a.Q : a.n;
  if (rows <= 0 || a.ncols <= 0) return 0;
  int64_t kchunk = (K + a.nchunks - 1) / a.nchunks;
  kchunk = ((kchunk + BK - 1) / BK) * BK;
  if (kchunk < BK) kchunk = BK;
  const int nch = static_cast<int>((K + kchunk - 1) / kchunk);
  if (kchunk_out) *kchunk_out = kchunk;
  return nch > 0 ? nch : 1;
}

int launch_gemm(const GemmArgs& a, hipStream_t st) {
  int64_t kchunk = 0;
  const int nch = gemm_chunks(a, &kchunk);
  if (nch == 0) return 0;
  const int64_t rows = a.right ? a.n : a.L * a.Q;
  dim3 grid(static_cast<unsigned>((rows + BR - 1) / BR), static_cast<unsigned>(nch),
            static_cast<unsigned>((a.ncols + BJ - 1) / BJ));
  if (a.right) gemm_dispatch_h<true>(a, grid, kchunk, st);
  else gemm_dispatch_h<false>(a, grid, kchunk, st);
  return nch;
}

BatchedGemm plan_gemm_batched(const std::vector<GemmArgs>& args) {
  BatchedGemm b;
  if (args.empty()) return b;
  b.right = args[0].right;
  b.th = args[0].th;
  b.td = args[0].td;
  b.out_f32 = args[0].out_f32;
  b.tasks.reserve(args.size());
  for (const GemmArgs& a : args) {
    TTNN_REQUIRE(a.right == b.right && a.th == b.th && a.td == b.td && a.out_f32 == b.out_f32, TTNN_E_INVALID,
                 "batched contraction with mixed kinds");
    GemmTask t{};
    const int nch = gemm_chunks(a, &t.kchunk);
    if (nch == 0) continue;
    const int64_t rows = a.right ? a.n : a.L * a.Q;
    t.H = a.H;
    t.D = a.D;
    t.out = a.out;
    t.L = a.L;
    t.n = a.n;
    t.Q = a.Q;
    t.sDr = a.sDr;
    t.sDc = a.sDc;
    t.ncols = a.ncols;
    t.amap = a.amap;
    t.bmap = a.bmap;
    t.hm = a.hm;
    t.ol = a.ol;
    t.row_blocks = (rows + BR - 1) / BR;
    t.nch = nch;
    t.col_blocks = (a.ncols + BJ - 1) / BJ;
    t.first_block = b.blocks;
    b.blocks += t.row_blocks * t.nch * t.col_blocks;
    b.tasks.push_back(t);
  }
  TTNN_REQUIRE(b.blocks < (int64_t(1) << 31), TTNN_E_INVALID, "batched launch too large");
  return b;
}

void launch_gemm_staged(const BatchedGemm& b, const GemmTask* d, hipStream_t st) {
  if (b.tasks.empty()) return;
  const int nt = static_cast<int>(b.tasks.size());
  if (b.right) batched_dispatch<true>(b.th, b.td, b.out_f32, d, nt, b.blocks, st);
  else batched_dispatch<false>(b.th, b.td, b.out_f32, d, nt, b.blocks, st);
}

void launch_gemm_batched(const std::vector<GemmArgs>& args, hipStream_t st) {
  const BatchedGemm b = plan_gemm_batched(args);
  if (b.tasks.empty()) return;
  StagingLock lock;
  const GemmTask* d =
      static_cast<const GemmTask*>(stage_descriptors(b.tasks.data(), b.tasks.size() * sizeof(GemmTask), st));
  launch_gemm_staged(b, d, st);
  fence_descriptors(st);
}

BatchedReduce plan_reduce_batched(const std::vector<ReduceTask>& in) {
  // the same two passes as launch_reduce, so batched and single results are bitwise equal
  BatchedReduce b;
  for (ReduceTask t : in) {
    if (t.rows <= 0 || t.ncols <= 0 || t.nchunks <= 0) continue;
    const int64_t E = t.rows * t.ncols;
    if (fold_pays(t.nchunks, E)) {
      ReduceTask f = t;
      f.groups = (t.nchunks + kFold - 1) / kFold;
      f.first_block = b.fblocks;
      b.fblocks += (E + 255) / 256 * f.groups;
      b.folds.push_back(f);
      t.nchunks = f.groups;
      t.cstride = E * kFold;
    }
    t.nblocks = grid_for(E);
    t.first_block = b.blocks;
    b.blocks += t.nblocks;
    b.tasks.push_back(t);
  }
  TTNN_REQUIRE(b.fblocks < (int64_t(1) << 31) && b.blocks < (int64_t(1) << 31), TTNN_E_INVALID,
               "batched launch too large");
  return b;
}

void launch_reduce_staged(const BatchedReduce& b, const ReduceTask* dfolds, const ReduceTask* dtasks,
                          hipStream_t st) {
  if (b.tasks.empty()) return;
  if (!b.folds.empty())
    hipLaunchKernelGGL(fold_batched_kernel, dim3(static_cast<unsigned>(b.fblocks)), dim3(256), 0, st, dfolds,
                       static_cast<int>(b.folds.size()));
  hipLaunchKernelGGL(reduce_batched_kernel, dim3(static_cast<unsigned>(b.blocks)), dim3(256), 0, st, dtasks,
                     static_cast<int>(b.tasks.size()));
}

void launch_reduce_batched(const std::vector<ReduceTask>& in, hipStream_t st) {
  const BatchedReduce b = plan_reduce_batched(in);
  if (b.tasks.empty()) return;
  StagingLock lock;
  const ReduceTask* df = nullptr;
  if (!b.folds.empty())
    df = static_cast<const ReduceTask*>(stage_descriptors(b.folds.data(), b.folds.size() * sizeof(ReduceTask), st));
  const ReduceTask* dt =
      static_cast<const ReduceTask*>(stage_descriptors(b.tasks.data(), b.tasks.size() * sizeof(ReduceTask), st));
  launch_reduce_staged(b, df, dt, st);
  fence_descriptors(st);
}

void launch_reduce(double* part, int nchunks, int64_t rows, int ncols, int mode, double alpha,
                   const IndexMap& rmap, int64_t ldr, double* dst, int64_t L, int64_t kdim, hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return;
  const int64_t E = rows * ncols;
  int64_t stride = E;
  if (fold_pays(nchunks, E)) {
    const int groups = (nchunks + kFold - 1) / kFold;
    hipLaunchKernelGGL(fold_chunks_kernel, dim3(static_cast<unsigned>((E + 255) / 256), groups), dim3(256), 0, st,
                       part, nchunks, E);
    nchunks = groups;
    stride = E * kFold;
  }
  hipLaunchKernelGGL(reduce_kernel, dim3(grid_for(E)), dim3(256), 0, st, part, nchunks, rows, ncols, mode, alpha,
                     rmap, ldr, dst, L, kdim, stride);
}

void launch_zero(double* p, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}
void launch_axpy(double* y, const double* x, double alpha, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n)), dim3(256), 0, st, y, x, alpha, n);
}
void launch_copy_f64(double* y, const double* x, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, st, y, x, n);
}
void launch_f64_to_f32(float* y, const double* x, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(f64_to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, st, y, x, n);
}
void launch_zero_int(int* p, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(zero_int_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}
static int list_blocks(const SegList& s) {
  int64_t b = 0;
  for (int i = 0; i < s.count; ++i) {
    int64_t nb = (s.n[i] + 255) / 256;
    b += nb > kSegBlocks ? kSegBlocks : (nb < 1 ? 1 : nb);
  }
  return static_cast<int>(b);
}
void launch_zero_list(const SegList& s, hipStream_t st) {
  if (s.count > 0) hipLaunchKernelGGL(zero_list_kernel, dim3(list_blocks(s)), dim3(256), 0, st, s);
}
void launch_finite_list(const SegList& s, int* flag, hipStream_t st) {
  if (s.count > 0) hipLaunchKernelGGL(finite_list_kernel, dim3(list_blocks(s)), dim3(256), 0, st, s, flag);
}

void launch_finite_check(const double* p, int64_t n, int* flag, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(finite_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, flag);
}

// ---------------------------------------------------------------- persistent ingest (host)
namespace {
template <typename TC>
int ingest_grid(int64_t want) {
  static std::mutex mu;
  static std::map<int, int> slots;              // device -> resident workgroups of the kernel
  int dev = 0;
  TTNN_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = slots.find(dev);
  if (it == slots.end()) {
    int coop = 0, cus = 0, per = 0;
    TTNN_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    TTNN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    TTNN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(ingest_kernel<TC>),
                                                            256, 0));
    it = slots.emplace(dev, coop ? per * cus : 0).first;
  }
  if (it->second <= 0) return 0;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, it->second)));
}
}  // namespace

bool launch_ingest(int cd, const std::vector<BatchedGemm>& gl, const std::vector<size_t>& level_end,
                   const std::vector<BatchedReduce>& rl, const std::vector<int*>& sticky, hipStream_t st) {
  if (sticky.size() > static_cast<size_t>(kIngestPlans)) return false;
  std::vector<IngestPhase> phases;
  // task tables follow the program, each 64-byte aligned
  const size_t head = (sizeof(IngestProgram) + 63) / 64 * 64;
  std::vector<std::pair<const void*, size_t>> tables;     // (host data, bytes)
  size_t off = head;
  auto add_table = [&](const void* data, size_t bytes) {
    const size_t at = off;
    tables.emplace_back(data, bytes);
    off = (off + bytes + 63) / 64 * 64;
    return static_cast<int64_t>(at);
  };
  int64_t most = 0;
  size_t g0 = 0;
  for (size_t lv = 0; lv < rl.size(); ++lv) {
    IngestPhase ph{};
    for (size_t k = g0; k < level_end[lv]; ++k) {
      const BatchedGemm& b = gl[k];
      if (b.tasks.empty()) continue;
      if (b.out_f32 || ph.nseg == kIngestSegs) return false;
      int kind;
      if (b.th == cd && b.td == cd) kind = b.right ? kSegRightRaw : kSegLeftRaw;
      else if (b.th == TTNN_F64 && b.td == TTNN_F64) kind = b.right ? kSegRightF64 : kSegLeftF64;
      else return false;
      IngestSeg& g = ph.seg[ph.nseg++];
      g.kind = kind;
      g.ntasks = static_cast<int32_t>(b.tasks.size());
      g.blocks = b.blocks;
      g.tasks = add_table(b.tasks.data(), b.tasks.size() * sizeof(GemmTask));
    }
    g0 = level_end[lv];
    auto push = [&](IngestPhase& q) {
      if (q.nseg == 0) return;
      int64_t t = 0;
      for (int i = 0; i < q.nseg; ++i) t += q.seg[i].blocks;
      most = std::max(most, t);
      phases.push_back(q);
    };
    push(ph);
    const BatchedReduce& r = rl[lv];
    if (!r.folds.empty()) {
      IngestPhase f{};
      f.nseg = 1;
      f.seg[0] = IngestSeg{add_table(r.folds.data(), r.folds.size() * sizeof(ReduceTask)), r.fblocks, kSegFold,
                           static_cast<int32_t>(r.folds.size())};
      push(f);
    }
    if (!r.tasks.empty()) {
      IngestPhase q{};
      q.nseg = 1;
      q.seg[0] = IngestSeg{add_table(r.tasks.data(), r.tasks.size() * sizeof(ReduceTask)), r.blocks, kSegReduce,
                           static_cast<int32_t>(r.tasks.size())};
      push(q);
    }
  }
  if (phases.empty()) return true;
  if (phases.size() > static_cast<size_t>(kIngestPhases)) return false;
  const int grid = cd == TTNN_BF16 ? ingest_grid<uint16_t>(most)
                   : cd == TTNN_F32 ? ingest_grid<float>(most)
                                    : ingest_grid<double>(most);
  if (grid <= 0) return false;
  std::vector<char> host(off, 0);
  IngestProgram* prog = reinterpret_cast<IngestProgram*>(host.data());
  prog->counter = 0;
  prog->nphases = static_cast<int32_t>(phases.size());
  prog->nsticky = static_cast<int32_t>(sticky.size());
  for (size_t i = 0; i < sticky.size(); ++i) prog->sticky[i] = sticky[i];
  for (size_t i = 0; i < phases.size(); ++i) prog->ph[i] = phases[i];
  size_t at = head;
  for (auto& t : tables) {
    std::memcpy(host.data() + at, t.first, t.second);
    at = (at + t.second + 63) / 64 * 64;
  }
  StagingLock lock;
  char* d = static_cast<char*>(stage_descriptors(host.data(), host.size(), st));
  void* args[] = {&d};
  hipError_t e;
  if (cd == TTNN_BF16)
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(ingest_kernel<uint16_t>), dim3(grid), dim3(256),
                                   args, 0, st);
  else if (cd == TTNN_F32)
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(ingest_kernel<float>), dim3(grid), dim3(256), args,
                                   0, st);
  else
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(ingest_kernel<double>), dim3(grid), dim3(256),
                                   args, 0, st);
  TTNN_HIP(e);
  fence_descriptors(st);
  return true;
}

}  // namespace ttnn
