// Rank-1 updates H = a_1 o a_2 o ... o a_d (streaming by linearity, Sec. 4).
//
// Every sketch of a rank-1 tensor factorises.  With u_I = kron of the factors of a
// mode group I (first mode fastest):
//   T^{(t)} = u_{I_t} u_{D\I_t}^T,  so  R_t = u_{I_t} (X_t^T u_{rows of X_t})^T;
// for STTNN the rows of X_t run over contracted groups s, whose factor becomes
// g_s = Y_s^T u_{I_s}; the root sketch is kron_c g_c.  Each product X^T u is a
// GEMV whose vector is never formed: the weight of a row is the product of one
// factor entry per position, read from the row's mixed-radix digits.
#include "kernels.hpp"

namespace ttnn {
namespace {

constexpr int kThreadsR = 256;
constexpr int kFacCache = 1024;   // factor entries kept in LDS by the GEMV (8 KB)

__device__ inline double kron_weight(const KronVec& kv, int64_t row) {
  double w = 1.0;
  for (int p = 0; p < kv.n; ++p) {
    const int64_t e = kv.len[p];
    const int64_t i = row % e;
    row /= e;
    w *= kv.v[p][i];
  }
  return w;
}

// partial[b][j] = sum over the rows of block b of D[row * ncols + j] * weight(row).  The
// block's rows are contiguous in D: each step copies RB of them into LDS with 16-byte
// loads (consecutive threads, consecutive vectors; rows padded by one element against
// bank conflicts), then one lane per row forms the row's weight and accumulates its
// ncols products in FP64 (NC >= ncols accumulators a lane); a fixed-order reduction
// over the lanes (shuffles, then the waves in order) ends the block.  A lane's row
// advances by RB a step, so its mixed-radix digits (one per factor) advance by the
// digits of RB with one carry test each instead of a division per factor and row.
// rows_per_block is a multiple of RB, so every step but the block's last is whole.
// Blocks: the chunks of rows, padded to a multiple of 8, times the terms; block b takes
// chunk x and term y with the terms of one chunk 8 blocks apart (the same XCD, dispatched
// together), x = 8 (b / 8m) + b % 8, y = (b % 8m) / 8.  Term y writes partial[y nb + x].
template <typename TD, int NC, typename DI>
__global__ __launch_bounds__(kThreadsR) void kron_gemv_kernel(const TD* __restrict__ D, int64_t rows, int ncols,
                                                              KronBatch kb, int64_t rows_per_block, int64_t nb,
                                                              double* __restrict__ partial) {
  const int64_t bx = blockIdx.x, g8 = 8 * static_cast<int64_t>(kb.m);
  const int64_t chunk = 8 * (bx / g8) + bx % 8;
  const int term = static_cast<int>((bx % g8) / 8);
  if (chunk >= nb) return;                 // padding chunks (whole block, before any barrier)
  const KronVec& kv = kb.kv[term];
  partial += static_cast<int64_t>(term) * nb * ncols;
  constexpr int RB = sizeof(TD) == 8 ? kThreadsR / 2 : kThreadsR;     // rows a step (LDS <= 66 KB)
  constexpr int V = 16 / static_cast<int>(sizeof(TD));                // elements a 16-byte load
  constexpr int PER = (NC * RB + kThreadsR * V - 1) / (kThreadsR * V);  // loads a thread a step
  typedef TD vec_t __attribute__((ext_vector_type(V)));
  __shared__ TD tile[RB * (NC + 1)];
  __shared__ double red[kThreadsR / 64][NC];
  __shared__ double fac[kFacCache];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the factors in LDS when they fit (the usual case: a few hundred entries), so that the
  // weights never wait on global memory: a wait for a global gather issued after the
  // next step's loads would also wait for those loads (the counter is in order)
  int foff[kMaxPos];
  bool cached;
  {
    int64_t tot = 0;
    for (int p = 0; p < kv.n; ++p) {
      foff[p] = static_cast<int>(tot < kFacCache ? tot : 0);
      tot += kv.len[p];
    }
    cached = tot <= kFacCache;
    if (cached)
      for (int p = 0; p < kv.n; ++p)
        for (int64_t i = tid; i < kv.len[p]; i += kThreadsR) fac[foff[p] + i] = kv.v[p][i];
    __syncthreads();
  }
  const int64_t r0 = chunk * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  const int ld = ncols + 1;
  // (row, column) of this thread's first element of each load, and the stride between
  // its loads (kThreadsR * V elements)
  const int x0 = tid * V;
  const int row0 = x0 / ncols, col0 = x0 - row0 * ncols;
  const int dr = (kThreadsR * V) / ncols, dc = (kThreadsR * V) % ncols;
  // digits of this lane's first row and of the step (DI: 32-bit when every factor is
  // shorter than 2^30, so that a digit plus a step digit plus a carry cannot overflow)
  DI dig[kMaxPos], stp[kMaxPos];
  {
    int64_t a = r0 + tid, b = RB;
    for (int p = 0; p < kv.n; ++p) {
      const int64_t e = kv.len[p];
      dig[p] = static_cast<DI>(a % e);
      a /= e;
      stp[p] = static_cast<DI>(b % e);
      b /= e;
    }
  }
  double acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = 0.0;
  vec_t v[PER];
  auto fetch = [&](int64_t b) {            // the step's loads, all in flight together
    const int64_t nr = r1 - b < RB ? r1 - b : RB;
    const TD* src = D + b * ncols;
    if (nr == RB) {
      // a whole step: RB * ncols elements, a multiple of V, 16-byte aligned (RB rows);
      // one predicated vector load each, no dependence between them
      const int total = RB * ncols;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = (tid + k * kThreadsR) * V;
        v[k] = e < total ? *reinterpret_cast<const vec_t*>(src + e) : vec_t{};
      }
    } else {
      // the block's last, partial step: element by element
      const int total = static_cast<int>(nr) * ncols;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = (tid + k * kThreadsR) * V;
        vec_t t{};
#pragma unroll
        for (int i = 0; i < V; ++i)
          if (e + i < total) t[i] = src[e + i];
        v[k] = t;
      }
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t base = r0; base < r1; base += RB) {
    const int nr = static_cast<int>(r1 - base < RB ? r1 - base : RB);
    const int total = nr * ncols;
    int rr = row0, cc = col0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = (tid + k * kThreadsR) * V;
      int r = rr, c = cc;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        if (e + i < total) tile[r * ld + c] = v[k][i];
        if (++c == ncols) {
          c = 0;
          ++r;
        }
      }
      rr += dr;
      cc += dc;
      if (cc >= ncols) {
        cc -= ncols;
        ++rr;
      }
    }
    __syncthreads();
    if (base + RB < r1) fetch(base + RB);  // next step's loads overlap this step's products
    if (tid < nr) {
      double w = 1.0;
      if (cached)
        for (int p = 0; p < kv.n; ++p) w *= fac[foff[p] + dig[p]];
      else
        for (int p = 0; p < kv.n; ++p) w *= kv.v[p][dig[p]];
      const TD* q = tile + tid * ld;
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (j < ncols) acc[j] += to_f64(q[j]) * w;
    }
    DI carry = 0;                            // row += RB in mixed radix
    for (int p = 0; p < kv.n; ++p) {
      const DI x = dig[p] + stp[p] + carry;
      const DI e = static_cast<DI>(kv.len[p]);
      carry = x >= e;
      dig[p] = carry ? x - e : x;
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    double x = acc[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) red[wave][j] = x;
  }
  __syncthreads();
  if (tid < ncols) {
    double s = red[0][tid];
#pragma unroll
    for (int q = 1; q < kThreadsR / 64; ++q) s += red[q][tid];
    partial[chunk * ncols + tid] = s;
  }
}

template <typename TD, typename DI>
void launch_gemv_di(const TD* D, int64_t rows, int ncols, const KronBatch& kb, int64_t per, int64_t nb, dim3 grid,
                    double* partial, hipStream_t st) {
#define TTNN_GEMV(NCV) \
  hipLaunchKernelGGL((kron_gemv_kernel<TD, NCV, DI>), grid, dim3(kThreadsR), 0, st, D, rows, ncols, kb, per, nb, partial)
  if (ncols <= 8) TTNN_GEMV(8);
  else if (ncols <= 16) TTNN_GEMV(16);
  else if (ncols <= 24) TTNN_GEMV(24);
  else if (ncols <= 32) TTNN_GEMV(32);
  else if (ncols <= 48) TTNN_GEMV(48);
  else TTNN_GEMV(64);
#undef TTNN_GEMV
}

template <typename TD>
void launch_gemv_dt(const TD* D, int64_t rows, int ncols, const KronBatch& kb, int64_t per, int64_t nb, dim3 grid,
                    double* partial, hipStream_t st) {
  bool short_factors = true;
  for (int y = 0; y < kb.m; ++y)
    for (int p = 0; p < kb.kv[y].n; ++p) short_factors = short_factors && kb.kv[y].len[p] < (int64_t(1) << 30);
  if (short_factors) launch_gemv_di<TD, int>(D, rows, ncols, kb, per, nb, grid, partial, st);
  else launch_gemv_di<TD, int64_t>(D, rows, ncols, kb, per, nb, grid, partial, st);
}

// w[y wstride + j] = sum_b partial[y nb + b][j]: one wave per (column, term), lane l
// summing blocks l, l + 64, .. in order, the 64 sums combined by a fixed butterfly
__global__ __launch_bounds__(64) void sum_blocks_kernel(const double* __restrict__ partial, int nb, int ncols,
                                                        double* __restrict__ w, int64_t wstride) {
  const int j = blockIdx.x, y = blockIdx.y, l = threadIdx.x;
  const double* p = partial + static_cast<int64_t>(y) * nb * ncols;
  double s = 0.0;
  for (int b = l; b < nb; b += 64) s += p[static_cast<int64_t>(b) * ncols + j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (l == 0) w[y * wstride + j] = s;
}

// R[i + n j] += alpha_y * weight_y(i) * (w ? w[y wstride + j] : 1), the terms in order
__global__ void outer_acc_kernel(double* __restrict__ R, int64_t n, int ncols, KronBatch ku,
                                 const double* __restrict__ w, int64_t wstride) {
  const int64_t total = n * ncols;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = e % n;
    const int64_t j = e / n;
    double r = R[e];
    for (int y = 0; y < ku.m; ++y) {
      const double wj = w ? w[y * wstride + j] : 1.0;
      r += ku.alpha[y] * kron_weight(ku.kv[y], i) * wj;
    }
    R[e] = r;
  }
}

}  // namespace

void launch_kron_gemv(const void* D, int dt, int64_t rows, int ncols, const KronBatch& kb, double* partial,
                      size_t partial_elems, double* w, int64_t wstride, hipStream_t st) {
  if (ncols <= 0 || kb.m <= 0) return;
  TTNN_REQUIRE(ncols <= 64, TTNN_E_INVALID, "rank-1 update with more than 64 map columns");
  TTNN_REQUIRE(kb.m <= kRank1Batch, TTNN_E_INVALID, "too many rank-1 terms in one launch");
  // >= 512 rows a block, at most 2048 blocks a term; the chunking depends on rows and
  // ncols only, never on the batch, so a term's sums are the same in any batch
  int64_t nb = (rows + 511) / 512;
  if (nb < 1) nb = 1;
  if (nb > 2048) nb = 2048;
  const int64_t cap = static_cast<int64_t>(partial_elems / (static_cast<size_t>(ncols) * kRank1Batch));
  if (nb > cap) nb = cap;
  TTNN_REQUIRE(nb >= 1, TTNN_E_INVALID, "rank-1 scratch too small");
  // rows a block: a multiple of the kernel's step (128 rows for FP64 maps, else 256)
  const int64_t rb = dt == TTNN_F64 ? kThreadsR / 2 : kThreadsR;
  int64_t per = (rows + nb - 1) / nb;
  per = (per + rb - 1) / rb * rb;
  if (per < rb) per = rb;
  nb = rows > 0 ? (rows + per - 1) / per : 1;
  const int64_t padded = (nb + 7) / 8 * 8;             // chunks padded to the XCD count
  const dim3 grid(static_cast<unsigned>(padded * kb.m));
  if (dt == TTNN_F64)
    launch_gemv_dt(static_cast<const double*>(D), rows, ncols, kb, per, nb, grid, partial, st);
  else if (dt == TTNN_F32)
    launch_gemv_dt(static_cast<const float*>(D), rows, ncols, kb, per, nb, grid, partial, st);
  else
    launch_gemv_dt(static_cast<const uint16_t*>(D), rows, ncols, kb, per, nb, grid, partial, st);
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(ncols, kb.m), dim3(64), 0, st, partial, static_cast<int>(nb), ncols, w,
                     wstride);
}

void launch_outer_acc(double* R, int64_t n, int ncols, const KronBatch& ku, const double* w, int64_t wstride,
                      hipStream_t st) {
  const int64_t total = n * ncols;
  if (total <= 0 || ku.m <= 0) return;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(outer_acc_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, R, n, ncols, ku, w,
                     wstride);
}

}  // namespace ttnn
