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
#include "mfma.hpp"

namespace ttnn {
namespace {

constexpr int kThreadsR = 256;
constexpr int kFacCache = 2048;   // factor entries of a term group kept in LDS by the GEMV (16 KB)

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

// partial[(y nb + b) ncols + j] = sum over the rows of block b of D[row * ncols + j] *
// weight_y(row), for the terms y of the batch.  The block's rows are contiguous in D:
// each step copies RB of them into LDS with 16-byte loads (rows padded by one element
// against bank conflicts); two lanes take a row, each half of its columns (NCH), two rows
// RH apart a step, and accumulate the products with the weights of up to MT terms in
// FP64, so one staged row serves every term of the block's group; a fixed-order reduction (shuffles over the
// lanes of a half, then the waves in order) ends the block.  A term's sums depend only
// on its own weights and on the row partition, which the batch does not change, so its
// result is bitwise the same in any batch.  A lane's row advances by RH at a time, so
// its mixed-radix digits (one per factor) advance by the digits of RH with one carry
// test each.  Blocks: the chunks of rows, padded to a multiple of 8, times the groups of MT
// terms, the groups of one chunk 8 blocks apart (the same XCD, dispatched together):
// block b takes chunk x = 8 (b / 8G) + b % 8 and group (b % 8G) / 8.  rows_per_block is
// a multiple of RB, so every step but the block's last is whole.
template <typename TD, int NCH, int MT, typename DI>
__global__ __launch_bounds__(kThreadsR) void kron_gemv_kernel(const TD* __restrict__ D, int64_t rows, int ncols,
                                                              KronBatch kb, int64_t rows_per_block, int64_t nb,
                                                              double* __restrict__ partial) {
  constexpr int NC = 2 * NCH;
  constexpr int RH = kThreadsR / 2;                                   // rows at once: two lanes a row
  constexpr int RB = 2 * RH;                                          // rows a step: two rows a lane pair
  constexpr int V = 16 / static_cast<int>(sizeof(TD));                // elements a 16-byte load
  constexpr int PER = (NC * RB + kThreadsR * V - 1) / (kThreadsR * V);  // loads a thread a step
  typedef TD vec_t __attribute__((ext_vector_type(V)));
  __shared__ __align__(16) TD tile[RB * (NC + 1)];
  __shared__ double red[kThreadsR / 64][MT][NC];
  __shared__ double fac[kFacCache];
  const int G = (kb.m + MT - 1) / MT;
  const int64_t bx = blockIdx.x, g8 = 8 * static_cast<int64_t>(G);
  const int64_t chunk = 8 * (bx / g8) + bx % 8;
  const int t0 = MT * static_cast<int>((bx % g8) / 8);                 // first term of the group
  if (chunk >= nb) return;                 // padding chunks (whole block, before any barrier)
  const int mg = kb.m - t0 < MT ? kb.m - t0 : MT;                     // terms of the group
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = tid >> 1, half = tid & 1;
  const int64_t r0 = chunk * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  const int ld = ncols + 1;
  const KronVec& k0 = kb.kv[0];            // every term has the same factor lengths
  const int np = k0.n;
  // the group's factors in LDS when they fit (the usual case: a few hundred entries a
  // term), so that the weights never wait on global memory: a wait for a global gather
  // issued after the next step's loads would also wait for those loads (the counter is
  // in order).  Every loop over the factor positions runs to the compile-time maximum
  // with a guard, so that these small arrays stay in registers.
  int foff[kMaxPos];
  int64_t flen = 0;
#pragma unroll
  for (int p = 0; p < kMaxPos; ++p) {
    foff[p] = static_cast<int>(flen < kFacCache ? flen : 0);
    if (p < np) flen += k0.len[p];
  }
  const bool cached = flen * mg <= kFacCache;
  if (cached)
    for (int y = 0; y < mg; ++y)
#pragma unroll
      for (int p = 0; p < kMaxPos; ++p)
        if (p < np)
          for (int64_t i = tid; i < k0.len[p]; i += kThreadsR) fac[y * flen + foff[p] + i] = kb.kv[t0 + y].v[p][i];
  // (row, column) of this thread's first element of each load, and the stride between
  // its loads (kThreadsR * V elements)
  const int x0 = tid * V;
  const int row0 = x0 / ncols, col0 = x0 - row0 * ncols;
  const int dr = (kThreadsR * V) / ncols, dc = (kThreadsR * V) % ncols;
  // digits of this lane's first row and of RH (a lane pair takes rows RH apart)
  DI dig[kMaxPos], stp[kMaxPos], len[kMaxPos];
  {
    int64_t a = r0 + row, b = RH;
#pragma unroll
    for (int p = 0; p < kMaxPos; ++p) {
      const int64_t e = p < np ? k0.len[p] : 1;
      len[p] = static_cast<DI>(e);
      dig[p] = static_cast<DI>(a % e);
      a /= e;
      stp[p] = static_cast<DI>(b % e);
      b /= e;
    }
  }
  double acc[MT][NCH];
#pragma unroll
  for (int y = 0; y < MT; ++y)
#pragma unroll
    for (int j = 0; j < NCH; ++j) acc[y][j] = 0.0;
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
  __syncthreads();                              // the factor cache is written
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
#pragma unroll
    for (int h = 0; h < 2; ++h) {
    const int rl = row + h * RH;               // this pair's row within the step
    if (rl < nr) {
      double w[MT];
#pragma unroll
      for (int y = 0; y < MT; ++y) {
        w[y] = 1.0;
        if (y < mg) {
          if (cached) {
            const int fb = y * static_cast<int>(flen);
#pragma unroll
            for (int p = 0; p < kMaxPos; ++p)
              if (p < np) w[y] *= fac[fb + foff[p] + static_cast<int>(dig[p])];
          } else {
#pragma unroll
            for (int p = 0; p < kMaxPos; ++p)
              if (p < np) w[y] *= kb.kv[t0 + y].v[p][dig[p]];
          }
        }
      }
      const TD* q = tile + rl * ld + half * NCH;
#pragma unroll
      for (int j = 0; j < NCH; ++j)
        if (half * NCH + j < ncols) {
          const double x = to_f64(q[j]);
#pragma unroll
          for (int y = 0; y < MT; ++y)
            if (y < mg) acc[y][j] += x * w[y];
        }
    }
    DI carry = 0;                            // row += RH in mixed radix
#pragma unroll
    for (int p = 0; p < kMaxPos; ++p) {
      const DI x = dig[p] + stp[p] + carry;
      carry = x >= len[p];
      dig[p] = carry ? x - len[p] : x;
    }
    }
    __syncthreads();
  }
  // the lanes of one half hold the same columns: add them (lane bits 1..5), then the
  // waves in order
#pragma unroll
  for (int y = 0; y < MT; ++y)
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      double x = acc[y][j];
#pragma unroll
      for (int o = 2; o < 64; o <<= 1) x += __shfl_xor(x, o);
      if (lane < 2) red[wave][y][lane * NCH + j] = x;
    }
  __syncthreads();
  for (int e = tid; e < mg * ncols; e += kThreadsR) {
    const int y = e / ncols, j = e - y * ncols;
    double sum = red[0][y][j];
#pragma unroll
    for (int q = 1; q < kThreadsR / 64; ++q) sum += red[q][y][j];
    partial[(static_cast<int64_t>(t0 + y) * nb + chunk) * ncols + j] = sum;
  }
}

template <typename TD, int NCH, typename DI>
void launch_gemv_nch(const TD* D, int64_t rows, int ncols, const KronBatch& kb, int64_t per, int64_t nb,
                     double* partial, hipStream_t st) {
  // term slots a block: one for a single term (the fewest registers), else two, or four
  // where the accumulators fit (up to 24 columns).  A term's arithmetic is the same in
  // every instance: its slot only repeats the same operations for it.
  const int mt = kb.m == 1 ? 1 : (kb.m == 2 || NCH > 12) ? 2 : 4;
  const dim3 grid(static_cast<unsigned>((nb + 7) / 8 * 8 * ((kb.m + mt - 1) / mt)));
  if (mt == 1)
    hipLaunchKernelGGL((kron_gemv_kernel<TD, NCH, 1, DI>), grid, dim3(kThreadsR), 0, st, D, rows, ncols, kb, per, nb,
                       partial);
  else if (mt == 2)
    hipLaunchKernelGGL((kron_gemv_kernel<TD, NCH, 2, DI>), grid, dim3(kThreadsR), 0, st, D, rows, ncols, kb, per, nb,
                       partial);
  else
    hipLaunchKernelGGL((kron_gemv_kernel<TD, NCH, (NCH > 12 ? 2 : 4), DI>), grid, dim3(kThreadsR), 0, st, D, rows,
                       ncols, kb, per, nb, partial);
}

template <typename TD, typename DI>
void launch_gemv_di(const TD* D, int64_t rows, int ncols, const KronBatch& kb, int64_t per, int64_t nb,
                    double* partial, hipStream_t st) {
  if (ncols <= 8) launch_gemv_nch<TD, 4, DI>(D, rows, ncols, kb, per, nb, partial, st);
  else if (ncols <= 16) launch_gemv_nch<TD, 8, DI>(D, rows, ncols, kb, per, nb, partial, st);
  else if (ncols <= 24) launch_gemv_nch<TD, 12, DI>(D, rows, ncols, kb, per, nb, partial, st);
  else if (ncols <= 32) launch_gemv_nch<TD, 16, DI>(D, rows, ncols, kb, per, nb, partial, st);
  else if (ncols <= 48) launch_gemv_nch<TD, 24, DI>(D, rows, ncols, kb, per, nb, partial, st);
  else launch_gemv_nch<TD, 32, DI>(D, rows, ncols, kb, per, nb, partial, st);
}

template <typename TD>
void launch_gemv_dt(const TD* D, int64_t rows, int ncols, const KronBatch& kb, int64_t per, int64_t nb,
                    double* partial, hipStream_t st) {
  bool short_factors = true;
  for (int y = 0; y < kb.m; ++y)
    for (int p = 0; p < kb.kv[y].n; ++p) short_factors = short_factors && kb.kv[y].len[p] < (int64_t(1) << 30);
  if (short_factors) launch_gemv_di<TD, int>(D, rows, ncols, kb, per, nb, partial, st);
  else launch_gemv_di<TD, int64_t>(D, rows, ncols, kb, per, nb, partial, st);
}

// Kronecker GEMV with the two fastest factor positions (lengths e0, e1) contracted on
// the FP64 MFMA.  Block b takes the e0 e1 consecutive map rows of its outer index b
// (the digits of positions 2, 3, ..) and forms for every term y
//   C_y[j] = sum_{i1 < e1} v1_y[i1] sum_{i0 < e0} v0_y[i0] D[i0 + e0 (i1 + e1 b)][j],
// the inner sum as a 16 x 16 x 4 MFMA product with the terms as rows (A[y][i0] =
// v0_y[i0]) and a 16-column block of the map as columns (B[i0][j], K = e0 in steps of
// 4), then writes partial[(y nb S + g) ncols + j] = wrest_y(b) C_y[j], wrest_y the
// product of the remaining factors at b's digits.  A block's i1 range may be split over
// S workgroups (partial row g = b S + s, written in place of b): wave w of split s
// takes i1 = 4 s + w, 4 s + w + 4 S, ..; it
// copies its e0 x ncols block of rows (contiguous in the map) into its own LDS buffer
// from registers loaded one block ahead, so no barrier is needed inside the loop (a
// wave's LDS accesses are in program order); the four waves' sums are added in wave
// order at the end.  A term's row of the product does not depend on the other rows,
// so its partials are the same in any batch.
constexpr int kKmTile = 6144;     // bytes of one wave's staged block of map rows
constexpr int kKmE0 = 64;         // largest e0
constexpr int kKmE1 = 64;         // largest e1

template <typename TD, int NCB>
__global__ __launch_bounds__(256) void kron_mfma_kernel(const TD* __restrict__ D, int ncols, KronBatch kb,
                                                       int64_t nb, int S, double* __restrict__ partial) {
  using P = Pol<TTNN_F64>;
  constexpr int V = 16 / static_cast<int>(sizeof(TD));
  constexpr int TE = kKmTile / static_cast<int>(sizeof(TD));     // elements of a staged block
  constexpr int PER = TE / (64 * V);                               // 16-byte loads a lane a block
  static_assert(PER * 64 * V == TE, "whole loads");
  static_assert(4 * 16 * 16 * NCB * sizeof(double) <= 4 * kKmTile, "wave sums fit the tiles");
  typedef TD vec_t __attribute__((ext_vector_type(V)));
  __shared__ __align__(16) TD tile[4][TE];
  // factor tables [position value][term]: the 16 lanes of a group read 16 consecutive
  // doubles (with [term][value] rows of 512 bytes they hit one bank)
  __shared__ double W0[kKmE0][16];
  __shared__ double W1[kKmE1][16];

  const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t g = blockIdx.x;             // partial row g: block b, i1 split s of S
  const int64_t b = g / S;
  const int s = static_cast<int>(g - b * S);
  const int m = kb.m;
  const KronVec& k0 = kb.kv[0];             // every term has the same factor lengths
  const int e0 = static_cast<int>(k0.len[0]), e1 = static_cast<int>(k0.len[1]);
  const int blk = e0 * ncols;               // elements of one i1 block

  for (int e = tid; e < 16 * kKmE0; e += 256) {
    const int y = e / kKmE0, i = e % kKmE0;
    W0[i][y] = (y < m && i < e0) ? kb.kv[y].v[0][i] : 0.0;
  }
  for (int e = tid; e < 16 * kKmE1; e += 256) {
    const int y = e / kKmE1, i = e % kKmE1;
    W1[i][y] = (y < m && i < e1) ? kb.kv[y].v[1][i] : 0.0;
  }
  __syncthreads();

  const TD* base = D + b * static_cast<int64_t>(e1) * blk;
  TD* t = tile[wave];
  vec_t ra[PER];                            // the next block's loads, in flight under the products
  auto fetch = [&](int i1) {
    const TD* src = base + static_cast<int64_t>(i1) * blk;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = (lane + 64 * k) * V;
      ra[k] = e < blk ? *reinterpret_cast<const vec_t*>(src + e) : vec_t{};
    }
  };
  auto stage = [&](const vec_t* ra) {
#pragma unroll
    for (int k = 0; k < PER; ++k) *reinterpret_cast<vec_t*>(t + (lane + 64 * k) * V) = ra[k];
    // the block's reads below stay after its writes (the LDS keeps a wave's accesses in
    // order; this keeps the compiler from moving them)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  };
  typename P::CFrag acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = typename P::CFrag{};
  // two independent MFMA chains a column block (even and odd steps of 4 values), added
  // at the end: a dependent FP64 MFMA waits for the previous one's result
  auto compute = [&](int i1) {
    typename P::CFrag c[2][NCB];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) c[h][cb] = typename P::CFrag{};
#pragma unroll 2
    for (int k = 0; k < e0; k += 8) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i0 = k + 4 * h + lg;
        const double a = i0 < e0 ? W0[i0][l16] : 0.0;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int j = 16 * cb + l16;
          const double bv = (i0 < e0 && j < ncols) ? to_f64(t[i0 * ncols + j]) : 0.0;
          c[h][cb] = P::mfma(a, bv, c[h][cb]);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double s1 = W1[i1][P::crow(lane, v)];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb][v] += s1 * (c[0][cb][v] + c[1][cb][v]);
    }
  };
  const int i1s = 4 * s + wave, step = 4 * S;
  if (i1s < e1) fetch(i1s);
  for (int i1 = i1s; i1 < e1; i1 += step) {
    stage(ra);
    if (i1 + step < e1) fetch(i1 + step);
    compute(i1);
  }
  __syncthreads();                            // every wave is done with its tile
  double* red = reinterpret_cast<double*>(&tile[0][0]);     // [wave][term][column]
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) red[(wave * 16 + P::crow(lane, v)) * (16 * NCB) + 16 * cb + l16] = acc[cb][v];
  __syncthreads();
  for (int e = tid; e < 16 * ncols; e += 256) {
    const int y = e / ncols, j = e % ncols;
    if (y >= m) continue;
    const int o = y * (16 * NCB) + j, ws = 16 * 16 * NCB;
    const double sum = ((red[o] + red[o + ws]) + red[o + 2 * ws]) + red[o + 3 * ws];
    double wrest = 1.0;                       // the remaining factors at b's digits
    int64_t rem = b;
    for (int p = 2; p < k0.n; ++p) {
      const int64_t len = k0.len[p];
      wrest *= kb.kv[y].v[p][rem % len];
      rem /= len;
    }
    partial[(static_cast<int64_t>(y) * nb * S + g) * ncols + j] = wrest * sum;
  }
}

// Workgroups a block's i1 range is split over (a partial row each): one where the map
// has 1,024 blocks or more, else enough for 1,024 partial rows, each wave keeping at
// least two steps.  A function of the map's shape only, never of the batch.
int kron_mfma_split(int64_t nb, int64_t e1) {
  if (nb >= 1024) return 1;
  const int64_t want = (1024 + nb - 1) / nb;
  const int64_t most = std::max<int64_t>(1, e1 / 8);
  return static_cast<int>(std::min(want, most));
}

// Whether the MFMA form covers this map and batch shape (never depends on the number
// of terms, so a term takes the same form alone and in any batch).
bool kron_mfma_eligible(int64_t rows, int ncols, const KronVec& k0, size_t esize, size_t partial_elems) {
  if (k0.n < 2 || ncols > 48) return false;
  const int64_t e0 = k0.len[0], e1 = k0.len[1];
  if (e0 < 16 || e0 > kKmE0 || e1 < 4 || e1 > kKmE1) return false;
  const int64_t bytes = e0 * ncols * static_cast<int64_t>(esize);
  if (bytes > kKmTile || bytes % 16 != 0) return false;
  const int64_t nb = rows / (e0 * e1);
  if (nb < 1 || nb * e0 * e1 != rows) return false;
  const int64_t ns = nb * kron_mfma_split(nb, e1);
  return ns >= 256 && static_cast<size_t>(ns) * static_cast<size_t>(ncols) * kRank1Batch <= partial_elems;
}

template <typename TD>
void launch_kron_mfma(const TD* D, int ncols, const KronBatch& kb, int64_t nb, int S, double* partial,
                      hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(nb * S));
  switch ((ncols + 15) / 16) {
    case 1: hipLaunchKernelGGL((kron_mfma_kernel<TD, 1>), grid, dim3(256), 0, st, D, ncols, kb, nb, S, partial); break;
    case 2: hipLaunchKernelGGL((kron_mfma_kernel<TD, 2>), grid, dim3(256), 0, st, D, ncols, kb, nb, S, partial); break;
    default: hipLaunchKernelGGL((kron_mfma_kernel<TD, 3>), grid, dim3(256), 0, st, D, ncols, kb, nb, S, partial); break;
  }
}

// w[y wstride + j] = sum_b partial[y nb + b][j]: one wave per (column, term), lane l
// summing blocks l, l + 64, .. in order, the 64 sums combined by a fixed butterfly
__global__ __launch_bounds__(64) void sum_blocks_kernel(const double* __restrict__ partial, int nb, int ncols,
                                                        double* __restrict__ w, int64_t wstride) {
  const int j = blockIdx.x, y = blockIdx.y, l = threadIdx.x;
  const double* p = partial + static_cast<int64_t>(y) * nb * ncols;
  // lane l adds blocks l, l + 64, .. in order, eight loads in flight at a time
  double s = 0.0;
  int b = l;
  for (; b + 7 * 64 < nb; b += 8 * 64) {
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[static_cast<int64_t>(b + 64 * i) * ncols + j];
#pragma unroll
    for (int i = 0; i < 8; ++i) s += v[i];
  }
  for (; b < nb; b += 64) s += p[static_cast<int64_t>(b) * ncols + j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (l == 0) w[y * wstride + j] = s;
}

// R[i + n j] += alpha_y * weight_y(i) * (w ? w[y wstride + j] : 1), the terms in order.
// The terms of a batch share their factor lengths (the caller checks), so a thread takes a
// row i, splits it into factor digits once, forms alpha_y weight_y(i) for every term (each
// weight multiplied out in factor order) and sweeps the columns j = blockIdx.y,
// blockIdx.y + gridDim.y, ..; neighbouring lanes take neighbouring rows, so every column
// access coalesces.
__global__ void outer_acc_kernel(double* __restrict__ R, int64_t n, int ncols, KronBatch ku,
                                 const double* __restrict__ w, int64_t wstride) {
  const int np = ku.kv[0].n;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double a[kRank1Batch];
#pragma unroll
    for (int y = 0; y < kRank1Batch; ++y) a[y] = 1.0;
    int64_t row = i;
    for (int p = 0; p < np; ++p) {
      const int64_t e = ku.kv[0].len[p];
      const int64_t dgt = row % e;
      row /= e;
#pragma unroll
      for (int y = 0; y < kRank1Batch; ++y)
        if (y < ku.m) a[y] *= ku.kv[y].v[p][dgt];
    }
#pragma unroll
    for (int y = 0; y < kRank1Batch; ++y) a[y] *= ku.alpha[y];
    for (int j = blockIdx.y; j < ncols; j += gridDim.y) {
      double r = R[i + n * j];
#pragma unroll
      for (int y = 0; y < kRank1Batch; ++y)
        if (y < ku.m) r += a[y] * (w ? w[y * wstride + j] : 1.0);
      R[i + n * j] = r;
    }
  }
}

}  // namespace

void launch_kron_gemv(const void* D, int dt, int64_t rows, int ncols, const KronBatch& kb, double* partial,
                      size_t partial_elems, double* w, int64_t wstride, bool grouped, hipStream_t st) {
  if (ncols <= 0 || kb.m <= 0) return;
  TTNN_REQUIRE(ncols <= 64, TTNN_E_INVALID, "rank-1 update with more than 64 map columns");
  TTNN_REQUIRE(kb.m <= kRank1Batch, TTNN_E_INVALID, "too many rank-1 terms in one launch");
  const size_t esize = dt == TTNN_F64 ? 8 : dt == TTNN_F32 ? 4 : 2;
  if (grouped && kron_mfma_eligible(rows, ncols, kb.kv[0], esize, partial_elems)) {
    const int64_t nbm = rows / (kb.kv[0].len[0] * kb.kv[0].len[1]);
    const int S = kron_mfma_split(nbm, kb.kv[0].len[1]);
    if (dt == TTNN_F64) launch_kron_mfma(static_cast<const double*>(D), ncols, kb, nbm, S, partial, st);
    else if (dt == TTNN_F32) launch_kron_mfma(static_cast<const float*>(D), ncols, kb, nbm, S, partial, st);
    else launch_kron_mfma(static_cast<const uint16_t*>(D), ncols, kb, nbm, S, partial, st);
    hipLaunchKernelGGL(sum_blocks_kernel, dim3(ncols, kb.m), dim3(64), 0, st, partial, static_cast<int>(nbm * S),
                       ncols, w, wstride);
    return;
  }
  // >= 512 rows a block, at most 2048 blocks a term; the chunking depends on rows and
  // ncols only, never on the batch, so a term's sums are the same in any batch
  int64_t nb = (rows + 511) / 512;
  if (nb < 1) nb = 1;
  if (nb > 2048) nb = 2048;
  const int64_t cap = static_cast<int64_t>(partial_elems / (static_cast<size_t>(ncols) * kRank1Batch));
  if (nb > cap) nb = cap;
  TTNN_REQUIRE(nb >= 1, TTNN_E_INVALID, "rank-1 scratch too small");
  // rows a block: a multiple of the kernel's step (256 rows)
  const int64_t rb = kThreadsR;
  int64_t per = (rows + nb - 1) / nb;
  per = (per + rb - 1) / rb * rb;
  if (per < rb) per = rb;
  nb = rows > 0 ? (rows + per - 1) / per : 1;
  if (dt == TTNN_F64)
    launch_gemv_dt(static_cast<const double*>(D), rows, ncols, kb, per, nb, partial, st);
  else if (dt == TTNN_F32)
    launch_gemv_dt(static_cast<const float*>(D), rows, ncols, kb, per, nb, partial, st);
  else
    launch_gemv_dt(static_cast<const uint16_t*>(D), rows, ncols, kb, per, nb, partial, st);
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(ncols, kb.m), dim3(64), 0, st, partial, static_cast<int>(nb), ncols, w,
                     wstride);
}

void launch_outer_acc(double* R, int64_t n, int ncols, const KronBatch& ku, const double* w, int64_t wstride,
                      hipStream_t st) {
  if (n <= 0 || ncols <= 0 || ku.m <= 0) return;
  for (int y = 1; y < ku.m; ++y) {
    TTNN_REQUIRE(ku.kv[y].n == ku.kv[0].n, TTNN_E_INVALID, "rank-1 terms of one batch differ in factor count");
    for (int p = 0; p < ku.kv[0].n; ++p)
      TTNN_REQUIRE(ku.kv[y].len[p] == ku.kv[0].len[p], TTNN_E_INVALID,
                   "rank-1 terms of one batch differ in factor length");
  }
  // column groups enough for about 2^20 threads (the weights are formed once a group)
  const int64_t cg = std::min<int64_t>(ncols, std::max<int64_t>(1, ((int64_t{1} << 20) + n - 1) / n));
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, std::max<int64_t>(1, 4096 / cg));
  hipLaunchKernelGGL(outer_acc_kernel, dim3(static_cast<unsigned>(blocks), static_cast<unsigned>(cg)), dim3(256), 0,
                     st, R, n, ncols, ku, w, wstride);
}

}  // namespace ttnn
