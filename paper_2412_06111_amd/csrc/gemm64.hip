// Batched strided FP64 GEMM on MFMA (v_mfma_f64_16x16x4f64) for the dense FP64
// work of the engine: the epilogue (Omega_t = Y_t^T R_t, Psi_t), the cores of the
// recovery phase, the reconstruction, and contractions of FP64 intermediates.
//
// A job computes, for every output batch cb < nbC,
//   C[cb](m, n) = (accumulate ? C[cb](m, n) : 0)
//                 + alpha * sum_{kb < nbK} sum_{k < K} A(m, k; cb, kb) B(k, n; cb, kb)
// with A(m, k; cb, kb) = A[m sAm + k sAk + cb sAc + kb sAkb] (B, C likewise).
// Long contractions are split over several workgroups whose partial tiles a second
// launch adds in split order, so results do not depend on scheduling.  (A last-block
// combine would need a device-scope fence, which on this chip writes back and
// invalidates the whole L2 of the XCD for every workgroup.)  Several jobs share one
// launch.
#include "kernels.hpp"
#include "mfma.hpp"

namespace ttnn {
namespace {

// A K-step of 64 keeps 16 loads a thread in flight: these products are short, so
// their time is the number of dependent memory round trips, not arithmetic.
constexpr int TM = 32, TN = 32, TK = 64;
constexpr int LPT = TM * TK / 256;          // elements of each operand tile per thread (8)

__global__ __launch_bounds__(256) void bgemm64_kernel(GJobList L) {
  __shared__ double As[TK][TM + 1];
  __shared__ double Bs[TK][TN + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int64_t b = blockIdx.x;
  int ji = 0;
  while (ji + 1 < L.n && L.jobs[ji + 1].first_block <= b) ++ji;
  const GJob& J = L.jobs[ji];
  int64_t rel = b - J.first_block;
  const int split = static_cast<int>(rel % J.splits);
  rel /= J.splits;
  const int64_t tn = rel % J.tiles_n;
  rel /= J.tiles_n;
  const int64_t tm = rel % J.tiles_m;
  const int64_t cb = rel / J.tiles_m;
  const int64_t m0 = tm * TM, n0 = tn * TN;

  // contraction range of this split over the flattened (kb, k) space
  const int64_t KK = static_cast<int64_t>(J.nbK) * J.K;
  const int64_t k_begin = (KK * split) / J.splits;
  const int64_t k_end = (KK * (split + 1)) / J.splits;

  const int wm = wave >> 1, wn = wave & 1;    // 16 x 16 block of the wave
  f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
  const double* Ab = J.A + cb * J.sAc;
  const double* Bb = J.B + cb * J.sBc;
  // thread -> (row, k) map of the tile loads: contiguous index fastest
  const bool a_k_fast = J.sAk == 1 && J.sAm != 1;
  const bool b_k_fast = J.sBk == 1 && J.sBn != 1;

  double ra[LPT], rb[LPT];
  int64_t kk = k_begin;
  int64_t kcur = 0;   // length of the staged step
  auto fetch = [&](int64_t kpos, int64_t& klen) {
    const int64_t kb = kpos / J.K;
    const int64_t k0 = kpos - kb * J.K;
    int64_t kstop = J.K - k0;                  // stay inside one kb
    if (kstop > k_end - kpos) kstop = k_end - kpos;
    if (kstop > TK) kstop = TK;
    klen = kstop;
    const double* Ak = Ab + kb * J.sAkb;
    const double* Bk = Bb + kb * J.sBkb;
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int e = tid + 256 * u;
      const int mm = a_k_fast ? e / TK : e % TM, kx = a_k_fast ? e % TK : e / TM;
      ra[u] = (kx < kstop && m0 + mm < J.M) ? Ak[(m0 + mm) * J.sAm + (k0 + kx) * J.sAk] : 0.0;
      const int nn = b_k_fast ? e / TK : e % TN, ky = b_k_fast ? e % TK : e / TN;
      rb[u] = (ky < kstop && n0 + nn < J.N) ? Bk[(k0 + ky) * J.sBk + (n0 + nn) * J.sBn] : 0.0;
    }
  };
  if (kk < k_end) fetch(kk, kcur);
  while (kk < k_end) {
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int e = tid + 256 * u;
      const int mm = a_k_fast ? e / TK : e % TM, kx = a_k_fast ? e % TK : e / TM;
      As[kx][mm] = ra[u];
      const int nn = b_k_fast ? e / TK : e % TN, ky = b_k_fast ? e % TK : e / TN;
      Bs[ky][nn] = rb[u];
    }
    __syncthreads();
    const int64_t knext = kk + kcur;
    int64_t klen_next = 0;
    if (knext < k_end) fetch(knext, klen_next);   // next step's loads overlap the MFMAs
    // rows past the staged length are zero; skip whole groups of 4 beyond it
    const int nmf = static_cast<int>((kcur + 3) / 4);
#pragma unroll 8
    for (int s = 0; s < nmf; ++s) {
      const double a = As[4 * s + lg][16 * wm + l16];
      const double bv = Bs[4 * s + lg][16 * wn + l16];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
    }
    __syncthreads();
    kk = knext;
    kcur = klen_next;
  }

  // C fragment: lane holds C[16 wm + 4 v + lg][16 wn + l16]
  if (J.splits == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t m = m0 + 16 * wm + 4 * v + lg, n = n0 + 16 * wn + l16;
      if (m < J.M && n < J.N) {
        double* c = J.C + cb * J.sCc + m * J.sCm + n * J.sCn;
        *c = (J.accumulate ? *c : 0.0) + J.alpha * acc[v];
      }
    }
    return;
  }
  // split contraction: store the partial tile; bgemm64_combine_kernel adds them
  const int64_t tile_id = (cb * J.tiles_m + tm) * J.tiles_n + tn;
  double* part = J.part + (tile_id * J.splits + split) * (TM * TN);
#pragma unroll
  for (int v = 0; v < 4; ++v) part[(16 * wm + 4 * v + lg) * TN + 16 * wn + l16] = acc[v];
}

// Four workgroups per tile of a split job, one element a thread: C = (accumulate ? C :
// 0) + alpha * sum of the partial tiles in split order (32 interleaved sums, combined
// pairwise in a fixed tree), so results do not depend on scheduling and a thread keeps
// 32 loads in flight.  A launch of its own: the kernel boundary makes the partials
// visible without a device-wide fence.
constexpr int kCombineParts = 4;          // workgroups per 32 x 32 tile
static_assert(kCombineParts * 256 == TM * TN, "one tile element per thread");
__global__ __launch_bounds__(256) void bgemm64_combine_kernel(GJobList L) {
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x / kCombineParts;
  const int part_of = static_cast<int>(blockIdx.x % kCombineParts);
  int ji = 0;
  while (ji + 1 < L.n && L.jobs[ji + 1].first_tile <= b) ++ji;
  const GJob& J = L.jobs[ji];
  const int64_t tile_id = b - J.first_tile;
  int64_t rel = tile_id;
  const int64_t tn = rel % J.tiles_n;
  rel /= J.tiles_n;
  const int64_t tm = rel % J.tiles_m;
  const int64_t cb = rel / J.tiles_m;
  const int64_t m0 = tm * TM, n0 = tn * TN;
  const double* parts = J.part + tile_id * J.splits * (TM * TN);
  const int e = part_of * 256 + tid;        // element of the tile
  constexpr int NS = 32;
  double s[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) s[q] = 0.0;
  // split sp + q goes to sum q; splits past the end add nothing (static indices only)
  for (int sp = 0; sp < J.splits; sp += NS) {
    double v[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) v[q] = sp + q < J.splits ? parts[(sp + q) * (TM * TN) + e] : 0.0;
#pragma unroll
    for (int q = 0; q < NS; ++q) s[q] += v[q];
  }
#pragma unroll
  for (int w = NS / 2; w > 0; w /= 2)
#pragma unroll
    for (int q = 0; q < w; ++q) s[q] += s[q + w];
  const int mm = e / TN, nn = e % TN;
  const int64_t m = m0 + mm, n = n0 + nn;
  if (m >= J.M || n >= J.N) return;
  double* c = J.C + cb * J.sCc + m * J.sCm + n * J.sCn;
  *c = (J.accumulate ? *c : 0.0) + J.alpha * s[0];
}

}  // namespace

void launch_bgemm64(std::vector<GJob>& jobs, double* part, size_t part_elems, hipStream_t st) {
  for (size_t j0 = 0; j0 < jobs.size(); j0 += kMaxGJobs) {
    GJobList L{};
    GJobList LC{};                              // split jobs, for the combine launch
    L.n = static_cast<int>(std::min<size_t>(kMaxGJobs, jobs.size() - j0));
    int64_t blocks = 0, ctiles = 0;
    size_t part_used = 0;
    for (int i = 0; i < L.n; ++i) {
      GJob j = jobs[j0 + i];
      j.tiles_m = (j.M + TM - 1) / TM;
      j.tiles_n = (j.N + TN - 1) / TN;
      const int64_t tiles = j.tiles_m * j.tiles_n * j.nbC;
      // split long contractions so that the launch has enough workgroups
      const int64_t KK = static_cast<int64_t>(j.nbK) * j.K;
      int64_t sp = 1;
      if (tiles < 512 && KK > 256) {
        sp = std::min<int64_t>((KK + 255) / 256, std::max<int64_t>(1, 1024 / tiles));
        sp = std::min<int64_t>(sp, 256);
      }
      const size_t need = static_cast<size_t>(tiles * sp * TM * TN);
      if (sp > 1 && part_used + need > part_elems) sp = 1;
      j.splits = static_cast<int>(sp);
      if (sp > 1) {
        j.part = part + part_used;
        part_used += need;
        j.first_tile = ctiles;
        ctiles += tiles;
      }
      j.first_block = blocks;
      blocks += tiles * sp;
      L.jobs[i] = j;
      if (sp > 1) LC.jobs[LC.n++] = j;
    }
    if (blocks > 0)
      hipLaunchKernelGGL(bgemm64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, L);
    if (ctiles > 0)
      hipLaunchKernelGGL(bgemm64_combine_kernel, dim3(static_cast<unsigned>(ctiles * kCombineParts)), dim3(256), 0,
                         st, LC);
  }
}

}  // namespace ttnn
