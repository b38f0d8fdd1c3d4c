// Tree contractions of a TTN-format tensor with Khatri-Rao maps (Sec. 7).
//
// Every contraction of the structured sketch that shares one column index j over all
// of its operands has the form
//   out[o, j] = sum over every core index except axis `oax` of
//               core[idx] * prod_{q != oax} F_q[idx_q, j]
// (core column-major, first axis fastest; F_q row-major size_q x cols, j fastest; out
// row-major size_o x cols).  With F_q the per-mode factors or the children's vectors it
// gives the down vectors of a node; with the siblings' and the parent's vectors, the up
// vectors of a child.  Split the reduction index into the first non-output axis a
// (size n0) and the rest e (the outer combinations):
//   out[o, j] = sum_e w_e[j] sum_a C_e[o, a] F_0[a, j],  w_e[j] = prod_{q>=1} F_q[e_q, j],
// a GEMM per outer combination, scaled by column and accumulated.  A workgroup owns a
// 32 (o) x 64 (j) tile; per unit (one outer combination, one chunk of at most 32 values
// of a, the chunks of equal length) it stages C_e (chunk x 32) and F_0 (chunk x 64) in
// LDS, loading the next unit into registers while it computes, and every thread
// accumulates a 2 x 4 register block in FP64 (VALU).  The units are cut into G contiguous slices, one workgroup
// each; for G > 1 a second kernel adds the G partials in a fixed order, so the result
// depends only on the shapes.
#include "kr.hpp"

namespace ttnn {

namespace {

constexpr int kTO = 32, kTJ = 64, kKC = 32;   // kKC: longest chunk of the inner axis per unit
constexpr int kCLD = kTO + 2;                  // LDS row of C: padded, 16-byte aligned
constexpr int kCR = kKC * kTO / 256, kFR = kKC * kTJ / 256;

// Chunks of the inner axis: as few as hold n0 in chunks of at most kKC, of equal length.
__host__ __device__ inline int64_t kr_nchunks(int64_t n0) { return (n0 + kKC - 1) / kKC; }
__host__ __device__ inline int kr_chunk(int64_t n0) {
  const int64_t nch = kr_nchunks(n0);
  return static_cast<int>((n0 + nch - 1) / nch);
}

__global__ __launch_bounds__(256) void kr_contract_kernel(KJobList L) {
  const int64_t b = blockIdx.x;
  int jid = 0;
  while (jid + 1 < L.n && b >= L.jobs[jid + 1].first_block) ++jid;
  const KJob& J = L.jobs[jid];
  int64_t local = b - J.first_block;
  const int64_t jt = local % J.colchunks;
  local /= J.colchunks;
  const int64_t ot = local % J.otiles;
  const int64_t g = local / J.otiles;
  const int64_t so = J.size[J.oax];
  const int cols = J.cols;
  const int tid = threadIdx.x;
  const int tj = tid & 15, to = tid >> 4;
  const int64_t o0 = ot * kTO, j0 = jt * kTJ;

  int ax[kMaxAxes];
  int na = 0;
  int64_t stride[kMaxAxes];
  int64_t sz = 1;
  for (int q = 0; q < J.naxes; ++q) {
    stride[q] = sz;
    sz *= J.size[q];
    if (q != J.oax) ax[na++] = q;
  }
  const int64_t n0 = na ? J.size[ax[0]] : 1;
  const int64_t st0 = na ? stride[ax[0]] : 0;
  const double* F0 = na ? J.fac[ax[0]] : nullptr;
  const int64_t nch = kr_nchunks(n0);
  const int kc = kr_chunk(n0);
  const int64_t units = (J.kred / n0) * nch;
  const int64_t ulo = units * g / J.G, uhi = units * (g + 1) / J.G;
  const int64_t so_stride = stride[J.oax];

  __shared__ __attribute__((aligned(16))) double Cs[kKC * kCLD];
  __shared__ __attribute__((aligned(16))) double Fs[kKC * kTJ];

  // the unit being loaded: outer combination (digits, core offset, column weights) and chunk
  int64_t dig[kMaxAxes] = {};
  int64_t eL = -1, offL = 0;
  double wL[4] = {1.0, 1.0, 1.0, 1.0};
  double cr[kCR], fr[kFR];
  auto load = [&](int64_t u) {
    const int64_t e = u / nch, c0 = u % nch;
    if (e != eL) {
      if (eL < 0) {
        int64_t rest = e;
        for (int q = 1; q < na; ++q) {
          dig[q] = rest % J.size[ax[q]];
          rest /= J.size[ax[q]];
        }
      } else {
        for (int q = 1; q < na; ++q) {
          if (++dig[q] < J.size[ax[q]]) break;
          dig[q] = 0;
        }
      }
      eL = e;
      offL = 0;
      for (int q = 1; q < na; ++q) offL += dig[q] * stride[ax[q]];
      for (int i = 0; i < 4; ++i) {
        const int64_t j = j0 + 4 * tj + i;
        double v = 1.0;
        if (j < cols)
          for (int q = 1; q < na; ++q) v *= J.fac[ax[q]][dig[q] * cols + j];
        wL[i] = v;
      }
    }
    const int64_t a0 = c0 * kc;
    const int64_t alim = (n0 - a0) < kc ? (n0 - a0) : kc;
#pragma unroll
    for (int i = 0; i < kCR; ++i) {            // C_e[o0 .. o0 + 32, a0 .. a0 + kc): a fastest
      const int idx = tid + 256 * i;
      const int a = idx % kKC, o = idx / kKC;
      double v = 0.0;
      if (o0 + o < so && a < alim) v = J.core[(o0 + o) * so_stride + offL + (a0 + a) * st0];
      cr[i] = v;
    }
#pragma unroll
    for (int i = 0; i < kFR; ++i) {            // F_0[a0 .. a0 + kc, j0 .. j0 + 64): j fastest
      const int idx = tid + 256 * i;
      const int j = idx % kTJ, a = idx / kTJ;
      double v = 0.0;
      if (j0 + j < cols && a < alim) v = F0 ? F0[(a0 + a) * cols + j0 + j] : 1.0;
      fr[i] = v;
    }
  };

  double acc[2][4] = {};
  if (ulo < uhi) load(ulo);
  for (int64_t u = ulo; u < uhi; ++u) {
    const double w[4] = {wL[0], wL[1], wL[2], wL[3]};
    const int64_t c0 = u % nch;
    const int arun = static_cast<int>((n0 - c0 * kc) < kc ? (n0 - c0 * kc) : kc);
#pragma unroll
    for (int i = 0; i < kCR; ++i) {
      const int idx = tid + 256 * i;
      Cs[(idx % kKC) * kCLD + idx / kKC] = cr[i];
    }
#pragma unroll
    for (int i = 0; i < kFR; ++i) {
      const int idx = tid + 256 * i;
      Fs[(idx / kTJ) * kTJ + idx % kTJ] = fr[i];
    }
    __syncthreads();
    if (u + 1 < uhi) load(u + 1);              // next unit's loads overlap this unit's arithmetic
    double t[2][4] = {};
    for (int a = 0; a < arun; ++a) {
      const double2 c = *reinterpret_cast<const double2*>(&Cs[a * kCLD + 2 * to]);
      const double2 f01 = *reinterpret_cast<const double2*>(&Fs[a * kTJ + 4 * tj]);
      const double2 f23 = *reinterpret_cast<const double2*>(&Fs[a * kTJ + 4 * tj + 2]);
      t[0][0] = fma(c.x, f01.x, t[0][0]);
      t[0][1] = fma(c.x, f01.y, t[0][1]);
      t[0][2] = fma(c.x, f23.x, t[0][2]);
      t[0][3] = fma(c.x, f23.y, t[0][3]);
      t[1][0] = fma(c.y, f01.x, t[1][0]);
      t[1][1] = fma(c.y, f01.y, t[1][1]);
      t[1][2] = fma(c.y, f23.x, t[1][2]);
      t[1][3] = fma(c.y, f23.y, t[1][3]);
    }
    for (int i = 0; i < 2; ++i)
      for (int jj = 0; jj < 4; ++jj) acc[i][jj] = fma(w[jj], t[i][jj], acc[i][jj]);
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i) {
    const int64_t o = o0 + 2 * to + i;
    if (o >= so) continue;
    for (int jj = 0; jj < 4; ++jj) {
      const int64_t j = j0 + 4 * tj + jj;
      if (j >= cols) continue;
      if (J.G == 1) J.out[o * cols + j] = acc[i][jj];
      else J.part[(g * so + o) * cols + j] = acc[i][jj];
    }
  }
}

// out[e] = sum_{g < G} part[g * size + e] in order, for the jobs split over G > 1.
__global__ __launch_bounds__(256) void kr_fold_kernel(KJobList L) {
  const int64_t b = blockIdx.x;
  int jid = -1;
  for (int i = 0; i < L.n; ++i)
    if (L.jobs[i].G > 1 && b >= L.jobs[i].fold_first) jid = i;
  if (jid < 0) return;
  const KJob& J = L.jobs[jid];
  const int64_t size = J.size[J.oax] * static_cast<int64_t>(J.cols);
  const int64_t e = (b - J.fold_first) * 256 + threadIdx.x;
  if (e >= size) return;
  // loads issued eight at a time, added in the fixed order g = 0, 1, ..
  double v = 0.0;
  int g = 0;
  for (; g + 8 <= J.G; g += 8) {
    double x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = J.part[(g + i) * size + e];
#pragma unroll
    for (int i = 0; i < 8; ++i) v += x[i];
  }
  for (; g < J.G; ++g) v += J.part[g * size + e];
  J.out[e] = v;
}

}  // namespace

int kr_split(int64_t so, int cols, int64_t n0, int64_t nouter) {
  const int64_t tiles = ((so + kTO - 1) / kTO) * ((cols + kTJ - 1) / kTJ);
  const int64_t units = nouter * kr_nchunks(n0);
  int64_t G = tiles >= 512 ? 1 : 512 / tiles;
  if (G > units / 2) G = units / 2;                    // at least two units per slice
  if (G > 32) G = 32;                                  // the fold reads G partials per output
  return G < 1 ? 1 : static_cast<int>(G);
}

size_t kr_part_elems(const KJob& j) {
  return j.G > 1 ? static_cast<size_t>(j.G) * j.size[j.oax] * j.cols : 0;
}

void launch_kr_contract(std::vector<KJob> jobs, hipStream_t stream) {
  for (size_t at = 0; at < jobs.size(); at += kMaxKJobs) {
    KJobList L{};
    int64_t blocks = 0, fblocks = 0;
    for (size_t i = at; i < jobs.size() && L.n < kMaxKJobs; ++i) {
      KJob j = jobs[i];
      TTNN_REQUIRE(j.naxes >= 1 && j.naxes <= kMaxAxes && j.oax >= 0 && j.oax < j.naxes && j.cols >= 1,
                   TTNN_E_INVALID, "bad tree contraction");
      TTNN_REQUIRE(j.G == 1 || j.part != nullptr, TTNN_E_INVALID, "split tree contraction without scratch");
      j.colchunks = (j.cols + kTJ - 1) / kTJ;
      j.otiles = (j.size[j.oax] + kTO - 1) / kTO;
      j.kred = 1;
      for (int q = 0; q < j.naxes; ++q)
        if (q != j.oax) j.kred *= j.size[q];
      j.first_block = blocks;
      blocks += j.otiles * j.colchunks * j.G;
      if (j.G > 1) {
        j.fold_first = fblocks;
        fblocks += (j.size[j.oax] * j.cols + 255) / 256;
      }
      L.jobs[L.n++] = j;
    }
    if (blocks > 0) kr_contract_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream>>>(L);
    if (fblocks > 0) kr_fold_kernel<<<dim3(static_cast<unsigned>(fblocks)), dim3(256), 0, stream>>>(L);
  }
}

}  // namespace ttnn
