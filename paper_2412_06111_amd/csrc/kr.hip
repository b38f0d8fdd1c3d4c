// Tree contractions of a TTN-format tensor with Khatri-Rao maps (Sec. 7).
//
// Every contraction of the structured sketch that shares one column index j over all
// of its operands has the form
//   out[o, j] = sum over every core index except axis `oax` of
//               core[idx] * prod_{q != oax} F_q[idx_q, j]
// (core column-major, first axis fastest; F_q row-major size_q x cols, j fastest; out
// row-major size_o x cols).  With F_q the per-mode factors or the children's vectors it
// gives the down vectors of a node; with the siblings' and the parent's vectors, the up
// vectors of a child.  FP64 VALU work: lanes run over j (coalesced factor reads), the
// core entry is the same for every lane.  The reduction is cut into 4 G contiguous
// slices of the flattened index (inner axis fastest); each wave sums one slice, the four
// waves of a workgroup combine in a fixed order and, for G > 1, a second kernel adds the
// G partials in a fixed order, so the result depends only on the shapes.
#include "kr.hpp"

namespace ttnn {

namespace {

constexpr int kWaves = 4;

__global__ __launch_bounds__(256) void kr_contract_kernel(KJobList L) {
  const int64_t b = blockIdx.x;
  int jid = 0;
  while (jid + 1 < L.n && b >= L.jobs[jid + 1].first_block) ++jid;
  const KJob& J = L.jobs[jid];
  int64_t local = b - J.first_block;
  const int64_t cc = local % J.colchunks;
  local /= J.colchunks;
  const int64_t so = J.size[J.oax];
  const int64_t o = local % so;
  const int64_t g = local / so;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = cc * 64 + lane;
  const bool act = j < J.cols;
  const int64_t jj = act ? j : 0;
  const int64_t cols = J.cols;

  int ax[kMaxAxes];
  int na = 0;
  int64_t stride[kMaxAxes];
  int64_t s = 1;
  for (int q = 0; q < J.naxes; ++q) {
    stride[q] = s;
    s *= J.size[q];
    if (q != J.oax) ax[na++] = q;
  }
  // inner axis: the first other axis (a pseudo-axis of size 1 when there is none)
  const int64_t n0 = na ? J.size[ax[0]] : 1;
  const int64_t st0 = na ? stride[ax[0]] : 0;
  const double* F0 = na ? J.fac[ax[0]] : nullptr;
  const int64_t kred = J.kred;
  const int64_t nsl = static_cast<int64_t>(J.G) * kWaves;
  const int64_t sl = g * kWaves + wave;
  const int64_t lo = kred * sl / nsl, hi = kred * (sl + 1) / nsl;
  const double* core = J.core + o * stride[J.oax];

  double acc = 0.0;
  if (lo < hi) {
    int64_t dig[kMaxAxes];
    int64_t rest = lo / n0;
    int64_t a0 = lo % n0;
    for (int q = 1; q < na; ++q) {
      dig[q] = rest % J.size[ax[q]];
      rest /= J.size[ax[q]];
    }
    int64_t e = lo;
    while (e < hi) {
      double w = 1.0;
      int64_t off = 0;
      for (int q = 1; q < na; ++q) {
        w *= J.fac[ax[q]][dig[q] * cols + jj];
        off += dig[q] * stride[ax[q]];
      }
      const int64_t run = (n0 - a0 < hi - e) ? n0 - a0 : hi - e;
      const double* cp = core + off + a0 * st0;
      double in = 0.0;
      if (F0) {
        const double* fp = F0 + a0 * cols + jj;
        int64_t t = 0;
        double in1 = 0.0;
        for (; t + 1 < run; t += 2) {
          in = fma(cp[t * st0], fp[t * cols], in);
          in1 = fma(cp[(t + 1) * st0], fp[(t + 1) * cols], in1);
        }
        if (t < run) in = fma(cp[t * st0], fp[t * cols], in);
        in += in1;
      } else {
        in = cp[0];
      }
      acc = fma(w, in, acc);
      e += run;
      a0 = 0;
      for (int q = 1; q < na; ++q) {           // next outer combination
        if (++dig[q] < J.size[ax[q]]) break;
        dig[q] = 0;
      }
    }
  }
  __shared__ double red[kWaves][64];
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && act) {
    const double v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    if (J.G == 1) J.out[o * cols + j] = v;
    else J.part[(g * so + o) * cols + j] = v;
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
  double v = 0.0;
  for (int g = 0; g < J.G; ++g) v += J.part[g * size + e];
  J.out[e] = v;
}

}  // namespace

int kr_split(int64_t so, int cols, int64_t kred) {
  const int64_t base = so * ((cols + 63) / 64);
  int64_t G = kred / (kWaves * 64);
  const int64_t cap = base >= 1024 ? 1 : 1024 / base;
  if (G > cap) G = cap;
  if (G > 256) G = 256;
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
      j.colchunks = (j.cols + 63) / 64;
      j.kred = 1;
      for (int q = 0; q < j.naxes; ++q)
        if (q != j.oax) j.kred *= j.size[q];
      j.first_block = blocks;
      blocks += j.size[j.oax] * j.colchunks * j.G;
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
