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
constexpr int kColsPerPass = 64;

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

// partial[b][j] = sum over rows of block b of D[row * ncols + j] * weight(row)
template <typename TD>
__global__ __launch_bounds__(kThreadsR) void kron_gemv_kernel(const TD* __restrict__ D, int64_t rows, int ncols,
                                                              KronVec kv, int64_t rows_per_block,
                                                              double* __restrict__ partial) {
  __shared__ double red[kThreadsR];
  const int tid = threadIdx.x;
  const int jl = tid % kColsPerPass, rl = tid / kColsPerPass;       // 4 row lanes x 64 columns
  constexpr int RL = kThreadsR / kColsPerPass;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  for (int j0 = 0; j0 < ncols; j0 += kColsPerPass) {
    const int j = j0 + jl;
    double acc = 0.0;
    if (j < ncols)
      for (int64_t row = r0 + rl; row < r1; row += RL)
        acc = fma(to_f64(D[row * ncols + j]), kron_weight(kv, row), acc);
    red[tid] = acc;
    __syncthreads();
    if (rl == 0 && j < ncols) {
      double s = red[jl];
#pragma unroll
      for (int q = 1; q < RL; ++q) s += red[q * kColsPerPass + jl];
      partial[static_cast<int64_t>(blockIdx.x) * ncols + j] = s;
    }
    __syncthreads();
  }
}

// w[j] = sum_b partial[b][j], blocks in order
__global__ void sum_blocks_kernel(const double* __restrict__ partial, int nb, int ncols, double* __restrict__ w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncols) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[static_cast<int64_t>(b) * ncols + j];
  w[j] = s;
}

// R[i + n j] += alpha * weight(i) * (w ? w[j] : 1)
__global__ void outer_acc_kernel(double* __restrict__ R, int64_t n, int ncols, KronVec ku, const double* __restrict__ w,
                                 double alpha) {
  const int64_t total = n * ncols;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = e % n;
    const int64_t j = e / n;
    const double wj = w ? w[j] : 1.0;
    R[e] += alpha * kron_weight(ku, i) * wj;
  }
}

}  // namespace

void launch_kron_gemv(const void* D, int dt, int64_t rows, int ncols, const KronVec& kv, double* partial,
                      size_t partial_elems, double* w, hipStream_t st) {
  if (ncols <= 0) return;
  int64_t nb = (rows + 4095) / 4096;                   // ~4096 rows per block
  if (nb < 1) nb = 1;
  if (nb > 2048) nb = 2048;
  const int64_t cap = static_cast<int64_t>(partial_elems / static_cast<size_t>(ncols));
  if (nb > cap) nb = cap;
  TTNN_REQUIRE(nb >= 1, TTNN_E_INVALID, "rank-1 scratch too small");
  const int64_t per = (rows + nb - 1) / nb;
  nb = rows > 0 ? (rows + per - 1) / per : 1;
  const dim3 grid(static_cast<unsigned>(nb));
  const int64_t pr = per > 0 ? per : 1;
  if (dt == TTNN_F64)
    hipLaunchKernelGGL(kron_gemv_kernel<double>, grid, dim3(kThreadsR), 0, st, static_cast<const double*>(D), rows,
                       ncols, kv, pr, partial);
  else if (dt == TTNN_F32)
    hipLaunchKernelGGL(kron_gemv_kernel<float>, grid, dim3(kThreadsR), 0, st, static_cast<const float*>(D), rows,
                       ncols, kv, pr, partial);
  else
    hipLaunchKernelGGL(kron_gemv_kernel<uint16_t>, grid, dim3(kThreadsR), 0, st, static_cast<const uint16_t*>(D),
                       rows, ncols, kv, pr, partial);
  hipLaunchKernelGGL(sum_blocks_kernel, dim3((ncols + 63) / 64), dim3(64), 0, st, partial, static_cast<int>(nb), ncols,
                     w);
}

void launch_outer_acc(double* R, int64_t n, int ncols, const KronVec& ku, const double* w, double alpha,
                      hipStream_t st) {
  const int64_t total = n * ncols;
  if (total <= 0) return;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(outer_acc_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, R, n, ncols, ku, w,
                     alpha);
}

}  // namespace ttnn
