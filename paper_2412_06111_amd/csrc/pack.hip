// Packing of a strided block: dst (column-major over the box extents, first mode
// fastest) = the block read through its element strides.  A large box read in place
// takes the generic contractions with per-position address maps for every node; packed
// once (one read and one write of the box at streaming speed) it takes the same
// kernels on contiguous data, with the same chunks and sums (so the same bits).
#include "kernels.hpp"

namespace ttnn {
namespace {

template <typename W>
__global__ __launch_bounds__(256) void pack_box_kernel(const W* __restrict__ src, int d, PackDims pd,
                                                       W* __restrict__ dst, int64_t total) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int64_t rest = e, off = 0;
    for (int m = 0; m < d; ++m) {
      const int64_t q = rest / pd.ext[m];
      off += (rest - q * pd.ext[m]) * pd.stride[m];
      rest = q;
    }
    dst[e] = src[off];
  }
}

}  // namespace

void launch_pack_box(const void* src, int dt, int d, const int64_t* ext, const int64_t* strides, void* dst,
                     hipStream_t st) {
  PackDims pd;
  int64_t total = 1;
  for (int m = 0; m < d; ++m) {
    pd.ext[m] = ext[m];
    pd.stride[m] = strides[m];
    total *= ext[m];
  }
  if (total <= 0) return;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  const dim3 grid(static_cast<unsigned>(blocks));
  if (dt == TTNN_F64)
    hipLaunchKernelGGL(pack_box_kernel<uint64_t>, grid, dim3(256), 0, st, static_cast<const uint64_t*>(src), d, pd,
                       static_cast<uint64_t*>(dst), total);
  else if (dt == TTNN_F32)
    hipLaunchKernelGGL(pack_box_kernel<uint32_t>, grid, dim3(256), 0, st, static_cast<const uint32_t*>(src), d, pd,
                       static_cast<uint32_t*>(dst), total);
  else
    hipLaunchKernelGGL(pack_box_kernel<uint16_t>, grid, dim3(256), 0, st, static_cast<const uint16_t*>(src), d, pd,
                       static_cast<uint16_t*>(dst), total);
  TTNN_HIP(hipGetLastError());
}

}  // namespace ttnn
