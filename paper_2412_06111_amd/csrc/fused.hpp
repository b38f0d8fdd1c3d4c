// Fused one-pass sketch kernels for large dense updates (see fused.hip).
#pragma once

#include "plan.hpp"

namespace ttnn {

// Runs the whole sketch phase of a box update with the fused kernels when the
// plan and the box have a shape they cover; returns false (doing nothing) otherwise.
bool try_fused_update(Plan& P, const void* block, const int64_t* off, const int64_t* ext, double alpha,
                      hipStream_t stream);

}  // namespace ttnn
