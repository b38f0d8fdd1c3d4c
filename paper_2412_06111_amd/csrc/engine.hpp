// Host-side drivers of the TTNN engine (enqueue kernels on a stream).
#pragma once

#include "plan.hpp"

namespace ttnn {

void size_chain_scratch(Plan& P);
void zero_accumulators(Plan& P, hipStream_t stream);

// Sketch phase on a box update (Sec. 4; Sec. 5 for STTNN): accumulators += alpha * sketch(H).
void update_box(Plan& P, const void* block, const int64_t* off, const int64_t* ext, double alpha,
                hipStream_t stream);
void update_rank1(Plan& P, const double* const* factors, double alpha, hipStream_t stream);

// Omega_t = Y_t^T R_t and Psi_t = (Y_cm^T kron ... kron Y_c1^T) R_t, FP64, from the accumulators.
void run_epilogue(Plan& P, hipStream_t stream);
// Recovery phase; cores[v] indexed by level-order id.  Returns the numeric status.
ttnn_status run_assemble(Plan& P, double* const* cores, hipStream_t stream);
void run_reconstruct(Plan& P, const double* const* cores, void* out, int out_dtype, hipStream_t stream);

// Core shape of level-order node v.
std::vector<int64_t> core_shape(const Plan& P, int v);

}  // namespace ttnn
