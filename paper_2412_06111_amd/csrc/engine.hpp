// Host-side drivers of the TTNN engine (enqueue kernels on a stream).
#pragma once

#include <string>

#include "kernels.hpp"
#include "plan.hpp"

namespace ttnn {

// One step of a box update on the generic kernels: a contraction and, when it was
// split or accumulates, the fixed-order reduction that delivers it (nchunks is
// filled in at execution).
struct BoxOp {
  GemmArgs g;
  bool reduce = false;
  ReduceTask r;
};

void size_chain_scratch(Plan& P);
void zero_accumulators(Plan& P, hipStream_t stream);

// Sketch phase on a box update (Sec. 4; Sec. 5 for STTNN): accumulators += alpha * sketch(H).
// strides: element strides of the block per mode (read in place), or nullptr = packed.
void update_box(Plan& P, const void* block, const int64_t* off, const int64_t* ext, const int64_t* strides,
                double alpha, hipStream_t stream);
// nterms rank-1 terms: factors holds nterms x order device pointers (term-major),
// alphas nterms host scales; equal, bitwise, to the terms applied one by one in order.
void update_rank1(Plan& P, int nterms, const double* const* factors, const double* alphas, hipStream_t stream);

// The steps of a box update that is not the whole tensor, in order.  Plans with equal
// batch_key() give step lists of equal length whose i-th steps have the same kind, so
// the i-th steps of several such updates can share one launch.
void record_box(Plan& P, const void* block, const int64_t* off, const int64_t* ext, const int64_t* strides,
                double alpha, std::vector<BoxOp>& ops);
void run_box_ops(Plan& P, const std::vector<BoxOp>& ops, hipStream_t stream);
void run_box_ops_batched(const std::vector<Plan*>& plans, const std::vector<const std::vector<BoxOp>*>& items,
                         hipStream_t stream);
std::string batch_key(const Plan& P);
bool whole_tensor(const Plan& P, const int64_t* off, const int64_t* ext);

// Omega_t = Y_t^T R_t and Psi_t = (Y_cm^T kron ... kron Y_c1^T) R_t, FP64, from the accumulators.
void run_epilogue(Plan& P, hipStream_t stream);
// Recovery phase; cores[v] indexed by level-order id.  Returns the numeric status.
// Enqueues the recovery phase; its status lands in the plan's call word and is
// or-ed into the sticky word (no host synchronisation).
void enqueue_assemble(Plan& P, double* const* cores, hipStream_t stream);
// Enqueues and reads this assembly's status back (synchronises `stream`).
ttnn_status run_assemble(Plan& P, double* const* cores, hipStream_t stream);
// Status of every assembly since the last query (synchronises `stream`), then clears it.
ttnn_status assemble_status(Plan& P, hipStream_t stream);
// The same status copied to pinned host memory in stream order (no synchronisation).
void assemble_status_async(Plan& P, int32_t* h_status, hipStream_t stream);
void run_reconstruct(Plan& P, const double* const* cores, void* out, int out_dtype, hipStream_t stream);

// Rows of Psi_t of internal node v: prod of the children's r_c + p_c.
int64_t psi_rows(const Plan& P, int v);
// FP64 mode products on the batched GEMM (see launch_bgemm64):
//   left_job: out(l, j, q) (+)= alpha sum_i H[l + L (i + n q)] M(i, j), M(i, j) = M[i sMi + j sMj],
//             out column-major [L][c][Q]
//   mode_job: position p of an operand with positions `sizes` (first fastest) contracted
//             with M (rows sizes[p], ncols columns), stored.
GJob left_job(const double* H, int64_t L, int64_t n, int64_t Q, const double* M, int64_t sMi, int64_t sMj,
              int64_t c, double* out, int acc, double alpha);
GJob mode_job(const double* in, const std::vector<int64_t>& sizes, int p, const double* M, int64_t sMi,
              int64_t sMj, int64_t ncols, double* out);

// Core shape of level-order node v.
std::vector<int64_t> core_shape(const Plan& P, int v);

}  // namespace ttnn
