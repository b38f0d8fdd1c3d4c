// Fused one-pass sketch kernels for large dense updates (see fused.hip).
#pragma once

#include <vector>

#include "plan.hpp"

namespace ttnn {

// Plan-time setup: decides whether the plan's shape is covered and, if so, builds
// the DRM copies in the kernel's fragment layouts and the partial-sum buffers.
void fused_prepare(Plan& P, hipStream_t stream);

// Runs the fused part of the sketch phase of a box update when covered; reports
// the nodes whose accumulators it updated and the contraction prefixes it stored
// in the chain scratch.  Returns false (doing nothing) otherwise.
bool try_fused_update(Plan& P, const void* block, const int64_t* off, const int64_t* ext, double alpha,
                      hipStream_t stream, std::vector<int>* done_nodes, std::vector<std::vector<int>>* done_prefixes);

// Work forked onto the plan's side stream (created on first use) after everything
// enqueued so far on `stream`; join_side makes `stream` wait for it (no-op when none
// is pending).  A fused update leaves its side work pending; the update joins it
// before returning and before any other launch that shares the partial scratch.
// `after`: an event just recorded on `stream` to fork from instead of recording one
// (NULL: record the plan's own fork event).
void fork_side(Plan& P, hipStream_t stream, hipEvent_t after = nullptr);
void join_side(Plan& P, hipStream_t stream);

}  // namespace ttnn
