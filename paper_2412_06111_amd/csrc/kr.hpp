// Khatri-Rao structured sketches of TTN-format tensors (Sec. 7): the shared-column tree
// contraction kernel and the host driver of the structured sketch and of TTN inner
// products.
#pragma once

#include <vector>

#include "common.hpp"

namespace ttnn {

struct Plan;

constexpr int kMaxAxes = TTNN_MAX_ORDER + 1;
constexpr int kMaxKJobs = 8;

// out[o, j] = sum over every core index but axis oax of core[idx] prod_{q != oax}
// fac[q][idx_q * cols + j]; core column-major with axis sizes size[0..naxes), out
// row-major size[oax] x cols.  G > 1 splits the reduction over G workgroups whose
// partials (part, G * size[oax] * cols doubles) are added in order by a second kernel.
struct KJob {
  const double* core = nullptr;
  const double* fac[kMaxAxes] = {};
  int64_t size[kMaxAxes] = {};
  double* out = nullptr;
  double* part = nullptr;
  int32_t naxes = 0, oax = 0, cols = 0, G = 1;
  // filled by the launcher
  int64_t kred = 0, colchunks = 0, otiles = 0, first_block = 0, fold_first = 0;
};
struct KJobList {
  KJob jobs[kMaxKJobs];
  int n;
};

// Reduction split of a contraction with so output rows and cols columns whose reduction
// runs over an inner axis of n0 values and nouter outer combinations (a function of the
// shapes only).
int kr_split(int64_t so, int cols, int64_t n0, int64_t nouter);
// Partial scratch a job needs (0 when G == 1).
size_t kr_part_elems(const KJob& j);
// Launch independent jobs (several kernels of at most kMaxKJobs jobs each).
void launch_kr_contract(std::vector<KJob> jobs, hipStream_t stream);

// ---- host driver (kr.cpp)
// Device scratch (bytes) of one structured update of a TTN with ranks s (level order,
// s[0] unused) and of one inner product of TTNs with ranks sa, sb.
size_t kr_update_work_bytes(const Plan& P, const std::vector<int64_t>& s);
size_t ttn_dot_work_bytes(const Plan& P, const std::vector<int64_t>& sa, const std::vector<int64_t>& sb);
// Accumulators of a Khatri-Rao plan += alpha * sketch of the TTN with cores[v] (level
// order, layout of the assembled cores, ranks s).  work: kr_update_work_bytes bytes.
void update_ttn(Plan& P, const double* const* cores, const std::vector<int64_t>& s, double alpha, void* work,
                hipStream_t stream);
// <A, B> of two TTNs on the plan's tree into d_out[0] (device), in stream order.
void ttn_dot(Plan& P, const double* const* a, const std::vector<int64_t>& sa, const double* const* b,
             const std::vector<int64_t>& sb, double* d_out, void* work, hipStream_t stream);

}  // namespace ttnn
