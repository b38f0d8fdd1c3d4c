// Plan of the TTNN engine: the validated index tree in level order, per-node DRM
// and sketch shapes, the STTNN reuse sets, and the device memory owned by a plan.
#pragma once

#include <map>
#include <memory>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace ttnn {

struct Node {
  int caller = -1;             // id in the caller's arrays
  int level = 0;
  int parent = -1;             // level-order id
  int first = 0, last = 0;     // 0-based mode interval
  std::vector<int> children;   // level-order ids, left to right
  std::vector<int> visit;      // the children in the STTNN visiting order (free modes last)
  int r = 0, p = 0, k = 0;     // rank, oversample, r + p
  int64_t n = 1;               // n_t = prod of dims over the interval
  int64_t m = 1;               // rows of X_t
  std::vector<int> S;          // STTNN reuse set (level-order ids) in the order its chain of
                               // contractions takes them: the ancestors' groups first
  std::vector<int64_t> xpos;   // sizes of the positions indexing the rows of X_t, in order
  int xsplit = 0;              // how many of them come before the modes of t
  bool ident = false;          // a free mode of the parent: identity maps, projector and core
                               // (r = k = n); no sketches of its own
  bool leaf() const { return children.empty(); }

  // device memory (views into the plan's allocations)
  double* X64 = nullptr;       // m x r row-major
  void* Xc = nullptr;          // compute-dtype copy (== X64 for FP64 plans)
  void* Xt = nullptr;          // transposed compute-dtype copy (r x m) for whole-tensor MFMA sketches
  double* Xt64 = nullptr;      // transposed FP64 copy (r x m) for MFMA right sketches of the
                               // FP64 intermediates (STTNN nodes with a reuse set)
  void* Yt = nullptr;          // transposed compute-dtype copy (k x n) for whole-tensor MFMA
                               // contractions with Y^T of a node that starts at mode 1
  double* Y64 = nullptr;       // n x k row-major
  void* Yc = nullptr;
  double* R = nullptr;         // n x r column-major FP64 accumulator
  double* Om = nullptr;        // k x r column-major
  double* Psi = nullptr;       // internal nodes: prod(k_c) x r column-major
  double* Q = nullptr;         // k x r column-major
  double* Pinv = nullptr;      // r x r column-major
};

// Fused one-pass STTNN kernel state (trees whose first root child is ({1},{2}))
struct FusedT4 {
  bool enabled = false;
  int R = 0, KP = 0, k = 0, B2 = 0, SC = 0, TA = 0, TB = 0, CB = 0;
  int64_t n2 = 0, nA = 0, nB = 0;
  int node_A = -1, node_1 = -1, node_2 = -1, node_B = -1;
  bool tt = false;                         // TTNN mode: R_B instead of the R_2 chain
  bool zout = false;                       // STTNN: Z1 written out, R_2 by a streaming contraction
  void* Z1 = nullptr;
  void *XA = nullptr, *X1 = nullptr, *YA = nullptr, *Y1 = nullptr, *X2 = nullptr, *XB = nullptr;
  void *PRA = nullptr, *PZA = nullptr, *PR1 = nullptr, *PR2 = nullptr, *PRB = nullptr;
};

struct Plan {
  int d = 0;
  int64_t dims[TTNN_MAX_ORDER] = {};
  int variant = TTNN_TTNN;
  int dtype = TTNN_F64;
  uint64_t seed = 0;
  double eps_factor = 0.0;
  std::vector<Node> nodes;                 // level order, root = 0; then the free modes' identity leaves
  int n_real = 0;                          // the caller's nodes: ids below n_real
  std::vector<int> level_of_caller;        // caller id -> level-order id
  int64_t N = 1;

  double* psi_root = nullptr;              // prod(k_c) FP64 accumulator
  int64_t psi_root_len = 0;

  // Khatri-Rao plans (Sec. 7): per-mode factors X_mu (n_mu x r) and Y_mu (n_mu x k),
  // row-major FP64; the nodes hold Omega_t, Psi_t (internal) and R_t (leaves) only
  double* kr_x[TTNN_MAX_ORDER] = {};
  double* kr_y[TTNN_MAX_ORDER] = {};
  bool recon_ok = true;                    // reconstruction scratch sized (not for large structured plans)

  // chain intermediates of the generic update path, keyed by contraction prefix
  std::map<std::vector<int>, size_t> prefix_offset;   // element offset into chain scratch
  double* chain = nullptr;
  size_t chain_elems = 0;
  double* partial = nullptr;               // split-K partials
  size_t partial_elems = 0;
  double* r1 = nullptr;                    // rank-1 updates: per batch term the g_s vectors
                                           // (r1_w each), then per term one X_t^T v (r1_rmax)
  size_t r1_w = 0;                         // g_s entries of a term (sum of k_s)
  size_t r1_rmax = 1;                      // largest r_t
  double* work = nullptr;                  // assembly / reconstruction scratch
  size_t work_elems = 0;
  int* d_flag = nullptr;                   // numeric-status flag written by kernels
  double* g64_part = nullptr;              // split-contraction scratch of the batched FP64 GEMM
  size_t g64_part_elems = 0;

  char* arena = nullptr;                   // the plan's one device block
  size_t arena_size = 0, arena_used = 0;
  bool owns_arena = true;                  // false: a caller-owned workspace (ttnn_plan)
  hipStream_t stream = nullptr;            // creation stream: allocations are ordered on it
  hipStream_t free_stream = nullptr;       // release stream (ttnn_destroy_async may change it)
  size_t footprint = 0;
  bool dry = false;                        // sizing only: alloc() counts and returns nullptr
  ttnn_status sticky = TTNN_OK;
  bool epilogue_valid = false;             // Om / Psi reflect the accumulators
  bool has_cores = false;
  FusedT4 fused;
  bool allow_fused = true;                 // off: every update takes the generic path
  bool lex = true;                         // STTNN visits the children left to right
  // measurement hook: events around the sweep of the last update (see ttnn_set_timing)
  bool timing = false;
  hipEvent_t sweep_ev[2] = {nullptr, nullptr};
  bool sweep_recorded = false;
  // side stream (default priority) for work that may run beside the caller's stream:
  // side_ev[0] forks it, side_ev[1] marks its end
  hipStream_t side = nullptr;
  hipEvent_t side_ev[2] = {nullptr, nullptr};
  bool side_pending = false;
  int rank1_form = TTNN_R1_TERMWISE;       // how rank-1 updates form X_t^T v_t
  // transposed DRM copies (Xt, Yt, Xt64) for the MFMA forms of whole-tensor updates:
  // reserved at creation, filled from the FP64 masters by the first whole-tensor update
  // (plans fed only boxes and rank-1 terms never read them)
  struct TransposedCopy {
    const double* src;
    void* dst;
    int dt;
    int64_t rows, cols;
  };
  std::vector<TransposedCopy> transposed_pending;

  ~Plan();
  void* alloc(size_t bytes);
};

// construction / validation (host); throws Error
// dry: validate and size everything, allocate nothing and launch nothing (the
// returned plan only reports its footprint).  ws: a caller-owned device workspace of
// ws_bytes (256-byte aligned) that holds every array of the plan; without it the plan
// allocates one block from the library's per-device pool.
std::unique_ptr<Plan> build_plan(const ttnn_problem* pr, hipStream_t stream, bool dry = false, void* ws = nullptr,
                                 size_t ws_bytes = 0);

// Fills the transposed DRM copies still pending, on `stream` (no-op once done).
void fill_transposed(Plan& P, hipStream_t stream);

// Stream-ordered device memory from the library's per-device pool (plans and per-call
// scratch); throws TTNN_E_NOMEM.
void* pool_alloc(size_t bytes, hipStream_t stream);
void pool_free(void* p, hipStream_t stream);

// IndexMap from a set of consecutive modes of a box to the column-major index of
// the same modes in the full tensor
IndexMap box_rows(const Plan& P, int first, int last, const int64_t* off, const int64_t* ext);

}  // namespace ttnn
