// Plan construction: validation of the index tree (Def. 3 read with equality:
// every internal node is the disjoint union of its children; contiguous mode
// intervals), level-order numbering (labels of Fig. 1), STTNN reuse sets
// (Sec. 5 and Fig. 5: preceding siblings of the node and of each ancestor), DRM
// shapes (Sec. 4, eq. "sketch"; Sec. 5 for the reduced X_t of STTNN) and the
// device memory of a plan.
#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "engine.hpp"
#include "fused.hpp"
#include "kernels.hpp"

namespace ttnn {

namespace {
// Plans allocate from a pool of their own per device that keeps released memory
// (release threshold: never), so a plan created after another was released reuses its
// pages instead of mapping new ones.  The pool lives until the process ends.
hipMemPool_t plan_pool() {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;
  int dev = 0;
  TTNN_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) return it->second;
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  TTNN_HIP(hipMemPoolCreate(&pool, &props));
  uint64_t keep = UINT64_MAX;
  TTNN_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  pools[dev] = pool;
  return pool;
}
}  // namespace

void* pool_alloc(size_t bytes, hipStream_t stream) {
  void* a = nullptr;
  if (hipMallocFromPoolAsync(&a, bytes, plan_pool(), stream) != hipSuccess || a == nullptr) {
    (void)hipGetLastError();
    throw Error{TTNN_E_NOMEM, "stream-ordered allocation of " + std::to_string(bytes) + " bytes failed"};
  }
  if (reinterpret_cast<uintptr_t>(a) % 256 != 0) {        // the kernels assume 256-byte aligned arrays
    (void)hipFreeAsync(a, stream);
    throw Error{TTNN_E_NOMEM, "device allocation not 256-byte aligned"};
  }
  return a;
}

void pool_free(void* p, hipStream_t stream) {
  if (p) (void)hipFreeAsync(p, stream);
}

void fill_transposed(Plan& P, hipStream_t stream) {
  for (const Plan::TransposedCopy& c : P.transposed_pending)
    copy_layout(c.src, c.dst, c.dt, c.rows, c.cols, 1, c.cols, 1, 0, 0, c.rows, stream);
  P.transposed_pending.clear();
}

// Device memory of a plan is stream ordered (allocated on the creation stream), so
// releasing it does not synchronise the device: the blocks return to the pool when
// the release stream reaches them.
Plan::~Plan() {
  if (arena && owns_arena) (void)hipFreeAsync(arena, free_stream);
  for (hipEvent_t e : sweep_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : side_ev)
    if (e) (void)hipEventDestroy(e);
  if (side) (void)hipStreamDestroy(side);
}

// One stream-ordered block per plan, sized by a dry build, handed out in order (every
// request rounded to 256 bytes, so every array is 256-byte aligned).
void* Plan::alloc(size_t bytes) {
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~static_cast<size_t>(255);
  if (dry) {
    footprint += bytes;
    return nullptr;
  }
  TTNN_REQUIRE(arena != nullptr && arena_used + bytes <= arena_size, TTNN_E_INVALID,
               "plan memory exceeds its sized footprint");
  void* p = arena + arena_used;
  arena_used += bytes;
  footprint += bytes;
  return p;
}

IndexMap box_rows(const Plan& P, int first, int last, const int64_t* off, const int64_t* ext) {
  IndexMap m;
  int64_t g = 1;
  for (int mu = first; mu <= last; ++mu) {
    m.push(ext[mu], off[mu], g);
    g *= P.dims[mu];
  }
  return m;
}

namespace {

void check_mul(int64_t a, int64_t b, const char* what) {
  if (a > 0 && b > (int64_t(1) << 62) / a)
    throw Error{TTNN_E_INVALID, std::string("size overflow in ") + what};
}

}  // namespace

std::unique_ptr<Plan> build_plan(const ttnn_problem* pr, hipStream_t stream, bool dry, void* ws, size_t ws_bytes) {
  TTNN_REQUIRE(pr != nullptr, TTNN_E_INVALID, "problem is NULL");
  TTNN_REQUIRE(pr->order >= 2 && pr->order <= TTNN_MAX_ORDER, TTNN_E_INVALID, "order must be in [2, 8]");
  TTNN_REQUIRE(pr->dims && pr->parent && pr->first_mode && pr->last_mode && pr->rank && pr->oversample,
               TTNN_E_INVALID, "problem has a NULL array");
  TTNN_REQUIRE(pr->num_nodes >= 2 && pr->num_nodes <= TTNN_MAX_NODES, TTNN_E_TREE,
               "num_nodes must be in [2, 64]");
  TTNN_REQUIRE(pr->variant == TTNN_TTNN || pr->variant == TTNN_STTNN || pr->variant == TTNN_KR, TTNN_E_INVALID,
               "bad variant");
  TTNN_REQUIRE(pr->variant != TTNN_KR || pr->dtype == TTNN_F64, TTNN_E_INVALID,
               "Khatri-Rao plans sketch FP64 TTN cores (dtype F64)");
  TTNN_REQUIRE(pr->dtype == TTNN_F64 || pr->dtype == TTNN_F32 || pr->dtype == TTNN_BF16, TTNN_E_INVALID,
               "bad dtype");
  TTNN_REQUIRE(pr->eps_factor >= 0.0, TTNN_E_INVALID, "eps_factor must be >= 0");

  size_t need = 0;                        // the real build first sizes itself with a dry one
  if (!dry) need = build_plan(pr, stream, true)->footprint;
  auto P = std::make_unique<Plan>();
  P->dry = dry;
  P->stream = stream;
  P->free_stream = stream;
  if (!dry && ws) {                      // the caller's workspace: views only, never freed here
    TTNN_REQUIRE(ws_bytes >= need, TTNN_E_INVALID,
                 "workspace of " + std::to_string(ws_bytes) + " bytes; the plan needs " + std::to_string(need));
    P->arena = static_cast<char*>(ws);
    P->arena_size = need;
    P->owns_arena = false;
  } else if (!dry) {
    P->arena = static_cast<char*>(pool_alloc(need, stream));
    P->arena_size = need;
  }
  P->d = pr->order;
  P->variant = pr->variant;
  P->dtype = pr->dtype;
  P->seed = pr->seed;
  P->eps_factor = pr->eps_factor > 0.0 ? pr->eps_factor : 10.0 * 0x1p-52;
  for (int mu = 0; mu < P->d; ++mu) {
    TTNN_REQUIRE(pr->dims[mu] >= 1, TTNN_E_INVALID, "dims must be >= 1");
    check_mul(P->N, pr->dims[mu], "tensor size");
    P->dims[mu] = pr->dims[mu];
    P->N *= pr->dims[mu];
  }

  // ---- tree structure in caller ids
  const int nn = pr->num_nodes;
  int root = -1;
  std::vector<std::vector<int>> kids(nn);
  for (int i = 0; i < nn; ++i) {
    const int par = pr->parent[i];
    TTNN_REQUIRE(pr->first_mode[i] >= 0 && pr->first_mode[i] <= pr->last_mode[i] && pr->last_mode[i] < P->d,
                 TTNN_E_TREE, "node " + std::to_string(i) + " has a bad mode interval");
    if (par < 0) {
      TTNN_REQUIRE(par == -1 && root < 0, TTNN_E_TREE, "the tree must have exactly one root");
      root = i;
    } else {
      TTNN_REQUIRE(par < nn && par != i, TTNN_E_TREE, "bad parent index");
      kids[par].push_back(i);
    }
  }
  TTNN_REQUIRE(root >= 0, TTNN_E_TREE, "no root");
  TTNN_REQUIRE(pr->first_mode[root] == 0 && pr->last_mode[root] == P->d - 1, TTNN_E_TREE,
               "the root must cover every mode");
  for (int i = 0; i < nn; ++i) {
    std::sort(kids[i].begin(), kids[i].end(),
              [&](int a, int b) { return pr->first_mode[a] < pr->first_mode[b]; });
    if (kids[i].empty()) continue;
    // children are disjoint intervals inside the node's, in order; modes of the node in
    // no child are its free modes (Def. 3: a node contains the union of its children)
    int expect = pr->first_mode[i];
    for (int c : kids[i]) {
      TTNN_REQUIRE(pr->first_mode[c] >= expect && pr->last_mode[c] <= pr->last_mode[i], TTNN_E_TREE,
                   "children of node " + std::to_string(i) + " overlap or leave its interval");
      expect = pr->last_mode[c] + 1;
    }
    if (i != root)
      TTNN_REQUIRE(kids[i].size() >= 2 || pr->first_mode[kids[i][0]] != pr->first_mode[i] ||
                       pr->last_mode[kids[i][0]] != pr->last_mode[i],
                   TTNN_E_TREE, "internal node " + std::to_string(i) + " has a single child equal to itself");
  }
  TTNN_REQUIRE(!kids[root].empty(), TTNN_E_TREE, "the root has no children");

  // ---- level order (breadth first, children left to right); reachability = no cycles
  std::vector<int> order{root};
  std::vector<int> level_caller(nn, -1);
  level_caller[root] = 0;
  for (size_t h = 0; h < order.size(); ++h)
    for (int c : kids[order[h]]) {
      TTNN_REQUIRE(level_caller[c] < 0, TTNN_E_TREE, "the parent links contain a cycle");
      level_caller[c] = level_caller[order[h]] + 1;
      order.push_back(c);
    }
  TTNN_REQUIRE(static_cast<int>(order.size()) == nn, TTNN_E_TREE, "some nodes are not reachable from the root");

  P->level_of_caller.assign(nn, -1);
  for (int v = 0; v < nn; ++v) P->level_of_caller[order[v]] = v;
  P->nodes.resize(nn);
  for (int v = 0; v < nn; ++v) {
    const int c = order[v];
    Node& nd = P->nodes[v];
    nd.caller = c;
    nd.level = level_caller[c];
    nd.parent = pr->parent[c] < 0 ? -1 : P->level_of_caller[pr->parent[c]];
    nd.first = pr->first_mode[c];
    nd.last = pr->last_mode[c];
    for (int k : kids[c]) nd.children.push_back(P->level_of_caller[k]);
    nd.n = 1;
    for (int mu = nd.first; mu <= nd.last; ++mu) nd.n *= P->dims[mu];
    if (v > 0) {
      TTNN_REQUIRE(pr->rank[c] >= 1 && pr->oversample[c] >= 0, TTNN_E_INVALID,
                   "ranks must be >= 1 and oversamples >= 0");
      TTNN_REQUIRE(pr->rank[c] <= 64 && pr->rank[c] + pr->oversample[c] <= 256, TTNN_E_INVALID,
                   "rank <= 64 and rank + oversample <= 256 are supported");
      TTNN_REQUIRE(qr_pinv_fits(pr->rank[c] + pr->oversample[c], pr->rank[c]), TTNN_E_INVALID,
                   "rank " + std::to_string(pr->rank[c]) + " with oversample " + std::to_string(pr->oversample[c]) +
                       ": the recovery of a node holds 2 (r + p) r doubles in one workgroup's LDS "
                       "(at r = 64, p <= 91)");
      nd.r = pr->rank[c];
      nd.p = pr->oversample[c];
      nd.k = nd.r + nd.p;
    }
  }

  // ---- STTNN visiting order of the children (Sec. 5 leaves it free; NULL = left to right)
  for (int v = 0; v < nn; ++v) {
    Node& nd = P->nodes[v];
    nd.visit = nd.children;
    if (!pr->visit) continue;
    const size_t m = nd.children.size();
    std::vector<int> slot(m, -1);
    for (int c : nd.children) {
      const int32_t q = pr->visit[P->nodes[c].caller];
      TTNN_REQUIRE(q >= 0 && static_cast<size_t>(q) < m && slot[q] < 0, TTNN_E_TREE,
                   "visit must number the children of every node 0..m-1 (node " + std::to_string(nd.caller) + ")");
      slot[q] = c;
    }
    if (P->variant != TTNN_STTNN) continue;      // checked, and without effect on TTNN
    nd.visit = slot;
    if (nd.visit != nd.children) P->lex = false;
  }

  // ---- free modes: one identity leaf per free mode, numbered after the caller's nodes
  // (so the caller's level-order ids, which seed the maps, do not move).  Its maps,
  // projector and core are identities (rank n_mu), the convention for dummy nodes.
  P->n_real = nn;
  for (int v = 0; v < nn; ++v) {
    if (P->nodes[v].children.empty()) continue;
    std::vector<char> covered(P->d, 0);
    for (int c : P->nodes[v].children)
      for (int mu = P->nodes[c].first; mu <= P->nodes[c].last; ++mu) covered[mu] = 1;
    for (int mu = P->nodes[v].first; mu <= P->nodes[v].last; ++mu) {
      if (covered[mu]) continue;
      TTNN_REQUIRE(P->variant != TTNN_KR, TTNN_E_TREE, "Khatri-Rao plans take trees without free modes");
      TTNN_REQUIRE(P->nodes.size() < static_cast<size_t>(TTNN_MAX_NODES), TTNN_E_TREE,
                   "more than 64 nodes and free modes");
      Node f;
      f.ident = true;
      f.level = P->nodes[v].level + 1;
      f.parent = v;
      f.first = f.last = mu;
      f.n = P->dims[mu];
      TTNN_REQUIRE(f.n <= 4096, TTNN_E_INVALID, "free modes of size up to 4096 are supported");
      f.r = f.k = static_cast<int>(f.n);
      f.m = f.n;
      const int id = static_cast<int>(P->nodes.size());
      P->nodes.push_back(f);
      P->nodes[v].children.push_back(id);
      P->nodes[v].visit.push_back(id);       // contracted with the identity: last, never a cost
    }
    auto& ch = P->nodes[v].children;
    std::sort(ch.begin(), ch.end(), [&](int a, int b) { return P->nodes[a].first < P->nodes[b].first; });
  }

  if (P->variant == TTNN_KR)                 // X_t, Y_t are Khatri-Rao products of shared per-mode factors
    for (int v = 2; v < nn; ++v)
      TTNN_REQUIRE(P->nodes[v].r == P->nodes[1].r && P->nodes[v].p == P->nodes[1].p, TTNN_E_INVALID,
                   "Khatri-Rao plans need one rank and one oversample for every node");

  // ---- STTNN reuse sets and X_t row positions
  for (int v = 1; v < nn; ++v) {
    Node& nd = P->nodes[v];
    if (P->variant == TTNN_STTNN) {
      // S_t: the siblings visited before t and before each ancestor of t, listed from
      // the top level down (each level in visiting order), so that the chain of
      // contractions T x Y_s^T of a node extends its parent's and its earlier siblings'
      std::vector<std::vector<int>> per_level;
      int cur = v;
      while (P->nodes[cur].parent >= 0) {
        const Node& par = P->nodes[P->nodes[cur].parent];
        std::vector<int> pre;
        for (int s : par.visit) {
          if (s == cur) break;
          pre.push_back(s);
        }
        per_level.push_back(pre);
        cur = P->nodes[cur].parent;
      }
      for (auto it = per_level.rbegin(); it != per_level.rend(); ++it) nd.S.insert(nd.S.end(), it->begin(), it->end());
      // X_t rows: the indices of T_{S_t} outside I_t in mode order, each contracted
      // group one index of size k_s at its place
      std::vector<int> group_of(P->d, -1);
      for (int s : nd.S)
        for (int mu = P->nodes[s].first; mu <= P->nodes[s].last; ++mu) group_of[mu] = s;
      for (int mu = 0; mu < P->d; ++mu) {
        if (mu >= nd.first && mu <= nd.last) continue;
        const int g = group_of[mu];
        if (g >= 0 && mu != P->nodes[g].first) continue;        // inside a group already placed
        nd.xpos.push_back(g < 0 ? P->dims[mu] : P->nodes[g].k);
        if (mu < nd.first) ++nd.xsplit;
      }
    } else {
      for (int mu = 0; mu < P->d; ++mu)
        if (mu < nd.first || mu > nd.last) nd.xpos.push_back(P->dims[mu]);
      nd.xsplit = nd.first;
    }
    nd.m = 1;
    for (int64_t s : nd.xpos) {
      check_mul(nd.m, s, "DRM rows");
      nd.m *= s;
    }
  }

  // ---- device memory
  const bool copy = P->dtype != TTNN_F64;
  const size_t cs = dtype_size(P->dtype);
  const bool kr = P->variant == TTNN_KR;
  for (int v = 1; v < nn && kr; ++v) {     // structured: no dense maps, no R_t of internal nodes
    Node& nd = P->nodes[v];
    nd.Om = static_cast<double*>(P->alloc(sizeof(double) * nd.k * nd.r));
    nd.Q = static_cast<double*>(P->alloc(sizeof(double) * nd.k * nd.r));
    nd.Pinv = static_cast<double*>(P->alloc(sizeof(double) * nd.r * nd.r));
    if (nd.leaf()) {
      check_mul(nd.n, nd.r, "R_t size");
      nd.R = static_cast<double*>(P->alloc(sizeof(double) * nd.n * nd.r));
    } else {
      int64_t kk = 1;
      for (int c : nd.children) {
        check_mul(kk, P->nodes[c].k, "Psi_t size");
        kk *= P->nodes[c].k;
      }
      check_mul(kk, nd.r, "Psi_t size");
      nd.Psi = static_cast<double*>(P->alloc(sizeof(double) * kk * nd.r));
    }
  }
  for (int mu = 0; mu < P->d && kr; ++mu) {
    P->kr_x[mu] = static_cast<double*>(P->alloc(sizeof(double) * P->dims[mu] * P->nodes[1].r));
    P->kr_y[mu] = static_cast<double*>(P->alloc(sizeof(double) * P->dims[mu] * P->nodes[1].k));
  }
  for (int v = 1; v < nn && !kr; ++v) {
    Node& nd = P->nodes[v];
    check_mul(nd.m, nd.r, "X_t size");
    nd.X64 = static_cast<double*>(P->alloc(sizeof(double) * nd.m * nd.r));
    nd.Xc = copy ? P->alloc(cs * nd.m * nd.r) : nd.X64;
    nd.Y64 = static_cast<double*>(P->alloc(sizeof(double) * nd.n * nd.k));
    nd.Yc = copy ? P->alloc(cs * nd.n * nd.k) : nd.Y64;
    nd.R = static_cast<double*>(P->alloc(sizeof(double) * nd.n * nd.r));
    nd.Om = static_cast<double*>(P->alloc(sizeof(double) * nd.k * nd.r));
    nd.Q = static_cast<double*>(P->alloc(sizeof(double) * nd.k * nd.r));
    nd.Pinv = static_cast<double*>(P->alloc(sizeof(double) * nd.r * nd.r));
    if (!nd.leaf()) {
      int64_t kk = 1;
      for (int c : nd.children) {
        check_mul(kk, P->nodes[c].k, "Psi_t size");
        kk *= P->nodes[c].k;
      }
      nd.Psi = static_cast<double*>(P->alloc(sizeof(double) * kk * nd.r));
    }
  }
  for (size_t v = nn; v < P->nodes.size(); ++v) {   // free modes: Y = Q = the identity
    Node& nd = P->nodes[v];
    nd.Y64 = static_cast<double*>(P->alloc(sizeof(double) * nd.n * nd.n));
    nd.Yc = copy ? P->alloc(cs * nd.n * nd.n) : nd.Y64;
    nd.Q = nd.Y64;
  }
  P->psi_root_len = 1;
  for (int c : P->nodes[0].children) {
    check_mul(P->psi_root_len, P->nodes[c].k, "root Psi size");
    P->psi_root_len *= P->nodes[c].k;
  }
  P->psi_root = static_cast<double*>(P->alloc(sizeof(double) * P->psi_root_len));
  P->d_flag = static_cast<int*>(P->alloc(sizeof(int) * 2 * TTNN_MAX_NODES));
  if (!dry) launch_zero_int(P->d_flag, 2 * TTNN_MAX_NODES, stream);     // status words start clear
  P->g64_part_elems = size_t(1) << 21;
  P->g64_part = static_cast<double*>(P->alloc(sizeof(double) * P->g64_part_elems));

  size_chain_scratch(*P);
  P->chain = static_cast<double*>(P->alloc(sizeof(double) * P->chain_elems));
  P->partial = static_cast<double*>(P->alloc(sizeof(double) * P->partial_elems));
  P->work = static_cast<double*>(P->alloc(sizeof(double) * P->work_elems));
  {
    size_t ks = 0, rmax = 1;
    for (size_t v = 1; v < P->nodes.size(); ++v) {       // g_s of every group, free modes too
      ks += static_cast<size_t>(P->nodes[v].k);
      if (!P->nodes[v].ident) rmax = std::max(rmax, static_cast<size_t>(P->nodes[v].r));
    }
    // per term of a rank-1 batch: the g_s (ks) and one node's X_t^T v (rmax)
    P->r1_w = ks;
    P->r1_rmax = rmax;
    P->r1 = static_cast<double*>(P->alloc(sizeof(double) * kRank1Batch * (ks + rmax)));
  }

  // TTNN_DISABLE_FUSED=1 routes every update through the generic kernels (parity checks)
  const char* nf = std::getenv("TTNN_DISABLE_FUSED");
  P->allow_fused = !(nf && nf[0] == '1') && !kr && P->nodes.size() == static_cast<size_t>(nn) && P->lex;
  // transposed DRM copies for whole-tensor right sketches on MFMA (large tensors only,
  // nodes sketched on the raw tensor that the fused kernel does not cover)
  auto plan_xt = [&](bool fill) {
    if (P->N < (int64_t(1) << 22) || kr) return;
    const FusedT4& F = P->fused;
    for (int v = 1; v < nn; ++v) {
      Node& nd = P->nodes[v];
      // Y_t^T applied to the raw tensor when t starts at mode 1 (the first contraction
      // of a chain): T viewed as [n_t][N / n_t] with the contraction index contiguous
      if (nd.first == 0 && right_mfma_eligible(nd.n, P->N / nd.n, 1, nd.k, P->dtype)) {
        nd.Yt = P->alloc(dtype_size(P->dtype) * nd.n * nd.k);
        if (fill) P->transposed_pending.push_back({nd.Y64, nd.Yt, P->dtype, nd.n, nd.k});
      }
      if (F.enabled && (v == F.node_A || v == F.node_1 || v == (F.tt ? F.node_B : F.node_2))) continue;
      if (!nd.S.empty()) {
        // the intermediate T x_{s in S_t} Y_s^T: [positions before t][n_t][after]; only
        // large ones (the small ones share batched FP64 launches), and only while the
        // copy stays modest (it doubles the FP64 DRM of the node)
        int64_t L = 1;
        for (int i = 0; i < nd.xsplit; ++i) L *= nd.xpos[i];
        const int64_t Q = nd.m / L;
        if (L * nd.n * Q >= (int64_t(1) << 22) && nd.m * nd.r <= (int64_t(1) << 26) &&
            right_mfma_eligible(L, nd.n, Q, nd.r, TTNN_F64)) {
          nd.Xt64 = static_cast<double*>(P->alloc(sizeof(double) * nd.m * nd.r));
          if (fill) P->transposed_pending.push_back({nd.X64, nd.Xt64, TTNN_F64, nd.m, nd.r});
        }
        continue;
      }
      int64_t L = 1;
      for (int mu = 0; mu < nd.first; ++mu) L *= P->dims[mu];
      int64_t n = nd.n, Q = nd.m / (L > 0 ? L : 1);
      if (!right_mfma_eligible(L, n, Q, nd.r, P->dtype)) continue;
      nd.Xt = P->alloc(dtype_size(P->dtype) * nd.m * nd.r);
      if (fill) P->transposed_pending.push_back({nd.X64, nd.Xt, P->dtype, nd.m, nd.r});
    }
  };
  if (dry) {
    if (P->allow_fused) fused_prepare(*P, stream);   // sizes its buffers only
    plan_xt(false);
    return P;
  }

  // ---- DRMs and zeroed accumulators
  for (int mu = 0; mu < P->d && kr; ++mu) {          // per-mode factors: tags 2 (64 + mu) + kind
    const uint32_t tx = static_cast<uint32_t>(2 * (TTNN_KR_TAG_BASE + mu)), ty = tx + 1;
    launch_drm(P->dims[mu], P->nodes[1].r, P->seed, tx, P->kr_x[mu], nullptr, nullptr, stream);
    launch_drm(P->dims[mu], P->nodes[1].k, P->seed, ty, P->kr_y[mu], nullptr, nullptr, stream);
  }
  for (size_t v = nn; v < P->nodes.size(); ++v) {
    Node& nd = P->nodes[v];
    launch_eye(nd.n, nd.Y64, P->dtype == TTNN_F32 ? static_cast<float*>(nd.Yc) : nullptr,
               P->dtype == TTNN_BF16 ? static_cast<uint16_t*>(nd.Yc) : nullptr, stream);
  }
  for (int v = 1; v < nn && !kr; ++v) {
    Node& nd = P->nodes[v];
    const uint32_t tx = static_cast<uint32_t>(2 * v + 0), ty = static_cast<uint32_t>(2 * v + 1);
    float* x32 = P->dtype == TTNN_F32 ? static_cast<float*>(nd.Xc) : nullptr;
    uint16_t* x16 = P->dtype == TTNN_BF16 ? static_cast<uint16_t*>(nd.Xc) : nullptr;
    float* y32 = P->dtype == TTNN_F32 ? static_cast<float*>(nd.Yc) : nullptr;
    uint16_t* y16 = P->dtype == TTNN_BF16 ? static_cast<uint16_t*>(nd.Yc) : nullptr;
    launch_drm(nd.m, nd.r, P->seed, tx, nd.X64, x32, x16, stream);
    launch_drm(nd.n, nd.k, P->seed, ty, nd.Y64, y32, y16, stream);
  }
  if (P->allow_fused) fused_prepare(*P, stream);
  plan_xt(true);
  zero_accumulators(*P, stream);
  TTNN_HIP(hipGetLastError());
  return P;
}

}  // namespace ttnn
