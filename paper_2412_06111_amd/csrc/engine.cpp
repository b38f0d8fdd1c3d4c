// Drivers of the sketch phase (Sec. 4 and 5), the FP64 epilogue that forms the
// "left" and "intersection" sketches from the accumulated right sketches, the
// recovery phase (Sec. 4, Alg. 2) and the reconstruction (Def. 5, matricised form).
//
// State kept per plan (all FP64, linear in the tensor, Sec. 4 streaming paragraph):
//   R_t for every non-root node t   (TTNN: T^{t} X_t;  STTNN: (T_{S_t})^{t} X_t)
//   Psi_0 at the root               (T contracted with Y_c^T over every child c)
// Omega_t = Y_t^T R_t and Psi_t = (kron_c Y_c^T) R_t are formed on demand.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>

#include "engine.hpp"
#include "fused.hpp"
#include "kernels.hpp"

namespace ttnn {

// d_flag: [0] non-finite count, [1, nn) kept singular values per node, then the call
// and sticky status words at the end of the array
constexpr int kCallWord = 2 * TTNN_MAX_NODES - 2, kStickyWord = 2 * TTNN_MAX_NODES - 1;

namespace {

// one index position of an operand during a contraction chain
struct Pos {
  int64_t ext;     // extent in the operand
  int64_t off;     // offset of the box in this position (0 for contracted indices)
  int64_t glob;    // full size (tensor dim, or r_s + p_s for a contracted group)
  int mode_first;  // first mode covered (contracted groups cover several)
  bool contracted;
};

int64_t prod_ext(const std::vector<Pos>& ps, size_t a, size_t b) {
  int64_t p = 1;
  for (size_t i = a; i < b; ++i) p *= ps[i].ext;
  return p;
}

// positions of the operand obtained from the box after contracting the groups of
// `prefix` (disjoint, in any order): in mode order, each contracted group one position
// of size k at its place
std::vector<Pos> positions_after(const Plan& P, const std::vector<int>& prefix, const int64_t* off,
                                 const int64_t* ext) {
  int group_of[TTNN_MAX_ORDER];
  for (int mu = 0; mu < P.d; ++mu) group_of[mu] = -1;
  for (int s : prefix)
    for (int mu = P.nodes[s].first; mu <= P.nodes[s].last; ++mu) group_of[mu] = s;
  std::vector<Pos> ps;
  for (int mu = 0; mu < P.d; ++mu) {
    const int s = group_of[mu];
    if (s < 0) {
      ps.push_back(Pos{ext[mu], off[mu], P.dims[mu], mu, false});
    } else if (mu == P.nodes[s].first) {
      const Node& g = P.nodes[s];
      ps.push_back(Pos{g.k, 0, g.k, g.first, true});
    }
  }
  return ps;
}

int position_of_mode(const std::vector<Pos>& ps, int mode) {
  for (size_t i = 0; i < ps.size(); ++i)
    if (!ps[i].contracted && ps[i].mode_first == mode) return static_cast<int>(i);
  return -1;
}

// Store (or accumulate) a LEFT contraction on the generic kernel, splitting the
// contraction when the output is small.  mode: 2 = store, 1 = accumulate alpha * result.
void left_op(Plan& P, GemmArgs g, double* dst, int mode, double alpha, hipStream_t st) {
  g.right = false;
  const int64_t rows = g.L * g.Q;
  g.nchunks = pick_chunks(rows, g.ncols, g.n, P.partial_elems);
  if (g.nchunks == 1 && mode == 2) {
    g.out = dst;
    g.out_f32 = false;
    g.ol = OutLayout{g.L, 1, g.L, g.L * g.ncols, 0};
    launch_gemm(g, st);
    return;
  }
  g.out = P.partial;
  g.out_f32 = false;
  g.ol = OutLayout{INT64_MAX, g.ncols, 1, 0, rows * g.ncols};
  const int nch = launch_gemm(g, st);
  if (nch == 0) return;
  IndexMap none;
  launch_reduce(P.partial, nch, rows, g.ncols, mode, alpha, none, 0, dst, g.L, g.ncols, st);
}

}  // namespace

// Dense FP64 mode product as a batched-GEMM job: the operand H is [L][n][Q]
// (L fastest); out[l][j][q] = (acc ? out : 0) + alpha * sum_i H[l][i][q] M(i, j),
// M(i, j) = M[i sMi + j sMj], j < c.
GJob left_job(const double* H, int64_t L, int64_t n, int64_t Q, const double* M, int64_t sMi, int64_t sMj,
              int64_t c, double* out, int acc, double alpha) {
  GJob j;
  j.K = n;
  j.N = c;
  j.B = M;
  j.sBk = sMi;
  j.sBn = sMj;
  j.A = H;
  j.C = out;
  j.accumulate = acc;
  j.alpha = alpha;
  if (L == 1) {            // one GEMM: rows q
    j.M = Q;
    j.sAm = n;
    j.sAk = 1;
    j.sCm = c;
    j.sCn = 1;
  } else {                 // one GEMM per q
    j.M = L;
    j.nbC = static_cast<int>(Q);
    j.sAm = 1;
    j.sAk = L;
    j.sAc = L * n;
    j.sCm = 1;
    j.sCn = L;
    j.sCc = L * c;
  }
  return j;
}

namespace {

// Dense FP64 right sketch as a job: R(i, j) += alpha * sum_{l,q} H[l][i][q] X[(l + L q) r + j]
// with R column-major n x r.
GJob right_job(const double* H, int64_t L, int64_t n, int64_t Q, const double* X, int64_t r, double* R,
               double alpha) {
  GJob j;
  j.M = n;
  j.N = r;
  j.A = H;
  j.B = X;
  j.C = R;
  j.sCm = 1;
  j.sCn = n;
  j.sBn = 1;
  j.accumulate = 1;
  j.alpha = alpha;
  if (L == 1) {
    j.K = Q;
    j.sAm = 1;
    j.sAk = n;
    j.sBk = r;
  } else {
    j.K = L;
    j.nbK = static_cast<int>(Q);
    j.sAm = L;
    j.sAk = 1;
    j.sAkb = L * n;
    j.sBk = r;
    j.sBkb = L * r;
  }
  return j;
}

// Jobs collected between dependency points and launched together.
struct Batch {
  Plan& P;
  hipStream_t st;
  std::vector<GJob> jobs;
  std::vector<const void*> outs;
  Batch(Plan& p, hipStream_t s) : P(p), st(s) {}
  void add(const GJob& j) {
    jobs.push_back(j);
    outs.push_back(j.C);
  }
  bool writes(const void* p) const { return std::find(outs.begin(), outs.end(), p) != outs.end(); }
  void flush() {
    if (jobs.empty()) return;
    launch_bgemm64(jobs, P.g64_part, P.g64_part_elems, st);
    jobs.clear();
    outs.clear();
  }
};

}  // namespace

// FP64 dense mode product on an operand with positions `sizes` (first fastest):
// contract position p with M (rows = sizes[p]; M(i, j) at M[i*sMi + j*sMj]), j < ncols.
GJob mode_job(const double* in, const std::vector<int64_t>& sizes, int p, const double* M, int64_t sMi,
              int64_t sMj, int64_t ncols, double* out) {
  int64_t L = 1, Q = 1;
  for (int i = 0; i < p; ++i) L *= sizes[i];
  for (size_t i = p + 1; i < sizes.size(); ++i) Q *= sizes[i];
  return left_job(in, L, sizes[p], Q, M, sMi, sMj, ncols, out, 0, 1.0);
}

namespace {

// Operand addressing of a contraction that reads the raw block, whose contracted
// positions are the modes [p0, p0 + w): packed, or in place with the caller's strides.
HMap raw_hmap(const Plan& P, const int64_t* ext, const int64_t* strides, int p0, int w) {
  HMap h;
  if (!strides) return h;
  h.strided = 1;
  for (int mu = 0; mu < P.d; ++mu) {
    IndexMap& m = mu < p0 ? h.ml : mu < p0 + w ? h.mi : h.mq;
    m.push(ext[mu], 0, strides[mu]);
  }
  return h;
}

bool whole_box(const Plan& P, const int64_t* off, const int64_t* ext) {
  for (int mu = 0; mu < P.d; ++mu)
    if (off[mu] != 0 || ext[mu] != P.dims[mu]) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------- sizing
void size_chain_scratch(Plan& P) {
  // Khatri-Rao plans take no box updates (no chains, no split partials) and keep no
  // R_t of internal nodes; they size the reconstruction only for tensors that fit
  const bool kr = P.variant == TTNN_KR;
  std::vector<std::vector<int>> prefixes;
  auto add_prefixes = [&](const std::vector<int>& chain, size_t upto) {
    for (size_t j = 1; j <= upto && j <= chain.size(); ++j)
      prefixes.emplace_back(chain.begin(), chain.begin() + j);
  };
  if (!kr) {
    for (size_t v = 1; v < P.nodes.size(); ++v) add_prefixes(P.nodes[v].S, P.nodes[v].S.size());
    const auto& rc = P.nodes[0].visit;
    add_prefixes(rc, rc.size() - 1);      // the last root step accumulates into Psi_0
  }
  size_t total = 0;
  for (auto& pf : prefixes) {
    if (P.prefix_offset.count(pf)) continue;
    // T with the groups of pf contracted: k_s for each group, n_mu for every other mode
    std::vector<char> covered(P.d, 0);
    int64_t e = 1;
    for (int s : pf) {
      e *= P.nodes[s].k;
      for (int mu = P.nodes[s].first; mu <= P.nodes[s].last; ++mu) covered[mu] = 1;
    }
    for (int mu = 0; mu < P.d; ++mu)
      if (!covered[mu]) e *= P.dims[mu];
    P.prefix_offset[pf] = total;
    total += static_cast<size_t>(e);
  }
  P.chain_elems = std::max<size_t>(total, 1);

  size_t part = kr ? 1 : size_t(1) << 22;
  for (size_t v = 1; v < P.nodes.size() && !kr; ++v) {
    const Node& nd = P.nodes[v];
    part = std::max(part, static_cast<size_t>(nd.n * nd.r));
    part = std::max(part, static_cast<size_t>(nd.k * nd.r));
  }
  if (!kr) part = std::max(part, static_cast<size_t>(P.psi_root_len));
  P.partial_elems = part;

  // work buffer: every intermediate of the epilogue chains, of the core chains, and
  // the reconstruction's U_t plus two ping-pong buffers
  size_t epi = 0, core = 0, ustore = 0, rinter = 1;
  for (size_t v = 0; v < P.nodes.size(); ++v) {
    const Node& nd = P.nodes[v];
    if (nd.leaf()) continue;
    const size_t m = nd.children.size();
    const int64_t rt = v == 0 ? 1 : nd.r;
    for (size_t step = 0; step + 1 < m; ++step) {          // epilogue: after step s, k for <= s, n after
      if (v == 0 || kr) break;
      int64_t e = rt;
      for (size_t j = 0; j < m; ++j) e *= j <= step ? P.nodes[nd.children[j]].k : P.nodes[nd.children[j]].n;
      epi += static_cast<size_t>(e);
    }
    const size_t nsteps = m + (v > 0 ? 1 : 0);
    for (size_t step = 0; step + 1 < nsteps; ++step) {     // cores: r for <= s, k after
      int64_t e = rt;
      for (size_t j = 0; j < m; ++j) e *= j <= step ? P.nodes[nd.children[j]].r : P.nodes[nd.children[j]].k;
      core += static_cast<size_t>(e);
    }
    for (size_t step = 0; step + 1 < m; ++step) {          // reconstruction: n for <= s, r after
      int64_t e = rt;
      for (size_t j = 0; j < m; ++j) e *= j <= step ? P.nodes[nd.children[j]].n : P.nodes[nd.children[j]].r;
      rinter = std::max(rinter, static_cast<size_t>(e));
    }
    if (v != 0) ustore += static_cast<size_t>(nd.n * nd.r);
  }
  P.recon_ok = !kr || ustore + 2 * rinter <= (size_t(1) << 27);
  P.work_elems = std::max({epi, core, P.recon_ok ? ustore + 2 * rinter : size_t(1), size_t(1)});
}

void zero_accumulators(Plan& P, hipStream_t st) {
  SegList s;
  if (P.variant == TTNN_KR) {               // structured plans accumulate Omega_t and Psi_t directly
    for (size_t v = 1; v < P.nodes.size(); ++v) {
      const Node& t = P.nodes[v];
      s.push(t.Om, t.k * t.r);
      if (t.leaf()) s.push(t.R, t.n * t.r);
      else s.push(t.Psi, psi_rows(P, static_cast<int>(v)) * t.r);
    }
  } else {
    for (size_t v = 1; v < P.nodes.size(); ++v)
      if (!P.nodes[v].ident) s.push(P.nodes[v].R, P.nodes[v].n * P.nodes[v].r);
  }
  s.push(P.psi_root, P.psi_root_len);
  launch_zero_list(s, st);
  P.epilogue_valid = P.variant == TTNN_KR;
}

int64_t psi_rows(const Plan& P, int v) {
  int64_t kk = 1;
  for (int c : P.nodes[v].children) kk *= P.nodes[c].k;
  return kk;
}

// ---------------------------------------------------------------- sketch phase
bool whole_tensor(const Plan& P, const int64_t* off, const int64_t* ext) { return whole_box(P, off, ext); }

std::string batch_key(const Plan& P) {
  std::string k = std::to_string(P.variant) + "/" + std::to_string(P.dtype) + "/" + std::to_string(P.d);
  for (const Node& nd : P.nodes)
    k += "/" + std::to_string(nd.parent) + ":" + std::to_string(nd.first) + "-" + std::to_string(nd.last);
  return k;
}

void record_box(Plan& P, const void* block, const int64_t* off, const int64_t* ext, const int64_t* strides,
                double alpha, std::vector<BoxOp>& ops) {
  const int cd = P.dtype;
  std::map<std::vector<int>, bool> done;
  auto chain_ptr = [&](const std::vector<int>& pf) { return P.chain + P.prefix_offset.at(pf); };

  // LEFT contraction into dst: mode 2 stores, mode 1 accumulates a * result
  auto left = [&](GemmArgs g, double* dst, int mode, double a) {
    g.right = false;
    const int64_t rows = g.L * g.Q;
    g.nchunks = pick_chunks(rows, g.ncols, g.n, P.partial_elems);
    g.out_f32 = false;
    BoxOp op;
    if (g.nchunks == 1 && mode == 2) {
      g.out = dst;
      g.ol = OutLayout{g.L, 1, g.L, g.L * g.ncols, 0};
    } else {
      g.out = P.partial;
      g.ol = OutLayout{INT64_MAX, g.ncols, 1, 0, rows * g.ncols};
      op.reduce = true;
      op.r.part = P.partial;
      op.r.rows = rows;
      op.r.ncols = g.ncols;
      op.r.mode = mode;
      op.r.alpha = a;
      op.r.dst = dst;
      op.r.L = g.L;
      op.r.kdim = g.ncols;
    }
    op.g = g;
    ops.push_back(op);
  };
  // contraction of a group g of the operand `before` (raw block if empty) with Y_g
  auto group_args = [&](const std::vector<int>& before, const Node& g) {
    const std::vector<Pos> ps = positions_after(P, before, off, ext);
    const int p0 = position_of_mode(ps, g.first);
    const int w = g.last - g.first + 1;
    GemmArgs a;
    a.H = before.empty() ? block : static_cast<const void*>(chain_ptr(before));
    a.th = before.empty() ? cd : TTNN_F64;
    a.L = prod_ext(ps, 0, p0);
    a.n = prod_ext(ps, p0, p0 + w);
    a.Q = prod_ext(ps, p0 + w, ps.size());
    a.D = before.empty() ? g.Yc : static_cast<const void*>(g.Y64);
    a.td = before.empty() ? cd : TTNN_F64;
    a.sDr = g.k;
    a.sDc = 1;
    a.ncols = g.k;
    a.amap = box_rows(P, g.first, g.last, off, ext);
    if (before.empty()) a.hm = raw_hmap(P, ext, strides, p0, w);
    return a;
  };
  auto operand = [&](const std::vector<int>& prefix) -> const void* {
    if (prefix.empty()) return block;
    std::vector<int> chain;
    for (size_t j = 0; j < prefix.size(); ++j) {
      chain.push_back(prefix[j]);
      if (done[chain]) continue;
      std::vector<int> before(chain.begin(), chain.end() - 1);
      left(group_args(before, P.nodes[chain.back()]), chain_ptr(chain), 2, 1.0);
      done[chain] = true;
    }
    return chain_ptr(prefix);
  };

  for (size_t v = 1; v < P.nodes.size(); ++v) {
    Node& t = P.nodes[v];
    if (t.ident) continue;                      // a free mode: no sketch of its own
    const std::vector<int>& pre = t.S;          // empty for TTNN
    const void* in = operand(pre);
    const std::vector<Pos> ps = positions_after(P, pre, off, ext);
    const int p0 = position_of_mode(ps, t.first);
    const int w = t.last - t.first + 1;
    // X_t rows: every position except those of t, first fastest
    IndexMap amap, bmap;
    int64_t C = 1;
    for (int i = 0; i < static_cast<int>(ps.size()); ++i) {
      if (i >= p0 && i < p0 + w) continue;
      if (i < p0) amap.push(ps[i].ext, ps[i].off, C);
      else bmap.push(ps[i].ext, ps[i].off, C);
      C *= ps[i].glob;
    }
    BoxOp op;
    GemmArgs& a = op.g;
    a.right = true;
    a.H = in;
    a.th = pre.empty() ? cd : TTNN_F64;
    a.L = prod_ext(ps, 0, p0);
    a.n = prod_ext(ps, p0, p0 + w);
    a.Q = prod_ext(ps, p0 + w, ps.size());
    a.D = pre.empty() ? t.Xc : static_cast<const void*>(t.X64);
    a.td = pre.empty() ? cd : TTNN_F64;
    a.sDr = t.r;
    a.sDc = 1;
    a.ncols = t.r;
    a.amap = amap;
    a.bmap = bmap;
    if (pre.empty()) a.hm = raw_hmap(P, ext, strides, p0, w);
    a.nchunks = pick_chunks(a.n, a.ncols, a.L * a.Q, P.partial_elems);
    a.out = P.partial;
    a.ol = OutLayout{INT64_MAX, a.ncols, 1, 0, a.n * a.ncols};
    op.reduce = true;
    op.r.part = P.partial;
    op.r.rows = a.n;
    op.r.ncols = a.ncols;
    op.r.mode = 0;
    op.r.alpha = alpha;
    op.r.rmap = box_rows(P, t.first, t.last, off, ext);
    op.r.ldr = t.n;
    op.r.dst = t.R;
    ops.push_back(op);
  }

  // root: T x_{c1} Y_c1^T ... x_{cm} Y_cm^T accumulated into Psi_0 (contracted in the
  // visiting order; the result keeps the children in mode order, c1 fastest)
  const auto& rc = P.nodes[0].visit;
  std::vector<int> before(rc.begin(), rc.end() - 1);
  operand(before);
  left(group_args(before, P.nodes[rc.back()]), P.psi_root, 1, alpha);
}

void run_box_ops_batched(const std::vector<Plan*>& plans, const std::vector<const std::vector<BoxOp>*>& items,
                         hipStream_t st) {
  // The steps of each update are grouped, in order, into levels: a step joins the
  // current level unless it reads a buffer that a step of the level writes, or its
  // partial sums no longer fit its plan's scratch next to those of the level (every step
  // gets its own slice).  Level l of every update in the call runs as one batched
  // contraction launch per kind of step and one batched reduction launch; updates
  // depend only on their own earlier levels.  Every step keeps its chunking and
  // summation order, so the results are bitwise those of running the steps one by one,
  // update by update.  All descriptor tables are built first and staged in one copy.
  TTNN_REQUIRE(plans.size() == items.size(), TTNN_E_INVALID, "one plan per batched update");
  std::vector<std::vector<BoxOp>> ops(items.size());
  std::vector<std::vector<int>> level(items.size());
  int nlev = 0;
  for (size_t u = 0; u < items.size(); ++u) {
    ops[u] = *items[u];
    Plan& P = *plans[u];
    level[u].assign(ops[u].size(), 0);
    std::vector<const void*> written;
    size_t used = 0;
    int lv = 0;
    for (size_t k = 0; k < ops[u].size(); ++k) {
      BoxOp& op = ops[u][k];
      const int nch = gemm_chunks(op.g, nullptr);
      const size_t need = op.reduce && nch > 0 ? static_cast<size_t>(nch) * op.r.rows * op.r.ncols : 0;
      const bool reads_level = std::find(written.begin(), written.end(), op.g.H) != written.end();
      if (!written.empty() && (reads_level || used + need > P.partial_elems)) {
        ++lv;
        written.clear();
        used = 0;
      }
      if (op.reduce) {
        op.g.out = P.partial + used;
        op.r.part = P.partial + used;
        used += need;
      }
      written.push_back(op.reduce ? static_cast<const void*>(op.r.dst) : op.g.out);
      level[u][k] = lv;
    }
    nlev = std::max(nlev, lv + 1);
  }
  std::vector<BatchedGemm> gl;               // launch order: a level's kinds, then ...
  std::vector<BatchedReduce> rl;             // ... its reduction (one per level)
  std::vector<size_t> level_end;             // gl index where each level's kinds end
  for (int lv = 0; lv < nlev; ++lv) {
    std::vector<GemmArgs> gemms;
    std::vector<ReduceTask> reds;
    for (size_t u = 0; u < ops.size(); ++u)
      for (size_t k = 0; k < ops[u].size(); ++k) {
        if (level[u][k] != lv) continue;
        const BoxOp& op = ops[u][k];
        const int nch = gemm_chunks(op.g, nullptr);
        if (nch == 0) continue;
        gemms.push_back(op.g);
        if (!op.reduce) continue;
        ReduceTask r = op.r;
        r.nchunks = nch;
        reds.push_back(r);
      }
    // one launch per kind of contraction (right / left, operand and output types)
    std::vector<bool> taken(gemms.size(), false);
    for (size_t a = 0; a < gemms.size(); ++a) {
      if (taken[a]) continue;
      std::vector<GemmArgs> kind;
      for (size_t b = a; b < gemms.size(); ++b) {
        const GemmArgs &x = gemms[a], &y = gemms[b];
        if (taken[b] || x.right != y.right || x.th != y.th || x.td != y.td || x.out_f32 != y.out_f32) continue;
        kind.push_back(y);
        taken[b] = true;
      }
      gl.push_back(plan_gemm_batched(kind));
    }
    level_end.push_back(gl.size());
    rl.push_back(plan_reduce_batched(reds));
  }
  // TTNN_PERSISTENT=1: the whole round as one persistent cooperative launch.  Measured
  // slower than one launch per level and kind (a grid barrier's device-scope fences,
  // one a workgroup, write back and invalidate each XCD's L2: ~0.1 ms a barrier), so it
  // is not the default; the results are bitwise the same either way.
  const char* pe = std::getenv("TTNN_PERSISTENT");
  if (pe && pe[0] == '1' && !plans.empty()) {
    std::vector<int*> sticky;
    for (Plan* P : plans)
      if (std::find(sticky.begin(), sticky.end(), P->d_flag + kStickyWord) == sticky.end())
        sticky.push_back(P->d_flag + kStickyWord);
    if (launch_ingest(plans[0]->dtype, gl, level_end, rl, sticky, st)) return;
  }
  constexpr size_t kAlignD = 64;
  auto aligned = [](size_t x) { return (x + kAlignD - 1) / kAlignD * kAlignD; };
  std::vector<size_t> og(gl.size()), of(rl.size()), orr(rl.size());
  size_t total = 0;
  for (size_t k = 0; k < gl.size(); ++k) {
    og[k] = total;
    total = aligned(total + gl[k].tasks.size() * sizeof(GemmTask));
  }
  for (size_t k = 0; k < rl.size(); ++k) {
    of[k] = total;
    total = aligned(total + rl[k].folds.size() * sizeof(ReduceTask));
    orr[k] = total;
    total = aligned(total + rl[k].tasks.size() * sizeof(ReduceTask));
  }
  if (total == 0) return;
  std::vector<char> host(total, 0);
  for (size_t k = 0; k < gl.size(); ++k)
    if (!gl[k].tasks.empty()) std::memcpy(host.data() + og[k], gl[k].tasks.data(), gl[k].tasks.size() * sizeof(GemmTask));
  for (size_t k = 0; k < rl.size(); ++k) {
    if (!rl[k].folds.empty())
      std::memcpy(host.data() + of[k], rl[k].folds.data(), rl[k].folds.size() * sizeof(ReduceTask));
    if (!rl[k].tasks.empty())
      std::memcpy(host.data() + orr[k], rl[k].tasks.data(), rl[k].tasks.size() * sizeof(ReduceTask));
  }
  StagingLock lock;
  char* d = static_cast<char*>(stage_descriptors(host.data(), total, st));
  size_t g0 = 0;
  for (size_t lv = 0; lv < rl.size(); ++lv) {
    for (size_t k = g0; k < level_end[lv]; ++k) launch_gemm_staged(gl[k], reinterpret_cast<const GemmTask*>(d + og[k]), st);
    g0 = level_end[lv];
    launch_reduce_staged(rl[lv], reinterpret_cast<const ReduceTask*>(d + of[lv]),
                         reinterpret_cast<const ReduceTask*>(d + orr[lv]), st);
  }
  fence_descriptors(st);
}

void run_box_ops(Plan& P, const std::vector<BoxOp>& ops, hipStream_t st) {
  run_box_ops_batched({&P}, {&ops}, st);
}

namespace {
void update_box_impl(Plan& P, const void* block, const int64_t* off, const int64_t* ext, const int64_t* strides,
                     double alpha, hipStream_t st) {
  P.epilogue_valid = false;
  // boxes, and any block read in place with strides, take the generic kernels (the
  // one-pass and MFMA right-sketch kernels stream a packed whole tensor)
  if (!whole_box(P, off, ext) || strides) {
    if (P.timing) {
      TTNN_HIP(hipEventRecord(P.sweep_ev[0], st));
      P.sweep_recorded = false;
    }
    std::vector<BoxOp> ops;
    record_box(P, block, off, ext, strides, alpha, ops);
    run_box_ops(P, ops, st);
    return;
  }
  fill_transposed(P, st);                       // the MFMA forms below read them
  std::vector<int> fused_nodes;
  std::vector<std::vector<int>> fused_prefixes;
  if (P.timing) {
    TTNN_HIP(hipEventRecord(P.sweep_ev[0], st));
    P.sweep_recorded = false;
  }
  if (P.allow_fused)
    try_fused_update(P, block, off, ext, alpha, st, &fused_nodes, &fused_prefixes);

  const int cd = P.dtype;                       // dtype of the block and of the DRM copies
  const bool whole = whole_box(P, off, ext);
  std::map<std::vector<int>, bool> done;        // prefixes computed for this update
  for (const auto& pf : fused_prefixes) done[pf] = true;
  Batch batch(P, st);
  // The first contraction of the raw block runs on the generic kernel with the
  // compute-dtype DRMs (on the MFMA right form when the whole tensor is contracted
  // with Y^T of a group at mode 1); every contraction of an FP64 intermediate uses the FP64
  // DRMs (batched MFMA GEMM for whole-tensor updates, generic kernel for boxes).
  auto chain_ptr = [&](const std::vector<int>& pf) { return P.chain + P.prefix_offset.at(pf); };

  auto operand = [&](const std::vector<int>& prefix) -> const void* {
    if (prefix.empty()) return block;
    std::vector<int> chain;
    for (size_t j = 0; j < prefix.size(); ++j) {
      chain.push_back(prefix[j]);
      if (done[chain]) continue;
      std::vector<int> before(chain.begin(), chain.end() - 1);
      const std::vector<Pos> ps = positions_after(P, before, off, ext);
      const Node& g = P.nodes[chain.back()];
      const int p0 = position_of_mode(ps, g.first);
      const int w = g.last - g.first + 1;
      const int64_t L = prod_ext(ps, 0, p0), n = prod_ext(ps, p0, p0 + w), Q = prod_ext(ps, p0 + w, ps.size());
      if (!before.empty() && whole) {
        if (batch.writes(chain_ptr(before))) batch.flush();
        batch.add(left_job(chain_ptr(before), L, n, Q, g.Y64, g.k, 1, g.k, chain_ptr(chain), 0, 1.0));
      } else {
        batch.flush();
        GemmArgs a;
        a.H = before.empty() ? block : static_cast<const void*>(chain_ptr(before));
        a.th = before.empty() ? cd : TTNN_F64;
        a.L = L;
        a.n = n;
        a.Q = Q;
        a.D = before.empty() ? g.Yc : static_cast<const void*>(g.Y64);
        a.td = before.empty() ? cd : TTNN_F64;
        a.sDr = g.k;
        a.sDc = 1;
        a.ncols = g.k;
        a.amap = box_rows(P, g.first, g.last, off, ext);
        join_side(P, st);                       // shares the partial scratch
        if (before.empty() && whole && L == 1 && g.Yt) {
          // raw tensor, group at mode 1: Z[j + k q] = sum_i T[i + n q] Y[i][j] is the
          // MFMA right form with the contraction (i) contiguous and q as the row.  Its
          // one-chunk partial layout is Z's, so when the scratch cannot hold two chunks
          // the kernel writes Z directly (one chunk: the rows alone fill the machine)
          const size_t out = static_cast<size_t>(Q) * static_cast<size_t>(g.k);
          if (!chain_head_in_place(Q, g.k, P.partial_elems)) {
            const int nch = launch_right_mfma(block, cd, n, Q, 1, g.Yt, n, g.k, P.partial, P.partial_elems, st);
            IndexMap none;
            launch_reduce(P.partial, nch, Q, g.k, 2, 1.0, none, 0, chain_ptr(chain), 1, g.k, st);
          } else {
            launch_right_mfma(block, cd, n, Q, 1, g.Yt, n, g.k, chain_ptr(chain), out, st);
          }
        } else if (before.empty() && whole && mid_mfma_eligible(L, n, Q, g.k, cd)) {
          // raw tensor, group past mode 1 (a visiting order that contracts a later
          // group first): the streaming MFMA mode product, written straight to Z
          launch_mid_mfma(block, cd, L, n, Q, g.Yc, g.k, chain_ptr(chain), st);
        } else {
          left_op(P, a, chain_ptr(chain), 2, 1.0, st);
        }
      }
      done[chain] = true;
    }
    return chain_ptr(prefix);
  };

  // root: T x_{c1} Y_c1^T ... x_{cm} Y_cm^T accumulated into Psi_0.  For a whole tensor
  // its last step is an FP64 job that depends only on the chain, so it joins the
  // first batch of node jobs (it runs first; the accumulators are independent).
  auto do_root = [&]() {
    const auto& rc = P.nodes[0].visit;
    std::vector<int> before(rc.begin(), rc.end() - 1);
    const void* in = operand(before);
    const std::vector<Pos> ps = positions_after(P, before, off, ext);
    const Node& g = P.nodes[rc.back()];
    const int p0 = position_of_mode(ps, g.first);
    const int w = g.last - g.first + 1;
    const int64_t L = prod_ext(ps, 0, p0), n = prod_ext(ps, p0, p0 + w), Q = prod_ext(ps, p0 + w, ps.size());
    if (!before.empty() && whole) {
      if (batch.writes(in)) batch.flush();
      batch.add(left_job(static_cast<const double*>(in), L, n, Q, g.Y64, g.k, 1, g.k, P.psi_root, 1, alpha));
      return;
    }
    batch.flush();
    GemmArgs a;
    a.H = in;
    a.th = before.empty() ? cd : TTNN_F64;
    a.L = L;
    a.n = n;
    a.Q = Q;
    a.D = before.empty() ? g.Yc : static_cast<const void*>(g.Y64);
    a.td = before.empty() ? cd : TTNN_F64;
    a.sDr = g.k;
    a.sDc = 1;
    a.ncols = g.k;
    a.amap = box_rows(P, g.first, g.last, off, ext);
    join_side(P, st);
    left_op(P, a, P.psi_root, 1, alpha, st);
  };
  do_root();

  for (size_t v = 1; v < P.nodes.size(); ++v) {
    if (std::find(fused_nodes.begin(), fused_nodes.end(), static_cast<int>(v)) != fused_nodes.end()) continue;
    Node& t = P.nodes[v];
    if (t.ident) continue;                      // a free mode: no sketch of its own
    const std::vector<int>& pre = t.S;          // empty for TTNN
    const void* in = operand(pre);
    const std::vector<Pos> ps = positions_after(P, pre, off, ext);
    const int p0 = position_of_mode(ps, t.first);
    const int w = t.last - t.first + 1;
    const int64_t L = prod_ext(ps, 0, p0), n = prod_ext(ps, p0, p0 + w), Q = prod_ext(ps, p0 + w, ps.size());
    if (!pre.empty() && whole && t.Xt64 && right_mfma_eligible(L, n, Q, t.r, TTNN_F64)) {
      // FP64 intermediate, contraction contiguous: MFMA right form
      batch.flush();
      join_side(P, st);
      const int nch = launch_right_mfma(in, TTNN_F64, L, n, Q, t.Xt64, t.m, t.r, P.partial, P.partial_elems, st);
      launch_reduce(P.partial, nch, n, t.r, 0, alpha, box_rows(P, t.first, t.last, off, ext), t.n, t.R, 1, 1, st);
      continue;
    }
    if (!pre.empty() && whole) {
      if (batch.writes(in)) batch.flush();
      batch.add(right_job(static_cast<const double*>(in), L, n, Q, t.X64, t.r, t.R, alpha));
      continue;
    }
    batch.flush();
    join_side(P, st);
    if (pre.empty() && whole && t.Xt) {          // raw tensor, contiguous contraction: MFMA
      const int nch = launch_right_mfma(block, cd, L, n, Q, t.Xt, t.m, t.r, P.partial, P.partial_elems, st);
      launch_reduce(P.partial, nch, n, t.r, 0, alpha, box_rows(P, t.first, t.last, off, ext), t.n, t.R, 1, 1, st);
      continue;
    }
    // X_t rows: every position except those of t, first fastest
    IndexMap amap, bmap;
    int64_t C = 1;
    for (int i = 0; i < static_cast<int>(ps.size()); ++i) {
      if (i >= p0 && i < p0 + w) continue;
      if (i < p0) amap.push(ps[i].ext, ps[i].off, C);
      else bmap.push(ps[i].ext, ps[i].off, C);
      C *= ps[i].glob;
    }
    GemmArgs a;
    a.right = true;
    a.H = in;
    a.th = pre.empty() ? cd : TTNN_F64;
    a.L = L;
    a.n = n;
    a.Q = Q;
    a.D = pre.empty() ? t.Xc : static_cast<const void*>(t.X64);
    a.td = pre.empty() ? cd : TTNN_F64;
    a.sDr = t.r;
    a.sDc = 1;
    a.ncols = t.r;
    a.amap = amap;
    a.bmap = bmap;
    a.nchunks = pick_chunks(a.n, a.ncols, a.L * a.Q, P.partial_elems);
    a.out = P.partial;
    a.ol = OutLayout{INT64_MAX, a.ncols, 1, 0, a.n * a.ncols};
    const int nch = launch_gemm(a, st);
    if (nch == 0) continue;
    launch_reduce(P.partial, nch, a.n, a.ncols, 0, alpha, box_rows(P, t.first, t.last, off, ext), t.n,
                  t.R, 1, 1, st);
  }

  batch.flush();
  join_side(P, st);
}
}  // namespace

void update_box(Plan& P, const void* block, const int64_t* off, const int64_t* ext, const int64_t* strides,
                double alpha, hipStream_t st) {
  update_box_impl(P, block, off, ext, strides, alpha, st);
  // without a one-pass sweep kernel the whole update counts as the sweep
  if (P.timing && !P.sweep_recorded) {
    TTNN_HIP(hipEventRecord(P.sweep_ev[1], st));
    P.sweep_recorded = true;
  }
}

// ---------------------------------------------------------------- epilogue
// Omega_t = Y_t^T R_t for every non-root node and Psi_t = (Y_cm^T kron ... kron Y_c1^T) R_t
// for internal nodes (child c1 fastest), in FP64 with the FP64 DRMs.  Jobs of one
// chain step are launched together.
void run_epilogue(Plan& P, hipStream_t st) {
  Batch batch(P, st);
  const int nn = static_cast<int>(P.nodes.size());
  // work buffers for the chain steps of every internal node (disjoint slices)
  std::vector<double*> buf(nn, nullptr), buf2(nn, nullptr);
  size_t used = 0;
  size_t maxstep = 1;
  for (int v = 1; v < nn; ++v) maxstep = std::max(maxstep, P.nodes[v].children.size());
  for (int v = 1; v < nn; ++v) {
    Node& t = P.nodes[v];
    if (!t.ident) batch.add(left_job(t.R, 1, t.n, t.r, t.Y64, t.k, 1, t.k, t.Om, 0, 1.0));
  }
  for (size_t step = 0; step < maxstep; ++step) {
    for (int v = 1; v < nn; ++v) {
      Node& t = P.nodes[v];
      if (t.leaf() || step >= t.children.size()) continue;
      // sizes after `step` contractions: k_c (done) then n_c (pending) then r
      std::vector<int64_t> sizes;
      for (size_t i = 0; i < t.children.size(); ++i)
        sizes.push_back(i < step ? P.nodes[t.children[i]].k : P.nodes[t.children[i]].n);
      sizes.push_back(t.r);
      int64_t elems = 1;
      for (int64_t x : sizes) elems *= x;
      const Node& c = P.nodes[t.children[step]];
      const bool last = step + 1 == t.children.size();
      const double* in = step == 0 ? t.R : (step % 2 == 1 ? buf[v] : buf2[v]);
      double* out;
      if (last) out = t.Psi;
      else {
        const size_t need = static_cast<size_t>(elems / c.n * c.k);
        double*& slot = (step % 2 == 0) ? buf[v] : buf2[v];
        if (!slot) {
          slot = P.work + used;
          used += need;
          TTNN_REQUIRE(used <= P.work_elems, TTNN_E_INVALID, "epilogue work buffer too small");
        }
        out = slot;
      }
      batch.add(mode_job(in, sizes, static_cast<int>(step), c.Y64, c.k, 1, c.k, out));
    }
    batch.flush();
  }
  batch.flush();
  P.epilogue_valid = true;
}

std::vector<int64_t> core_shape(const Plan& P, int v) {
  const Node& nd = P.nodes[v];
  std::vector<int64_t> s;
  if (v == 0) {
    for (int c : nd.children) s.push_back(P.nodes[c].r);
    return s;
  }
  if (nd.leaf()) return {nd.n, nd.r};
  for (int c : nd.children) s.push_back(P.nodes[c].r);
  s.push_back(nd.r);
  return s;
}

// ---------------------------------------------------------------- recovery phase

void enqueue_assemble(Plan& P, double* const* cores, hipStream_t st) {
  if (!P.epilogue_valid) run_epilogue(P, st);
  const int nn = static_cast<int>(P.nodes.size());
  // finite check of the sketches
  launch_zero_int(P.d_flag, kCallWord, st);
  {
    SegList s;
    for (int v = 1; v < nn; ++v) {
      const Node& t = P.nodes[v];
      if (t.ident) continue;
      if (P.variant != TTNN_KR) s.push(t.R, t.n * t.r);
      else {                                   // the structured accumulators themselves
        s.push(t.Om, t.k * t.r);
        s.push(t.leaf() ? t.R : t.Psi, (t.leaf() ? t.n : psi_rows(P, v)) * t.r);
      }
    }
    s.push(P.psi_root, P.psi_root_len);
    launch_finite_list(s, P.d_flag, st);
  }

  QrJobList jl{};
  for (int v = 1; v < nn; ++v) {
    const Node& t = P.nodes[v];
    if (t.ident) continue;                      // Q = I, no pseudo-inverse
    jl.jobs[jl.n] = QrJob{t.Om, t.Q, t.Pinv, t.k, t.r, jl.n};
    ++jl.n;
  }
  launch_qr_pinv(jl, P.eps_factor, P.d_flag + 1, st);

  // cores: leaves B = Psi Pinv; internal nodes and root contract Psi with Q_c^T child by
  // child, then (non-root) apply Pinv.
  Batch batch(P, st);
  std::vector<double*> buf(nn, nullptr), buf2(nn, nullptr);
  size_t used = 0;
  size_t maxstep = 0;
  for (int v = 0; v < nn; ++v)
    if (!P.nodes[v].leaf()) maxstep = std::max(maxstep, P.nodes[v].children.size() + (v > 0 ? 1 : 0));
  for (int v = 1; v < nn; ++v)
    if (P.nodes[v].leaf() && !P.nodes[v].ident) {
      const Node& t = P.nodes[v];
      batch.add(mode_job(t.R, {t.n, t.r}, 1, t.Pinv, 1, t.r, t.r, cores[v]));
    }
  for (size_t step = 0; step < maxstep; ++step) {
    for (int v = 0; v < nn; ++v) {
      const Node& t = P.nodes[v];
      if (t.leaf()) continue;
      const size_t m = t.children.size();
      const size_t nsteps = m + (v > 0 ? 1 : 0);
      if (step >= nsteps) continue;
      const double* in = step == 0 ? (v == 0 ? P.psi_root : t.Psi) : (step % 2 == 1 ? buf[v] : buf2[v]);
      const bool last = step + 1 == nsteps;
      std::vector<int64_t> sizes;
      for (size_t i = 0; i < m; ++i) sizes.push_back(i < step ? P.nodes[t.children[i]].r : P.nodes[t.children[i]].k);
      if (v > 0) sizes.push_back(t.r);
      int64_t elems = 1;
      for (int64_t x : sizes) elems *= x;
      double* out;
      if (last) out = cores[v];
      else {
        const Node& c = P.nodes[t.children[step]];
        const size_t need = static_cast<size_t>(elems / c.k * c.r);
        double*& slot = (step % 2 == 0) ? buf[v] : buf2[v];
        if (!slot) {
          slot = P.work + used;
          used += need;
          TTNN_REQUIRE(used <= P.work_elems, TTNN_E_INVALID, "assembly work buffer too small");
        }
        out = slot;
      }
      if (step < m) {
        const Node& c = P.nodes[t.children[step]];
        batch.add(mode_job(in, sizes, static_cast<int>(step), c.Q, 1, c.k, c.r, out));   // Q_c^T
      } else {
        int64_t rows = elems / t.r;
        batch.add(mode_job(in, {rows, t.r}, 1, t.Pinv, 1, t.r, t.r, out));
      }
    }
    batch.flush();
  }
  batch.flush();
  launch_status_fold(P.d_flag, jl.n + 1, P.d_flag + kCallWord, P.d_flag + kStickyWord, st);
  P.has_cores = true;
}

ttnn_status run_assemble(Plan& P, double* const* cores, hipStream_t st) {
  enqueue_assemble(P, cores, st);
  int bad = 0;
  TTNN_HIP(hipMemcpyAsync(&bad, P.d_flag + kCallWord, sizeof(int), hipMemcpyDeviceToHost, st));
  TTNN_HIP(hipStreamSynchronize(st));
  return bad ? TTNN_E_NUMERIC : TTNN_OK;
}

void assemble_status_async(Plan& P, int32_t* h_status, hipStream_t st) {
  TTNN_HIP(hipMemcpyAsync(h_status, P.d_flag + kStickyWord, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  launch_zero_int(P.d_flag + kStickyWord, 1, st);
}

ttnn_status assemble_status(Plan& P, hipStream_t st) {
  int bad = 0;
  TTNN_HIP(hipMemcpyAsync(&bad, P.d_flag + kStickyWord, sizeof(int), hipMemcpyDeviceToHost, st));
  TTNN_HIP(hipStreamSynchronize(st));
  launch_zero_int(P.d_flag + kStickyWord, 1, st);
  return bad ? TTNN_E_NUMERIC : TTNN_OK;
}

// ---------------------------------------------------------------- reconstruction
// U_leaf = B_leaf, U_t = (U_cm kron ... kron U_c1) B_t, vec(T_hat) = (U_cm kron ... kron U_c1) B_0,
// deepest nodes first; the final contraction writes the caller's buffer.
void run_reconstruct(Plan& P, const double* const* cores, void* out, int out_dtype, hipStream_t st) {
  const int nn = static_cast<int>(P.nodes.size());
  std::vector<const double*> U(nn, nullptr);
  size_t inter = 0;
  for (int v = 1; v < nn; ++v)
    if (!P.nodes[v].leaf()) inter += static_cast<size_t>(P.nodes[v].n * P.nodes[v].r);
  double* ustore = P.work;
  double* bufs[2] = {P.work + inter, P.work + inter + (P.work_elems - inter) / 2};
  size_t used = 0;
  int maxlevel = 0;
  for (const Node& t : P.nodes) maxlevel = std::max(maxlevel, t.level);
  for (int v = 1; v < nn; ++v)
    if (P.nodes[v].leaf()) U[v] = P.nodes[v].ident ? P.nodes[v].Q : cores[v];   // free mode: U = I
  Batch batch(P, st);
  for (int lev = maxlevel; lev >= 0; --lev) {
    for (int v = nn - 1; v >= 0; --v) {
      const Node& t = P.nodes[v];
      if (t.level != lev || t.leaf()) continue;
      std::vector<int64_t> sizes;
      for (int c : t.children) sizes.push_back(P.nodes[c].r);
      if (v > 0) sizes.push_back(t.r);
      const double* cur = cores[v];
      const size_t m = t.children.size();
      double* dest = nullptr;
      if (v > 0) {
        dest = ustore + used;
        used += static_cast<size_t>(t.n * t.r);
      }
      for (size_t i = 0; i < m; ++i) {
        const Node& c = P.nodes[t.children[i]];
        const bool last = i + 1 == m;
        if (last && v == 0) {
          batch.flush();
          // final step writes the dense tensor (dtype of the caller's buffer) directly
          GemmArgs g;
          g.right = false;
          g.H = cur;
          g.th = TTNN_F64;
          g.L = 1;
          for (size_t j = 0; j < i; ++j) g.L *= sizes[j];
          g.n = sizes[i];
          g.Q = 1;
          g.D = U[t.children[i]];
          g.td = TTNN_F64;
          g.sDr = c.n;
          g.sDc = 1;
          g.ncols = static_cast<int>(c.n);
          IndexMap id;
          id.push(g.n, 0, 1);
          g.amap = id;
          g.nchunks = 1;
          g.out = out;
          g.out_f32 = out_dtype == TTNN_F32;
          g.ol = OutLayout{g.L, 1, g.L, g.L * g.ncols, 0};
          if (out_dtype == TTNN_F64) {
            std::vector<GJob> one{mode_job(cur, sizes, static_cast<int>(i), U[t.children[i]], c.n, 1, c.n,
                                           static_cast<double*>(out))};
            launch_bgemm64(one, P.g64_part, P.g64_part_elems, st);
          } else {
            launch_gemm(g, st);
          }
          break;
        }
        double* o = last ? dest : bufs[i % 2];
        // contract position i (size r_c) with U_c^T: M(i', j) = U_c[j + n_c i']
        std::vector<GJob> one{mode_job(cur, sizes, static_cast<int>(i), U[t.children[i]], c.n, 1, c.n, o)};
        launch_bgemm64(one, P.g64_part, P.g64_part_elems, st);
        sizes[i] = c.n;
        cur = o;
      }
      if (v > 0) U[v] = dest;
    }
  }
  batch.flush();
}

// Rank-1 update H = a_1 o ... o a_d (Sec. 4, streaming by linearity).  With u_I the
// Kronecker vector of the factors of a mode group (first mode fastest):
//   R_t += alpha * u_{I_t} (X_t^T v_t)^T,   v_t = kron over the rows of X_t,
// where the rows run over the modes outside I_t (TTNN) or over the indices of T_{S_t}
// outside I_t in mode order, a contracted group s contributing g_s = Y_s^T u_{I_s} and
// any other mode its factor (STTNN); and
//   Psi_0 += alpha * kron_c g_c over the root's children.
// The maps are the ones a box update uses: the compute-dtype copy for a contraction
// of the raw tensor (a chain's first group, or X_t when S_t is empty), the FP64
// master for a contraction of an FP64 intermediate; products and sums are FP64.
// Reads every row of every X_t once.
void update_rank1(Plan& P, int nterms, const double* const* factors, const double* alphas, hipStream_t st) {
  P.epilogue_valid = false;
  const int cd = P.dtype;
  const int d = P.d;
  // the terms in batches of kRank1Batch: a batch reads each map about once; every
  // term's arithmetic is that of a batch of one, so the result does not depend on the
  // batching
  for (int t0 = 0; t0 < nterms; t0 += kRank1Batch) {
    const int m = std::min(kRank1Batch, nterms - t0);
    const double* const* f = factors + static_cast<size_t>(t0) * d;
    auto modes = [&](int y, int first, int last) {
      KronVec kv;
      for (int mu = first; mu <= last; ++mu) kv.push(f[y * d + mu], P.dims[mu]);
      return kv;
    };
    // g_s = Y_s^T u_{I_s} per term, at P.r1 + y * r1_w + goff[s]; a group is contracted
    // from the raw tensor exactly when it heads its chains, that is when its own reuse
    // set is empty (free modes: identity maps, exact in any dtype)
    std::vector<int64_t> goff(P.nodes.size(), -1);
    int64_t used = 0;
    auto g_of = [&](int s) {
      if (goff[s] < 0) {
        const Node& g = P.nodes[s];
        goff[s] = used;
        used += g.k;
        const bool raw = g.S.empty();
        KronBatch kb;
        for (int y = 0; y < m; ++y) kb.push(modes(y, g.first, g.last));
        launch_kron_gemv(raw ? g.Yc : static_cast<const void*>(g.Y64), raw ? cd : TTNN_F64, g.n, g.k, kb, P.partial,
                         P.partial_elems, P.r1 + goff[s], P.r1_w, P.rank1_form == TTNN_R1_GROUPED, st);
      }
      return goff[s];
    };
    double* w = P.r1 + static_cast<int64_t>(kRank1Batch) * P.r1_w;     // m x rmax
    const int64_t wstride = P.r1_rmax;
    for (size_t v = 1; v < P.nodes.size(); ++v) {
      const Node& t = P.nodes[v];
      if (t.ident) continue;                    // a free mode: no sketch of its own
      KronBatch kx, ku;
      for (int y = 0; y < m; ++y) {
        KronVec k;
        if (P.variant == TTNN_STTNN) {
          // the rows of X_t: the indices of T_{S_t} outside I_t in mode order
          std::vector<int> group_of(d, -1);
          for (int s : t.S)
            for (int mu = P.nodes[s].first; mu <= P.nodes[s].last; ++mu) group_of[mu] = s;
          for (int mu = 0; mu < d; ++mu) {
            if (mu >= t.first && mu <= t.last) continue;
            const int s = group_of[mu];
            if (s < 0) k.push(f[y * d + mu], P.dims[mu]);
            else if (mu == P.nodes[s].first) k.push(P.r1 + y * P.r1_w + g_of(s), P.nodes[s].k);
          }
        } else {
          for (int mu = 0; mu < d; ++mu)
            if (mu < t.first || mu > t.last) k.push(f[y * d + mu], P.dims[mu]);
        }
        kx.push(k);
        ku.push(modes(y, t.first, t.last), alphas[t0 + y]);
      }
      const bool raw = t.S.empty();
      launch_kron_gemv(raw ? t.Xc : static_cast<const void*>(t.X64), raw ? cd : TTNN_F64, t.m, t.r, kx, P.partial,
                       P.partial_elems, w, wstride, P.rank1_form == TTNN_R1_GROUPED, st);
      launch_outer_acc(t.R, t.n, t.r, ku, w, wstride, st);
    }
    KronBatch kg;
    for (int y = 0; y < m; ++y) {
      KronVec k;
      for (int c : P.nodes[0].children) k.push(P.r1 + y * P.r1_w + g_of(c), P.nodes[c].k);
      kg.push(k, alphas[t0 + y]);
    }
    launch_outer_acc(P.psi_root, P.psi_root_len, 1, kg, nullptr, 0, st);
  }
}

}  // namespace ttnn
