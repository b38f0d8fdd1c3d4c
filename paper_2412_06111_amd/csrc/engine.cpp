// Drivers of the sketch phase (Sec. 4 and 5), the FP64 epilogue that forms the
// "left" and "intersection" sketches from the accumulated right sketches, the
// recovery phase (Sec. 4, Alg. 2) and the reconstruction (Def. 5, matricised form).
//
// State kept per plan (all FP64, linear in the tensor, Sec. 4 streaming paragraph):
//   R_t for every non-root node t   (TTNN: T^{t} X_t;  STTNN: (T_{S_t})^{t} X_t)
//   Psi_0 at the root               (T contracted with Y_c^T over every child c)
// Omega_t = Y_t^T R_t and Psi_t = (kron_c Y_c^T) R_t are formed on demand.
#include <algorithm>
#include <map>

#include "engine.hpp"
#include "fused.hpp"
#include "kernels.hpp"

namespace ttnn {
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

// positions of the operand obtained from the box after contracting `prefix`
std::vector<Pos> positions_after(const Plan& P, const std::vector<int>& prefix, const int64_t* off,
                                 const int64_t* ext) {
  std::vector<Pos> ps;
  int next_mode = 0;
  for (int s : prefix) {
    const Node& g = P.nodes[s];
    ps.push_back(Pos{g.k, 0, g.k, g.first, true});
    next_mode = g.last + 1;
  }
  for (int mu = next_mode; mu < P.d; ++mu) ps.push_back(Pos{ext[mu], off[mu], P.dims[mu], mu, false});
  return ps;
}

int position_of_mode(const std::vector<Pos>& ps, int mode) {
  for (size_t i = 0; i < ps.size(); ++i)
    if (!ps[i].contracted && ps[i].mode_first == mode) return static_cast<int>(i);
  return -1;
}

// Store (or accumulate) a LEFT contraction, splitting the contraction when the
// output is small.  mode: 2 = store, 1 = accumulate alpha * result.
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

// FP64 dense mode product on an operand with positions `sizes` (first fastest):
// contract position p with M (rows = sizes[p]; M(i, j) at M[i*sMi + j*sMj]), j < ncols.
void mode_product(Plan& P, const double* in, const std::vector<int64_t>& sizes, int p, const double* M,
                  int64_t sMi, int64_t sMj, int ncols, double* out, hipStream_t st) {
  GemmArgs g;
  g.H = in;
  g.th = TTNN_F64;
  g.L = 1;
  for (int i = 0; i < p; ++i) g.L *= sizes[i];
  g.n = sizes[p];
  g.Q = 1;
  for (size_t i = p + 1; i < sizes.size(); ++i) g.Q *= sizes[i];
  g.D = M;
  g.td = TTNN_F64;
  g.sDr = sMi;
  g.sDc = sMj;
  g.ncols = ncols;
  IndexMap id;
  id.push(g.n, 0, 1);
  g.amap = id;
  left_op(P, g, out, 2, 1.0, st);
}

}  // namespace

// ---------------------------------------------------------------- sizing
void size_chain_scratch(Plan& P) {
  std::vector<std::vector<int>> prefixes;
  auto add_prefixes = [&](const std::vector<int>& chain, size_t upto) {
    for (size_t j = 1; j <= upto && j <= chain.size(); ++j)
      prefixes.emplace_back(chain.begin(), chain.begin() + j);
  };
  for (size_t v = 1; v < P.nodes.size(); ++v) add_prefixes(P.nodes[v].S, P.nodes[v].S.size());
  const auto& rc = P.nodes[0].children;
  add_prefixes(rc, rc.size() - 1);      // the last root step accumulates into Psi_0
  size_t total = 0;
  for (auto& pf : prefixes) {
    if (P.prefix_offset.count(pf)) continue;
    int64_t e = 1;
    for (int s : pf) e *= P.nodes[s].k;
    for (int mu = P.nodes[pf.back()].last + 1; mu < P.d; ++mu) e *= P.dims[mu];
    P.prefix_offset[pf] = total;
    total += static_cast<size_t>(e);
  }
  P.chain_elems = std::max<size_t>(total, 1);

  size_t part = size_t(1) << 22;
  size_t work = 1, ustore = 0, inter = 1;
  for (size_t v = 1; v < P.nodes.size(); ++v) {
    const Node& nd = P.nodes[v];
    part = std::max(part, static_cast<size_t>(nd.n * nd.r));
    part = std::max(part, static_cast<size_t>(nd.k * nd.r));
  }
  for (size_t v = 0; v < P.nodes.size(); ++v) {
    const Node& nd = P.nodes[v];
    if (nd.leaf()) continue;
    const int64_t rt = v == 0 ? 1 : nd.r;
    // epilogue / cores: prod_{<=i} k * prod_{>i} n * r  and  prod_{<=i} r_c * prod_{>i} k * r
    for (size_t i = 0; i < nd.children.size(); ++i) {
      int64_t a = rt, b = rt, c = rt;
      for (size_t j = 0; j < nd.children.size(); ++j) {
        const Node& ch = P.nodes[nd.children[j]];
        a *= j <= i ? ch.k : ch.n;
        b *= j <= i ? ch.r : ch.k;
        c *= j <= i ? ch.n : ch.r;     // reconstruction
      }
      inter = std::max<size_t>(inter, std::max<int64_t>(a, b));
      if (v != 0 || i + 1 < nd.children.size()) inter = std::max<size_t>(inter, c);
    }
    if (v != 0) ustore += static_cast<size_t>(nd.n * nd.r);
  }
  work = 2 * inter + ustore;
  part = std::max(part, static_cast<size_t>(P.psi_root_len));
  P.partial_elems = part;
  P.work_elems = work;
}

void zero_accumulators(Plan& P, hipStream_t st) {
  for (size_t v = 1; v < P.nodes.size(); ++v) launch_zero(P.nodes[v].R, P.nodes[v].n * P.nodes[v].r, st);
  launch_zero(P.psi_root, P.psi_root_len, st);
  P.epilogue_valid = false;
}

// ---------------------------------------------------------------- sketch phase
void update_box(Plan& P, const void* block, const int64_t* off, const int64_t* ext, double alpha,
                hipStream_t st) {
  P.epilogue_valid = false;
  std::vector<int> fused_nodes;
  std::vector<std::vector<int>> fused_prefixes;
  if (P.allow_fused)
    try_fused_update(P, block, off, ext, alpha, st, &fused_nodes, &fused_prefixes);

  const int cd = P.dtype;                       // dtype of the block and of the DRM copies
  std::map<std::vector<int>, bool> done;        // prefixes computed for this update
  for (const auto& pf : fused_prefixes) done[pf] = true;

  // returns the operand after contracting `prefix` (FP64 intermediate, or the block)
  auto operand = [&](const std::vector<int>& prefix, int& th) -> const void* {
    if (prefix.empty()) {
      th = cd;
      return block;
    }
    th = TTNN_F64;
    double* dst = P.chain + P.prefix_offset.at(prefix);
    if (done[prefix]) return dst;
    std::vector<int> chain;
    for (size_t j = 0; j < prefix.size(); ++j) {
      chain.push_back(prefix[j]);
      double* out = P.chain + P.prefix_offset.at(chain);
      if (done[chain]) continue;
      std::vector<int> before(chain.begin(), chain.end() - 1);
      int thin = cd;
      const void* in = before.empty() ? block : static_cast<const void*>(P.chain + P.prefix_offset.at(before));
      if (!before.empty()) thin = TTNN_F64;
      const std::vector<Pos> ps = positions_after(P, before, off, ext);
      const Node& g = P.nodes[chain.back()];
      const int p0 = position_of_mode(ps, g.first);
      const int w = g.last - g.first + 1;
      GemmArgs a;
      a.H = in;
      a.th = thin;
      a.L = prod_ext(ps, 0, p0);
      a.n = prod_ext(ps, p0, p0 + w);
      a.Q = prod_ext(ps, p0 + w, ps.size());
      a.D = g.Yc;
      a.td = cd;
      a.sDr = g.k;
      a.sDc = 1;
      a.ncols = g.k;
      a.amap = box_rows(P, g.first, g.last, off, ext);
      left_op(P, a, out, 2, 1.0, st);
      done[chain] = true;
    }
    return dst;
  };

  for (size_t v = 1; v < P.nodes.size(); ++v) {
    if (std::find(fused_nodes.begin(), fused_nodes.end(), static_cast<int>(v)) != fused_nodes.end()) continue;
    Node& t = P.nodes[v];
    const std::vector<int>& pre = t.S;          // empty for TTNN
    int th = cd;
    const void* in = operand(pre, th);
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
    GemmArgs a;
    a.right = true;
    a.H = in;
    a.th = th;
    a.L = prod_ext(ps, 0, p0);
    a.n = prod_ext(ps, p0, p0 + w);
    a.Q = prod_ext(ps, p0 + w, ps.size());
    a.D = t.Xc;
    a.td = cd;
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

  // root: T x_{c1} Y_c1^T ... x_{cm} Y_cm^T accumulated into Psi_0
  const auto& rc = P.nodes[0].children;
  std::vector<int> before(rc.begin(), rc.end() - 1);
  int th = cd;
  const void* in = operand(before, th);
  const std::vector<Pos> ps = positions_after(P, before, off, ext);
  const Node& g = P.nodes[rc.back()];
  const int p0 = position_of_mode(ps, g.first);
  const int w = g.last - g.first + 1;
  GemmArgs a;
  a.H = in;
  a.th = th;
  a.L = prod_ext(ps, 0, p0);
  a.n = prod_ext(ps, p0, p0 + w);
  a.Q = prod_ext(ps, p0 + w, ps.size());
  a.D = g.Yc;
  a.td = cd;
  a.sDr = g.k;
  a.sDc = 1;
  a.ncols = g.k;
  a.amap = box_rows(P, g.first, g.last, off, ext);
  left_op(P, a, P.psi_root, 1, alpha, st);
}

// ---------------------------------------------------------------- epilogue
void run_epilogue(Plan& P, hipStream_t st) {
  for (size_t v = 1; v < P.nodes.size(); ++v) {
    Node& t = P.nodes[v];
    // Omega_t = Y_t^T R_t  (R_t viewed as [1][n_t][r_t])
    mode_product(P, t.R, {t.n, t.r}, 0, t.Y64, t.k, 1, t.k, t.Om, st);
    if (t.leaf()) continue;
    // Psi_t = (Y_cm^T kron ... kron Y_c1^T) R_t
    std::vector<int64_t> sizes;
    for (int c : t.children) sizes.push_back(P.nodes[c].n);
    sizes.push_back(t.r);
    const double* cur = t.R;
    double* bufs[2] = {P.work, P.work + (P.work_elems / 2)};
    for (size_t i = 0; i < t.children.size(); ++i) {
      const Node& c = P.nodes[t.children[i]];
      double* out = (i + 1 == t.children.size()) ? t.Psi : bufs[i % 2];
      mode_product(P, cur, sizes, static_cast<int>(i), c.Y64, c.k, 1, c.k, out, st);
      sizes[i] = c.k;
      cur = out;
    }
  }
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
ttnn_status run_assemble(Plan& P, double* const* cores, hipStream_t st) {
  if (!P.epilogue_valid) run_epilogue(P, st);
  const int nn = static_cast<int>(P.nodes.size());
  // finite check of the sketches
  TTNN_HIP(hipMemsetAsync(P.d_flag, 0, sizeof(int) * 2 * TTNN_MAX_NODES, st));
  for (int v = 1; v < nn; ++v) launch_finite_check(P.nodes[v].R, P.nodes[v].n * P.nodes[v].r, P.d_flag, st);
  launch_finite_check(P.psi_root, P.psi_root_len, P.d_flag, st);

  std::vector<QrJob>& jobs = P.host_jobs;
  jobs.clear();
  int max_k = 1, max_r = 1;
  for (int v = 1; v < nn; ++v) {
    const Node& t = P.nodes[v];
    jobs.push_back(QrJob{t.Om, t.Q, t.Pinv, t.k, t.r});
    max_k = std::max(max_k, t.k);
    max_r = std::max(max_r, t.r);
  }
  TTNN_REQUIRE(static_cast<size_t>(max_k * max_r + 2 * max_r * max_r) * 8 <= 160 * 1024, TTNN_E_INVALID,
               "ranks too large for the in-LDS recovery kernel");
  TTNN_HIP(hipMemcpyAsync(P.d_jobs, jobs.data(), sizeof(QrJob) * jobs.size(), hipMemcpyHostToDevice, st));
  int* d_kept = P.d_flag + 1;
  launch_qr_pinv(P.d_jobs, static_cast<int>(jobs.size()), max_k, max_r, P.eps_factor, d_kept, st);

  // cores
  double* bufs[2] = {P.work, P.work + (P.work_elems / 2)};
  for (int v = 0; v < nn; ++v) {
    const Node& t = P.nodes[v];
    if (v > 0 && t.leaf()) {
      // B_t = Psi_t Pinv_t  (Psi_t = R_t, n_t x r_t; Pinv col-major r x r)
      mode_product(P, t.R, {t.n, t.r}, 1, t.Pinv, 1, t.r, t.r, cores[v], st);
      continue;
    }
    std::vector<int64_t> sizes;
    for (int c : t.children) sizes.push_back(P.nodes[c].k);
    if (v > 0) sizes.push_back(t.r);
    const double* cur = v == 0 ? P.psi_root : t.Psi;
    const size_t m = t.children.size();
    for (size_t i = 0; i < m; ++i) {
      const Node& c = P.nodes[t.children[i]];
      const bool last = (i + 1 == m) && v == 0;
      double* out = last ? cores[v] : bufs[i % 2];
      mode_product(P, cur, sizes, static_cast<int>(i), c.Q, 1, c.k, c.r, out, st);   // Q_c^T
      sizes[i] = c.r;
      cur = out;
    }
    if (v > 0) {
      int64_t rows = 1;
      for (size_t i = 0; i < m; ++i) rows *= sizes[i];
      mode_product(P, cur, {rows, t.r}, 1, t.Pinv, 1, t.r, t.r, cores[v], st);
    }
  }
  // status: flag[0] = non-finite, kept counts of each job
  std::vector<int> host(nn, 0);
  TTNN_HIP(hipMemcpyAsync(host.data(), P.d_flag, sizeof(int) * nn, hipMemcpyDeviceToHost, st));
  TTNN_HIP(hipStreamSynchronize(st));
  P.has_cores = true;
  if (host[0] != 0) return TTNN_E_NUMERIC;
  for (int v = 1; v < nn; ++v)
    if (host[v] == 0) return TTNN_E_NUMERIC;
  return TTNN_OK;
}

// ---------------------------------------------------------------- reconstruction
void run_reconstruct(Plan& P, const double* const* cores, void* out, int out_dtype, hipStream_t st) {
  const int nn = static_cast<int>(P.nodes.size());
  // U_t for internal non-root nodes, children before parents
  std::vector<const double*> U(nn, nullptr);
  double* ustore = P.work;
  size_t inter = 0;
  for (int v = 1; v < nn; ++v)
    if (!P.nodes[v].leaf()) inter += static_cast<size_t>(P.nodes[v].n * P.nodes[v].r);
  double* bufs[2] = {P.work + inter, P.work + inter + (P.work_elems - inter) / 2};
  size_t used = 0;
  for (int v = nn - 1; v >= 0; --v) {
    const Node& t = P.nodes[v];
    if (v > 0 && t.leaf()) {
      U[v] = cores[v];
      continue;
    }
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
        launch_gemm(g, st);
        break;
      }
      double* o = last ? dest : bufs[i % 2];
      // contract position i (size r_c) with U_c^T: M(i', j) = U_c[j + n_c i']
      mode_product(P, cur, sizes, static_cast<int>(i), U[t.children[i]], c.n, 1, static_cast<int>(c.n), o, st);
      sizes[i] = c.n;
      cur = o;
    }
    if (v > 0) U[v] = dest;
  }
}

void update_rank1(Plan& P, const double* const* factors, double alpha, hipStream_t st) {
  // H = a_1 o ... o a_d is materialised in FP64 in the chain scratch only when it
  // fits; otherwise the update is rejected by the caller.  Rank-1 terms arrive as
  // dense blocks through the same path as box updates.
  (void)P;
  (void)factors;
  (void)alpha;
  (void)st;
  throw Error{TTNN_E_INVALID, "rank-1 updates are not available in this build"};
}

}  // namespace ttnn
