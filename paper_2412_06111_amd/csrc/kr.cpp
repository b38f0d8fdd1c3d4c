// Host driver of the Khatri-Rao structured sketch of a TTN-format tensor (Sec. 7) and
// of TTN inner products.
//
// With per-mode factors X_mu (n_mu x r) and Y_mu (n_mu x k), the maps of node t are
// X_t = khatri-rao of X_mu over the modes outside I_t and Y_t = khatri-rao of Y_mu over
// I_t (column j of each is the Kronecker product of the factors' columns j).  For a
// tensor given by TTN cores B_t (Def. 5) the sketches of Sec. 4 then factor over the
// tree, which is how the two entry-wise contractions pictured for Omega and Psi in
// Sec. 7 are evaluated, at a cost linear in the n_mu and without forming the tensor:
//   down vectors  dx_t, dy_t (s_t x r, s_t x k): the subtree of t contracted with the
//                 X (Y) columns j of its modes -- leaves U_t^T X_t, internal nodes B_t
//                 contracted with the children's vectors sharing j;
//   up vectors    u_t (s_t x r): everything outside the subtree of t contracted with the
//                 X columns j -- the parent's core contracted with the siblings' dx and
//                 the parent's u (no u above the root);
//   Omega_t  += alpha dy_t^T u_t,
//   Psi_t    += alpha B_t x_{c} dy_c^T x_t u_t^T   (internal; each child its own column),
//   R_t = Psi_t += alpha U_t u_t                    (leaves),
//   Psi_0    += alpha B_0 x_{c} dy_c^T              (root).
// The shared-column contractions run on the tree-contraction kernel, the mode products
// on the batched FP64 GEMM; everything is FP64.
#include <algorithm>

#include "engine.hpp"
#include "kernels.hpp"
#include "kr.hpp"
#include "plan.hpp"

namespace ttnn {

namespace {

// Bump allocation over the caller's scratch; with no base it only sizes.
struct Bump {
  char* base = nullptr;
  size_t used = 0;
  double* take(size_t elems) {
    const size_t b = (std::max<size_t>(elems, 1) * sizeof(double) + 255) & ~static_cast<size_t>(255);
    double* p = base ? reinterpret_cast<double*>(base + used) : nullptr;
    used += b;
    return p;
  }
};

int max_level(const Plan& P) {
  int m = 0;
  for (const Node& t : P.nodes) m = std::max(m, t.level);
  return m;
}

int64_t prod(const std::vector<int64_t>& v, size_t a, size_t b) {
  int64_t p = 1;
  for (size_t i = a; i < b; ++i) p *= v[i];
  return p;
}

// Axis sizes of node v's core in a TTN of ranks s: a leaf split into its modes (so that
// the per-mode factors apply axis by axis) or kept as (n_t, s_t); internal (s_c.., s_t);
// root (s_c..).
std::vector<int64_t> axes_of(const Plan& P, int v, const std::vector<int64_t>& s, bool split_leaf) {
  const Node& t = P.nodes[v];
  std::vector<int64_t> a;
  if (t.leaf()) {
    if (split_leaf)
      for (int mu = t.first; mu <= t.last; ++mu) a.push_back(P.dims[mu]);
    else
      a.push_back(t.n);
    a.push_back(s[v]);
    return a;
  }
  for (int c : t.children) a.push_back(s[c]);
  if (v > 0) a.push_back(s[v]);
  return a;
}

KJob contraction(const double* core, const std::vector<int64_t>& axes, int oax, int cols, double* out, Bump& bump) {
  KJob j;
  j.core = core;
  j.naxes = static_cast<int32_t>(axes.size());
  j.oax = oax;
  j.cols = cols;
  j.out = out;
  int64_t kred = 1, n0 = 0;
  for (size_t q = 0; q < axes.size(); ++q) {
    j.size[q] = axes[q];
    if (static_cast<int>(q) == oax) continue;
    if (n0 == 0) n0 = axes[q];                         // the kernel's inner axis: first non-output axis
    kred *= axes[q];
  }
  if (n0 == 0) n0 = 1;
  j.G = kr_split(axes[oax], cols, n0, kred / n0);
  if (j.G > 1) j.part = bump.take(kr_part_elems(j));
  return j;
}

void check_ranks(const Plan& P, const std::vector<int64_t>& s) {
  for (size_t v = 1; v < P.nodes.size(); ++v)
    TTNN_REQUIRE(s[v] >= 1 && s[v] <= 4096, TTNN_E_INVALID, "TTN ranks must be in [1, 4096]");
  for (size_t v = 0; v < P.nodes.size(); ++v) {       // core sizes stay far from overflow
    double e = 1.0;
    for (int64_t x : axes_of(P, static_cast<int>(v), s, false)) e *= static_cast<double>(x);
    TTNN_REQUIRE(e < 0x1p40, TTNN_E_INVALID, "TTN core too large");
  }
}

// The structured update; with run == false only the scratch is sized (bump.base null).
void kr_update(Plan& P, const double* const* cores, const std::vector<int64_t>& s, double alpha, Bump& bump,
               bool run, hipStream_t st) {
  const int nn = static_cast<int>(P.nodes.size());
  const int r = P.nodes[1].r, k = P.nodes[1].k;
  std::vector<double*> dx(nn), dy(nn), u(nn);
  for (int v = 1; v < nn; ++v) {
    dx[v] = bump.take(static_cast<size_t>(s[v]) * r);
    dy[v] = bump.take(static_cast<size_t>(s[v]) * k);
    u[v] = bump.take(static_cast<size_t>(s[v]) * r);
  }
  const int maxlev = max_level(P);
  // down vectors, deepest level first
  for (int lev = maxlev; lev >= 1; --lev) {
    std::vector<KJob> jobs;
    for (int v = 1; v < nn; ++v) {
      const Node& t = P.nodes[v];
      if (t.level != lev) continue;
      const auto ax = axes_of(P, v, s, true);
      const int oax = static_cast<int>(ax.size()) - 1;
      KJob jx = contraction(cores[v], ax, oax, r, dx[v], bump);
      KJob jy = contraction(cores[v], ax, oax, k, dy[v], bump);
      for (int q = 0; q < oax; ++q) {
        if (t.leaf()) {
          jx.fac[q] = P.kr_x[t.first + q];
          jy.fac[q] = P.kr_y[t.first + q];
        } else {
          jx.fac[q] = dx[t.children[q]];
          jy.fac[q] = dy[t.children[q]];
        }
      }
      jobs.push_back(jx);
      jobs.push_back(jy);
    }
    if (run) launch_kr_contract(jobs, st);
  }
  // up vectors, root first
  for (int lev = 0; lev < maxlev; ++lev) {
    std::vector<KJob> jobs;
    for (int v = 0; v < nn; ++v) {
      const Node& t = P.nodes[v];
      if (t.level != lev || t.leaf()) continue;
      const auto ax = axes_of(P, v, s, true);
      const int m = static_cast<int>(t.children.size());
      for (int q = 0; q < m; ++q) {
        KJob j = contraction(cores[v], ax, q, r, u[t.children[q]], bump);
        for (int q2 = 0; q2 < m; ++q2)
          if (q2 != q) j.fac[q2] = dx[t.children[q2]];
        if (v > 0) j.fac[m] = u[v];
        jobs.push_back(j);
      }
    }
    if (run) launch_kr_contract(jobs, st);
  }
  // Omega_t, leaf R_t and the Psi chains on the batched FP64 GEMM
  struct Chain {
    int v;
    std::vector<int64_t> sizes;
    const double* cur;
    double* buf[2];
    int step, nsteps;
  };
  std::vector<Chain> chains;
  std::vector<GJob> first;
  for (int v = 1; v < nn; ++v) {
    const Node& t = P.nodes[v];
    GJob o;
    o.M = k;
    o.N = r;
    o.K = s[v];
    o.A = dy[v];
    o.sAm = 1;
    o.sAk = k;
    o.B = u[v];
    o.sBk = r;
    o.sBn = 1;
    o.C = t.Om;
    o.sCm = 1;
    o.sCn = k;
    o.alpha = alpha;
    o.accumulate = 1;
    first.push_back(o);
    if (t.leaf()) first.push_back(left_job(cores[v], t.n, s[v], 1, u[v], r, 1, r, t.R, 1, alpha));
  }
  for (int v = 0; v < nn; ++v) {
    const Node& t = P.nodes[v];
    if (t.leaf()) continue;
    Chain c{v, axes_of(P, v, s, false), cores[v], {nullptr, nullptr}, 0,
            static_cast<int>(t.children.size()) + (v > 0 ? 1 : 0)};
    // largest intermediate before the last step
    int64_t big = 1;
    std::vector<int64_t> sz = c.sizes;
    for (int step = 0; step + 1 < c.nsteps; ++step) {
      if (v > 0 && step == 0) sz.back() = r;
      else sz[v > 0 ? step - 1 : step] = k;
      big = std::max(big, prod(sz, 0, sz.size()));
    }
    if (c.nsteps > 1) {
      c.buf[0] = bump.take(static_cast<size_t>(big));
      c.buf[1] = c.nsteps > 2 ? bump.take(static_cast<size_t>(big)) : nullptr;
    }
    chains.push_back(c);
  }
  const int maxsteps = 1 + static_cast<int>(TTNN_MAX_NODES);
  for (int step = 0; step < maxsteps; ++step) {
    std::vector<GJob> jobs;
    if (step == 0) jobs = first;
    for (Chain& c : chains) {
      if (step >= c.nsteps) continue;
      const Node& t = P.nodes[c.v];
      const bool last = step + 1 == c.nsteps;
      double* out = last ? (c.v == 0 ? P.psi_root : t.Psi) : c.buf[step % 2];
      const int pos = c.v > 0 ? (step == 0 ? static_cast<int>(c.sizes.size()) - 1 : step - 1) : step;
      const int64_t L = prod(c.sizes, 0, pos), Q = prod(c.sizes, pos + 1, c.sizes.size());
      if (c.v > 0 && step == 0) {           // x_t u_t^T on the parent rank index
        jobs.push_back(left_job(c.cur, L, c.sizes[pos], Q, u[c.v], r, 1, r, out, last ? 1 : 0, last ? alpha : 1.0));
        c.sizes[pos] = r;
      } else {                               // x_c dy_c^T on child c's index
        const int ch = t.children[pos];
        jobs.push_back(left_job(c.cur, L, c.sizes[pos], Q, dy[ch], k, 1, k, out, last ? 1 : 0, last ? alpha : 1.0));
        c.sizes[pos] = k;
      }
      c.cur = out;
    }
    if (jobs.empty()) break;
    if (run) launch_bgemm64(jobs, P.g64_part, P.g64_part_elems, st);
  }
}

void kr_dot(Plan& P, const double* const* a, const std::vector<int64_t>& sa, const double* const* b,
            const std::vector<int64_t>& sb, double* d_out, Bump& bump, bool run, hipStream_t st) {
  const int nn = static_cast<int>(P.nodes.size());
  std::vector<double*> G(nn, nullptr);
  for (int v = 1; v < nn; ++v) G[v] = bump.take(static_cast<size_t>(sa[v]) * sb[v]);
  // leaves: G_t = U_a^T U_b
  std::vector<GJob> leaves;
  for (int v = 1; v < nn; ++v) {
    const Node& t = P.nodes[v];
    if (!t.leaf()) continue;
    GJob j;
    j.M = sa[v];
    j.N = sb[v];
    j.K = t.n;
    j.A = a[v];
    j.sAm = t.n;
    j.sAk = 1;
    j.B = b[v];
    j.sBk = 1;
    j.sBn = t.n;
    j.C = G[v];
    j.sCm = 1;
    j.sCn = sa[v];
    leaves.push_back(j);
  }
  if (run) launch_bgemm64(leaves, P.g64_part, P.g64_part_elems, st);
  // internal nodes and the root, deepest level first: W = B_a x_c G_c (child by child),
  // then G_t = W^T B_b over the children's B-side indices
  for (int lev = max_level(P); lev >= 0; --lev) {
    struct Chain {
      int v;
      std::vector<int64_t> sizes;
      const double* cur;
      double* buf[2];
    };
    std::vector<Chain> ch;
    size_t maxm = 0;
    for (int v = 0; v < nn; ++v) {
      const Node& t = P.nodes[v];
      if (t.level != lev || t.leaf()) continue;
      Chain c{v, axes_of(P, v, sa, false), a[v], {nullptr, nullptr}};
      std::vector<int64_t> sz = c.sizes;
      int64_t big = 1;
      for (size_t q = 0; q < t.children.size(); ++q) {
        sz[q] = sb[t.children[q]];
        big = std::max(big, prod(sz, 0, sz.size()));
      }
      c.buf[0] = bump.take(static_cast<size_t>(big));
      c.buf[1] = bump.take(static_cast<size_t>(big));
      maxm = std::max(maxm, t.children.size());
      ch.push_back(c);
    }
    for (size_t q = 0; q < maxm; ++q) {
      std::vector<GJob> jobs;
      for (Chain& c : ch) {
        const Node& t = P.nodes[c.v];
        if (q >= t.children.size()) continue;
        const int cq = t.children[q];
        const int64_t L = prod(c.sizes, 0, q), Q = prod(c.sizes, q + 1, c.sizes.size());
        double* out = c.buf[q % 2];
        jobs.push_back(left_job(c.cur, L, c.sizes[q], Q, G[cq], 1, sa[cq], sb[cq], out, 0, 1.0));
        c.sizes[q] = sb[cq];
        c.cur = out;
      }
      if (run && !jobs.empty()) launch_bgemm64(jobs, P.g64_part, P.g64_part_elems, st);
    }
    std::vector<GJob> fin;
    for (Chain& c : ch) {
      const Node& t = P.nodes[c.v];
      const int64_t Pb = prod(c.sizes, 0, t.children.size());
      GJob j;
      j.M = c.v > 0 ? sa[c.v] : 1;
      j.N = c.v > 0 ? sb[c.v] : 1;
      j.K = Pb;
      j.A = c.cur;
      j.sAm = Pb;
      j.sAk = 1;
      j.B = b[c.v];
      j.sBk = 1;
      j.sBn = Pb;
      j.C = c.v > 0 ? G[c.v] : d_out;
      j.sCm = 1;
      j.sCn = j.M;
      fin.push_back(j);
    }
    if (run && !fin.empty()) launch_bgemm64(fin, P.g64_part, P.g64_part_elems, st);
  }
}

}  // namespace

size_t kr_update_work_bytes(const Plan& P, const std::vector<int64_t>& s) {
  check_ranks(P, s);
  std::vector<const double*> none(P.nodes.size(), nullptr);
  Bump b;
  kr_update(const_cast<Plan&>(P), none.data(), s, 1.0, b, false, nullptr);
  return b.used;
}

size_t ttn_dot_work_bytes(const Plan& P, const std::vector<int64_t>& sa, const std::vector<int64_t>& sb) {
  check_ranks(P, sa);
  check_ranks(P, sb);
  std::vector<const double*> none(P.nodes.size(), nullptr);
  Bump b;
  kr_dot(const_cast<Plan&>(P), none.data(), sa, none.data(), sb, nullptr, b, false, nullptr);
  return b.used;
}

void update_ttn(Plan& P, const double* const* cores, const std::vector<int64_t>& s, double alpha, void* work,
                hipStream_t st) {
  TTNN_REQUIRE(P.variant == TTNN_KR, TTNN_E_STATE, "TTN-format updates need a Khatri-Rao plan");
  Bump b;
  b.base = static_cast<char*>(work);
  kr_update(P, cores, s, alpha, b, true, st);
}

void ttn_dot(Plan& P, const double* const* a, const std::vector<int64_t>& sa, const double* const* b,
             const std::vector<int64_t>& sb, double* d_out, void* work, hipStream_t st) {
  Bump bump;
  bump.base = static_cast<char*>(work);
  kr_dot(P, a, sa, b, sb, d_out, bump, true, st);
}

}  // namespace ttnn
