// STTNN visiting orders: cost model and search (see order.hpp).
#include "order.hpp"

#include <algorithm>
#include <map>

namespace ttnn {

namespace {

// entries of T with the groups of `set` contracted (k_s each, n_mu on the other modes)
double contracted_entries(const Plan& P, const std::vector<int>& set) {
  std::vector<char> covered(P.d, 0);
  double e = 1.0;
  for (int s : set) {
    e *= static_cast<double>(P.nodes[s].k);
    for (int mu = P.nodes[s].first; mu <= P.nodes[s].last; ++mu) covered[mu] = 1;
  }
  for (int mu = 0; mu < P.d; ++mu)
    if (!covered[mu]) e *= static_cast<double>(P.dims[mu]);
  return e;
}

}  // namespace

double order_cost(const Plan& P, int objective) {
  double cost = 0.0;
  std::map<std::vector<int>, bool> steps;       // chain prefixes formed, each once
  auto chain = [&](const std::vector<int>& pf, size_t upto) {
    for (size_t j = 1; j <= upto && j <= pf.size(); ++j) {
      std::vector<int> p(pf.begin(), pf.begin() + j);
      if (steps[p]) continue;
      steps[p] = true;
      const Node& g = P.nodes[p.back()];
      if (g.ident) continue;                    // identity contraction: nothing to compute
      p.pop_back();
      cost += 2.0 * contracted_entries(P, p) * g.k;
    }
  };
  for (size_t v = 1; v < P.nodes.size(); ++v) {
    const Node& t = P.nodes[v];
    if (t.ident) continue;
    if (objective == TTNN_COST_MAPS) {
      cost += static_cast<double>(t.m) * t.r;
      continue;
    }
    chain(t.S, t.S.size());
    cost += 2.0 * contracted_entries(P, t.S) * t.r;
  }
  if (objective == TTNN_COST_FLOPS) chain(P.nodes[0].visit, P.nodes[0].visit.size());
  return cost;
}

std::vector<int> order_search(const Plan& P, int objective, double* cost) {
  const int nn = static_cast<int>(P.nodes.size());
  const double N = static_cast<double>(P.N);
  std::vector<double> sub(nn, 0.0);             // subtree cost with nothing contracted above
  std::vector<std::vector<int>> best(nn);
  for (int v = nn - 1; v >= 0; --v) {           // level order: children after their parent
    const Node& p = P.nodes[v];
    std::vector<int> ch;
    for (int c : p.children)
      if (!P.nodes[c].ident) ch.push_back(c);
    if (ch.empty()) continue;
    const size_t m = ch.size();
    // w(c, chained): the cost of child c with nothing contracted before it, its chain
    // step included when a later sibling (or, at the root, the root sketch) needs it
    auto w = [&](int c, bool chained) {
      const Node& t = P.nodes[c];
      if (objective == TTNN_COST_MAPS) return N / static_cast<double>(t.n) * t.r + sub[c];
      return 2.0 * N * t.r + sub[c] + (chained ? 2.0 * N * t.k : 0.0);
    };
    auto rho = [&](int c) { return static_cast<double>(P.nodes[c].k) / static_cast<double>(P.nodes[c].n); };
    auto eval = [&](const std::vector<int>& ord) {
      double f = 1.0, s = 0.0;
      for (size_t j = 0; j < m; ++j) {
        s += f * w(ord[j], v == 0 || j + 1 < m);
        f *= rho(ord[j]);
      }
      return s;
    };
    std::vector<int> ord = ch;                  // left to right: the lexicographic order
    double c_best = eval(ord);
    std::vector<int> o_best = ord;
    // every order of the children (at most 8: a node has at most `order` of them); ch
    // ascends, so next_permutation visits each once
    while (std::next_permutation(ord.begin(), ord.end())) {
      const double c = eval(ord);
      if (c < c_best * (1.0 - 1e-12)) {
        c_best = c;
        o_best = ord;
      }
    }
    sub[v] = c_best;
    best[v] = o_best;
  }
  std::vector<int> place(P.n_real, 0);
  for (int v = 0; v < nn; ++v)
    for (size_t j = 0; j < best[v].size(); ++j) place[P.nodes[best[v][j]].caller] = static_cast<int>(j);
  *cost = sub[0];
  return place;
}

}  // namespace ttnn
