// STTNN visiting orders (Sec. 5): the cost model of the sketch phase and the search
// for the cheapest order under it.
#pragma once

#include <vector>

#include "plan.hpp"

namespace ttnn {

// Cost of one whole-tensor sketch pass of an STTNN plan in the plan's own visiting
// order.  objective TTNN_COST_FLOPS: 2 x (entries of the operand) x (columns of the
// map) over every contraction: each R_t = (T_{S_t})^{t} X_t, and each step of the
// chains T x Y_s^T that some S_t or the root sketch needs, once.  TTNN_COST_MAPS: the
// entries of every X_t.  Free modes (identity maps) cost nothing.
double order_cost(const Plan& P, int objective);

// The visiting order of least cost: for every node, the order of its children that
// minimises the cost of its subtree, over all orders (a node has at most 8 children).
// The cost of a subtree is the product of the compressions k_s / n_s of the groups
// contracted before it times its cost with nothing contracted, and the order of the
// ancestors changes nothing else, so the choices of the nodes are independent and the
// result is the optimum of the model over all orders of the tree.  Returns the place of
// each caller node among its siblings (root: 0) and the cost.
std::vector<int> order_search(const Plan& P, int objective, double* cost);

}  // namespace ttnn
