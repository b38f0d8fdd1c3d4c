"""Independent routes to the same quantities, used only to pin the oracle.

Everything here is brute force on tiny tensors: explicit dense Kronecker
products and explicit n_t x n_t projectors, never the group-product route of
sketch.py / recover.py.

  * projector form of the approximant (Sec. 4, eq. of the projectors and the
    product over levels; Sec. 5, eq. of the sequential projection and the STTNN
    approximant): T_hat^D = prod_{l=L..1} (kron_k P_{l,k}) T^D, dummies and free
    modes = identity;
  * stabilised generalised Nystrom for a matrix (Sec. 2, Alg. 1 and the
    eps-pseudoinverse variant);
  * the error-analysis quantities of Lemma 2, Lemma 3 / Theorems 1 and 3, and the
    expected bound of Theorem 2 (with the constants of Lemma 4).
"""

import numpy as np

from .recover import DEFAULT_EPS_FACTOR
from .tree import Tree


def unfold_explicit(T, modes):
    """Def. 2 by its index formula, one entry at a time (tiny tensors only)."""
    d = T.ndim
    modes = sorted(modes)
    rest = [a for a in range(d) if a not in modes]
    nI = int(np.prod([T.shape[a] for a in modes]))
    nR = int(np.prod([T.shape[a] for a in rest]))
    M = np.zeros((nI, nR))
    for idx in np.ndindex(*T.shape):
        i, s = 0, 1
        for a in modes:
            i += idx[a] * s
            s *= T.shape[a]
        j, s = 0, 1
        for a in rest:
            j += idx[a] * s
            s *= T.shape[a]
        M[i, j] = T[idx]
    return M


def vec_f(T):
    return T.reshape(-1, order="F")


def pinv_eps_svd(M, eps_factor=DEFAULT_EPS_FACTOR):
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    keep = s > eps_factor * s[0]
    return Vt[keep].T @ np.diag(1.0 / s[keep]) @ U[:, keep].T


def kron_rev(mats):
    """kron(mats[-1], ..., mats[0]): first factor is the fastest index."""
    out = np.ones((1, 1))
    for M in mats:
        out = np.kron(M, out)
    return out


def contracted_unfolding(T, tree: Tree, D, t, variant):
    """T_{S_t}^{t} as an explicit matrix: T^{t} (I kron Y_sq kron ... kron Y_s1),
    the form written in the STTNN analysis (Sec. 6.3).  For TTNN, T^{t}."""
    node = tree[t]
    Tt = unfold_explicit(T, [m - 1 for m in node.modes])
    if variant == "ttnn":
        return Tt
    # the column index of T^{t} runs over the modes outside t in order: Y_s on each
    # contracted group of S_t, the identity on every other mode
    items, covered = [], set()
    for s in tree.S(t):
        items.append((tree[s].first, D.Y[s]))
        covered.update(tree[s].modes)
    for m in range(1, tree.d + 1):
        if m not in node.modes and m not in covered:
            items.append((m, np.eye(tree.dims[m - 1])))
    K = kron_rev([M for _, M in sorted(items, key=lambda it: it[0])])
    return Tt @ K


def projector(T, tree: Tree, D, t, variant, eps_factor=DEFAULT_EPS_FACTOR):
    A = contracted_unfolding(T, tree, D, t, variant)
    AX = A @ D.X[t]
    return AX @ pinv_eps_svd(D.Y[t].T @ AX, eps_factor) @ D.Y[t].T


def level_groups(tree: Tree, level):
    """Mode groups at `level` of the extended tree, left to right: real nodes at
    that level, dummy extensions of shallower leaves, and the free modes of
    shallower nodes (identity groups, ("f", mode))."""
    out = []
    for n in tree.nodes:
        if n.level == level or (n.is_leaf and n.level < level):
            out.append((n.first, n.id))
        if n.level < level:
            out += [(m, ("f", m)) for m in n.free]
    return [g for _, g in sorted(out, key=lambda it: it[0])]


def level_operator(tree: Tree, level, mats):
    """kron over the groups of `level` of mats[id] (identity where id not in mats)."""
    facs = []
    for g in level_groups(tree, level):
        if isinstance(g, tuple):
            facs.append(np.eye(tree.dims[g[1] - 1]))
        elif g in mats and tree[g].level == level:
            facs.append(mats[g])
        else:
            facs.append(np.eye(tree.n_of(g)))
    return kron_rev(facs)


def approximant_projector_form(T, tree: Tree, D, variant, eps_factor=DEFAULT_EPS_FACTOR):
    P = {n.id: projector(T, tree, D, n.id, variant, eps_factor) for n in tree.nodes[1:]}
    v = vec_f(T)
    for lev in range(1, tree.depth + 1):
        v = level_operator(tree, lev, P) @ v
    return v.reshape(tree.dims, order="F"), P


def stab_gn(A, X, Y, eps_factor=DEFAULT_EPS_FACTOR):
    """A X (Y^T A X)^{+eps} Y^T A (Sec. 2, stabilised generalised Nystrom)."""
    AX = A @ X
    return AX @ pinv_eps_svd(Y.T @ AX, eps_factor) @ (Y.T @ A)


def gn_qr(A, X, Y):
    """Alg. 1: (A X R^{-1}) (Q^T Y^T A) with Q R = Y^T A X."""
    Q, R = np.linalg.qr(Y.T @ A @ X)
    return np.linalg.solve(R.T, (A @ X).T).T @ (Q.T @ (Y.T @ A))


# ---- error analysis ----------------------------------------------------------
def later_nodes(tree: Tree, t):
    """Real nodes (s) with (level, k) after t: deeper levels, or same level to the right."""
    n = tree[t]
    return [m.id for m in tree.nodes[1:]
            if m.level > n.level or (m.level == n.level and m.first > n.first)]


def lemma2_terms(T, tree: Tree, P):
    """The summands of Lemma 2, one per real non-root node."""
    v = vec_f(T)
    terms = {}
    for n in tree.nodes[1:]:
        mats = {}
        for g in level_groups(tree, n.level):
            if g == n.id:
                mats[g] = np.eye(P[g].shape[0]) - P[g]
            elif tree[g].level == n.level and tree[g].first > n.first:
                mats[g] = P[g]
        w = level_operator(tree, n.level, mats) @ v
        for lev in range(n.level + 1, tree.depth + 1):
            w = level_operator(tree, lev, P) @ w
        terms[n.id] = np.linalg.norm(w)
    return terms


def eta(T, tree: Tree, D, t, variant):
    """eta_t = 1 + ||(Y^T Q)^+ Y^T Q_perp||_2 with Q = orth(A X) (Lemma 3)."""
    A = contracted_unfolding(T, tree, D, t, variant)
    Qf, _ = np.linalg.qr(A @ D.X[t], mode="complete")
    r = D.X[t].shape[1]
    Q, Qp = Qf[:, :r], Qf[:, r:]
    Y = D.Y[t]
    if Qp.shape[1] == 0:
        return 1.0
    return 1.0 + np.linalg.norm(np.linalg.pinv(Y.T @ Q) @ (Y.T @ Qp), 2)


def lemma3_bounds(T, tree: Tree, D, P, variant):
    """Per-node right-hand side of Lemma 3: prod(eta over later nodes) * ||(I-P_t) A_t||_F,
    with A_t the (possibly contracted) unfolding of T used to build P_t."""
    et = {n.id: eta(T, tree, D, n.id, variant) for n in tree.nodes[1:]}
    out = {}
    for n in tree.nodes[1:]:
        Tt = unfold_explicit(T, [m - 1 for m in n.modes])
        base = np.linalg.norm(Tt - P[n.id] @ Tt)
        out[n.id] = float(np.prod([et[s] for s in later_nodes(tree, n.id)])) * base
    return out, et


def theorem2_bound(T, tree: Tree, rhat):
    """First line of Theorem 2: expected-error bound for Gaussian DRMs."""
    total = 0.0
    for n in tree.nodes[1:]:
        r, p, rh = n.rank, n.over, rhat
        assert p >= 2 and rh < r - 1
        sv = np.linalg.svd(unfold_explicit(T, [m - 1 for m in n.modes]), compute_uv=False)
        tail = np.sqrt(np.sum(sv[rh:] ** 2))
        cprime = np.sqrt(1 + r / (p - 1)) * np.sqrt(1 + rh / (r - rh - 1))
        prod = 1.0
        for s in later_nodes(tree, n.id):
            prod *= 1 + np.sqrt(tree[s].rank / (tree[s].over - 1))
        total += prod * cprime * tail
    return total
