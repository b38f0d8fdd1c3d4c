"""Khatri-Rao structured sketches of tensors given in TTN format (test infrastructure).

Sec. 7 of the paper: with per-mode Gaussian factors X_i (n_i x r) and Y_i (n_i x (r+p)),
the maps of node t are the column-wise Khatri-Rao products
    X_t = khatri-rao of X_i over the modes outside I_t,
    Y_t = khatri-rao of Y_i over the modes of I_t,
so column j of X_t is the Kronecker product of the j-th columns of its factors.  Row
order is the column-major index over the modes (first mode fastest), as for every map
here: X_t[row(i), j] = prod_{mu} X_mu[i_mu, j].  The factor entries are the oracle's
counter-based Gaussians with tag 2 (64 + mu) + kind (mu 0-based, kind 0 = X, 1 = Y),
beside the per-node tags 2 v + kind (v < 64) of the unstructured maps.

For a tensor in TTN format (cores as in Def. 5, stored column-major: leaf (n_t, s_t),
internal (s_c1, .., s_cm, s_t), root (s_c1, .., s_cm)) the TTNN sketches of Sec. 4 with
these maps are formed by contracting the tree, at a cost linear in the n_i (the two
entry-wise formulas of Sec. 7 for Omega and Psi), never forming the tensor:
    d_t^x[:, j] = the subtree of t contracted with the X columns j of its modes,
    d_t^y[:, j] = the same with the Y columns,
    u_t[:, j]   = everything outside the subtree of t contracted with the X columns j,
    Omega_t = (d_t^y)^T u_t,
    Psi_t   = B_t contracted with d_c^y (each child c, its own column index) and u_t,
    Psi_leaf = R_leaf = U_t u_t,  Psi_root = B_root contracted with every d_c^y.
`kr_drms` gives the same maps as dense matrices, so that oracle.sketch of the dense
tensor is the definition these contractions are pinned to (tests/test_oracle_structured.py).
"""
import numpy as np

from .drm import drm as _drm
from .tree import Tree

FACTOR_TAG_BASE = 64


def factor_tag(mode0, kind):
    """Tag of the per-mode factor (0-based mode, kind 0 = X, 1 = Y)."""
    return 2 * (FACTOR_TAG_BASE + mode0) + kind


def factors(seed, dims, r, p):
    """Per-mode factors: X[mu] (n_mu x r), Y[mu] (n_mu x (r + p)), 0-based mu."""
    X = [_drm(seed, FACTOR_TAG_BASE + mu, 0, n, r) for mu, n in enumerate(dims)]
    Y = [_drm(seed, FACTOR_TAG_BASE + mu, 1, n, r + p) for mu, n in enumerate(dims)]
    return X, Y


def khatri_rao(mats):
    """Column-wise Khatri-Rao product with the first matrix's row index fastest:
    out[i_1 + n_1 i_2 + .., j] = prod_q mats[q][i_q, j]."""
    out = mats[0]
    for M in mats[1:]:
        out = (out[:, None, :] * M[None, :, :]).reshape(-1, out.shape[1], order="F")
    return out


class KRDRMs:
    """Dense Khatri-Rao maps of every non-root node (the definition)."""

    def __init__(self, tree: Tree, X, Y):
        if tree.has_free_modes:
            raise ValueError("Khatri-Rao maps are modelled for trees without free modes")
        self.X, self.Y = {}, {}
        for n in tree.nodes[1:]:
            outside = [m - 1 for m in range(1, tree.d + 1) if m not in n.modes]
            inside = [m - 1 for m in n.modes]
            self.X[n.id] = khatri_rao([X[m] for m in outside])
            self.Y[n.id] = khatri_rao([Y[m] for m in inside])


def kr_drms(tree: Tree, X, Y):
    return KRDRMs(tree, X, Y)


def _contract_children(B, child_mats, last=None):
    """sum over a_1..a_m of B[a_1, .., a_m, (a_t)] prod_q child_mats[q][a_q, j] (the same
    j for every child) -> (s_t, r) if B has a trailing parent index, else (r,)."""
    m = len(child_mats)
    letters = "abcdefghijklmnop"
    sub_b = letters[:m] + ("z" if last else "")
    subs = [sub_b] + [letters[q] + "y" for q in range(m)]
    out = ("z" if last else "") + "y"
    return np.einsum(",".join(subs) + "->" + out, B, *child_mats, optimize=True)


def _leaf_map(tree, t, F):
    return khatri_rao([F[m - 1] for m in tree[t].modes])


def down_vectors(tree: Tree, cores, F):
    """d_t for every non-root node: the subtree of t contracted with the columns of the
    per-mode factors F (X or Y), one column index j shared by every mode."""
    d = {}
    for n in reversed(tree.nodes[1:]):               # children before parents
        B = cores[n.modes]
        if n.is_leaf:
            d[n.id] = B.T @ _leaf_map(tree, n.id, F)
        else:
            d[n.id] = _contract_children(B, [d[c] for c in n.children], last=True)
    return d


def up_vectors(tree: Tree, cores, dx):
    """u_t for every non-root node: everything outside the subtree of t contracted with
    the X columns j (top-down)."""
    u = {}
    for n in tree.nodes:                               # parents before children
        if n.is_leaf:
            continue
        B = cores[n.modes]
        m = len(n.children)
        letters = "abcdefghijklmnop"
        for q, c in enumerate(n.children):
            subs_b = letters[:m] + ("z" if n.id != 0 else "")
            ops, subs = [B], [subs_b]
            for q2, c2 in enumerate(n.children):
                if q2 != q:
                    ops.append(dx[c2])
                    subs.append(letters[q2] + "y")
            if n.id != 0:
                ops.append(u[n.id])
                subs.append("zy")
            u[c] = np.einsum(",".join(subs) + "->" + letters[q] + "y", *ops, optimize=True)
    return u


def ttn_sketch(cores, tree: Tree, X, Y):
    """Omega_t, Psi_t (R_t for leaves) and Psi_0 of the TTN with the given cores under
    the Khatri-Rao maps of X, Y, by tree contraction (same dict layout as oracle.sketch,
    without R for internal nodes)."""
    if tree.has_free_modes:
        raise ValueError("Khatri-Rao maps are modelled for trees without free modes")
    dx = down_vectors(tree, cores, X)
    dy = down_vectors(tree, cores, Y)
    u = up_vectors(tree, cores, dx)
    R, Om, Psi = {}, {}, {}
    letters = "abcdefghijklmnop"
    for n in tree.nodes[1:]:
        Om[n.id] = dy[n.id].T @ u[n.id]
        B = cores[n.modes]
        if n.is_leaf:
            R[n.id] = B @ u[n.id]
            Psi[n.id] = R[n.id]
            continue
        m = len(n.children)
        subs = [letters[:m] + "z"] + [letters[q] + letters[q].upper() for q in range(m)] + ["zy"]
        out = "".join(letters[q].upper() for q in range(m)) + "y"
        P = np.einsum(",".join(subs) + "->" + out, B, *[dy[c] for c in n.children], u[n.id], optimize=True)
        Psi[n.id] = P.reshape((-1, P.shape[-1]), order="F")
    root = tree[0]
    m = len(root.children)
    subs = [letters[:m]] + [letters[q] + letters[q].upper() for q in range(m)]
    out = "".join(letters[q].upper() for q in range(m))
    P0 = np.einsum(",".join(subs) + "->" + out, cores[root.modes], *[dy[c] for c in root.children], optimize=True)
    Psi[0] = P0.reshape(-1, order="F")
    return {"R": R, "Omega": Om, "Psi": Psi}


def ttn_dot(tree: Tree, A, B):
    """<A, B> of two TTNs on the same tree (cores keyed by node modes), by contracting
    the two networks node by node (Gram matrices of the frames, bottom-up)."""
    G = {}
    letters = "abcdefghijklmnop"
    caps = "ABCDEFGHIJKLMNOP"
    for n in reversed(tree.nodes):
        a, b = A[n.modes], B[n.modes]
        if n.is_leaf:
            G[n.id] = a.T @ b
            continue
        m = len(n.children)
        tail_a, tail_b = ("z", "Z") if n.id != 0 else ("", "")
        subs = [letters[:m] + tail_a, caps[:m] + tail_b] + [letters[q] + caps[q] for q in range(m)]
        out = tail_a + tail_b
        G[n.id] = np.einsum(",".join(subs) + "->" + out, a, b, *[G[c] for c in n.children], optimize=True)
    return float(G[0])
