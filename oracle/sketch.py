"""TTNN and STTNN sketch phase of the oracle (test infrastructure).

Arrays hold tensors by logical index, T[i1, ..., id] (0-based); every unfolding
follows Def. 2: row index over the chosen modes ascending with the first mode
fastest, column index over the remaining modes ascending with the first fastest.

TTNN (Sec. 4, "Sketch phase"), for every non-root node t:
    R_t   = T^{t} X_t                                  (n_t x r_t)
    Omega = Y_t^T R_t                                  ((r_t+p_t) x r_t)
    Psi_t = R_t                                        (leaf)
    Psi_t = (Y_cm^T kron ... kron Y_c1^T) R_t          (internal; child c1 fastest)
    Psi_0 = T x_{c1} Y_c1^T ... x_{cm} Y_cm^T, vectorised with c1 fastest (root)
The Kronecker order is written so that it matches the column-major unfolding of
Def. 2 (the paper lists the factors from c1 to cm; with c1 the fastest index the
matching Kronecker product has c1 as its last factor).

STTNN (Sec. 5, eq. of the sequential projection): R_t = (T_{S_t})^{t} X_t where
T_{S_t} contracts every group I_s, s in S_t, with Y_s^T, each group replaced in
place by one index of size r_s + p_s; Omega and Psi are then formed from R_t as in
TTNN, and the root sketch is the same.
"""

import numpy as np

from .drm import drm as _drm, rounded
from .tree import Tree


def unfold(T, modes):
    """Def. 2 matricisation of T (logical indexing) over 0-based axis list `modes`."""
    modes = list(modes)
    rest = [a for a in range(T.ndim) if a not in modes]
    nI = int(np.prod([T.shape[a] for a in modes], dtype=np.int64))
    nR = int(np.prod([T.shape[a] for a in rest], dtype=np.int64))
    return np.transpose(T, modes + rest).reshape((nI, nR), order="F")


def fold(M, shape, modes):
    """Inverse of unfold for a tensor of the given shape."""
    modes = list(modes)
    rest = [a for a in range(len(shape)) if a not in modes]
    perm = modes + rest
    Tp = M.reshape([shape[a] for a in perm], order="F")
    return np.transpose(Tp, np.argsort(perm))


def group_product(Z, axes, M):
    """Contract the consecutive axes `axes` of Z (jointly, first fastest) with the
    first index of matrix M; the result index (size M.shape[1]) takes the place
    of the group.  This is the generalised mode product of Def. 1 with the
    contracted group matricised as in Def. 2."""
    axes = list(axes)
    assert axes == list(range(axes[0], axes[0] + len(axes)))
    G = unfold(Z, axes)                                  # (n_group, rest)
    out = M.T @ G                                        # (k, rest)
    rest_shape = [Z.shape[a] for a in range(Z.ndim) if a not in axes]
    new = out.reshape([M.shape[1]] + rest_shape, order="F")
    return np.moveaxis(new, 0, axes[0])


class DRMs:
    """The X_t, Y_t of a tree: float64 masters, optionally rounded to a storage dtype."""

    def __init__(self, tree: Tree, seed: int, variant: str, dtype: str = "f64"):
        self.tree, self.seed, self.variant, self.dtype = tree, seed, variant, dtype
        self.X, self.Y = {}, {}
        for n in tree.nodes[1:]:
            mt = tree.x_rows(n.id, variant)
            self.X[n.id] = rounded(_drm(seed, n.id, 0, mt, n.rank), dtype)
            self.Y[n.id] = rounded(_drm(seed, n.id, 1, tree.n_of(n.id), n.k), dtype)


def _node_axes(tree, t):
    return [m - 1 for m in tree[t].modes]


def root_sketch(T, tree: Tree, D: DRMs):
    """Psi at the root: T contracted with Y_c^T over every child group (free modes of
    the root left as they are), vectorised."""
    Z = T
    pos = 0
    for kind, x in tree.positions(0):
        if kind == "c":
            width = len(tree[x].modes)
            Z = group_product(Z, range(pos, pos + width), D.Y[x])
        pos += 1
    return Z.reshape(-1, order="F")


def right_sketch(T, tree: Tree, D: DRMs, t: int, variant: str):
    """R_t of TTNN (S_t empty) or STTNN (S_t from tree.S): T contracted with Y_s^T over
    every group s of S_t (each collapsed in place to one index), then unfolded at the
    modes of t and multiplied by X_t (rows over the remaining indices in order)."""
    Z = T
    S = tree.S(t) if variant == "sttnn" else []
    labels = list(range(1, tree.d + 1))          # each axis labelled by its first mode
    for s in S:
        i, width = labels.index(tree[s].first), len(tree[s].modes)
        Z = group_product(Z, range(i, i + width), D.Y[s])
        labels[i:i + width] = [tree[s].first]
    i = labels.index(tree[t].first)
    tax = list(range(i, i + len(tree[t].modes)))
    return unfold(Z, tax) @ D.X[t]


def psi_internal(tree: Tree, D: DRMs, t: int, R):
    """(Y_cm^T kron ... kron Y_c1^T) R_t computed as successive group products, with
    the identity at free-mode positions."""
    pos = tree.positions(t)
    sizes = [tree.n_of(x) if kind == "c" else tree.dims[x - 1] for kind, x in pos]
    r = R.shape[1]
    Z = R.reshape(sizes + [r], order="F")
    for i, (kind, x) in enumerate(pos):
        if kind == "c":
            Z = group_product(Z, [i], D.Y[x])
    return Z.reshape((-1, r), order="F")


def sketch(T, tree: Tree, D: DRMs, variant: str):
    """All sketches of the sketch phase.  Returns dict with R, Omega, Psi (by node id)."""
    assert variant in ("ttnn", "sttnn")
    T = np.asarray(T, dtype=np.float64)
    assert T.shape == tree.dims
    R, Om, Psi = {}, {}, {}
    for n in tree.nodes[1:]:
        R[n.id] = right_sketch(T, tree, D, n.id, variant)
        Om[n.id] = D.Y[n.id].T @ R[n.id]
        Psi[n.id] = R[n.id] if n.is_leaf else psi_internal(tree, D, n.id, R[n.id])
    Psi[0] = root_sketch(T, tree, D)
    return {"R": R, "Omega": Om, "Psi": Psi}


def sketch_update(state, block, offset, alpha, tree: Tree, D: DRMs, variant: str):
    """Streaming (Sec. 4, linearity paragraph): add alpha * sketch of the
    zero-padded block placed at `offset` to the running sums in `state`."""
    full = np.zeros(tree.dims)
    sl = tuple(slice(o, o + e) for o, e in zip(offset, np.shape(block)))
    full[sl] = block
    sk = sketch(full, tree, D, variant)
    if state is None:
        return {k: {i: alpha * v for i, v in d.items()} for k, d in sk.items()}
    for k, d in sk.items():
        for i, v in d.items():
            state[k][i] = state[k][i] + alpha * v
    return state


def _box_rows(dims, modes, off, ext):
    """Column-major row indices (over `modes`) of the box entries, first fastest."""
    idx = np.zeros(1, dtype=np.int64)
    stride = 1
    for m in modes:
        r = np.arange(off[m - 1], off[m - 1] + ext[m - 1], dtype=np.int64) * stride
        idx = (idx[:, None] + r[None, :]).reshape(-1, order="F")
        stride *= dims[m - 1]
    return idx


def box_drms(tree: Tree, seed: int, variant: str, offset, ext):
    """The DRM rows a box update touches: Y_s rows over the box for every group that
    is contracted (STTNN reuse sets and root children), X_t rows over the box
    (full range on contracted indices) for every non-root t."""
    if tree.has_free_modes:
        raise ValueError("box updates of trees with free modes are not modelled here")
    from .drm import gaussian
    dims = tree.dims
    off = tuple(int(o) for o in offset)
    ext = tuple(int(e) for e in ext)
    groups = set(tree[0].children)
    if variant == "sttnn":
        for n in tree.nodes[1:]:
            groups.update(tree.S(n.id))
    Y = {}
    for s in sorted(groups):
        rows = _box_rows(dims, tree[s].modes, off, ext)
        Y[s] = gaussian(seed, s, 1, rows[:, None].astype(np.uint64), np.arange(tree[s].k, dtype=np.uint64)[None, :])
    X = {}
    for n in tree.nodes[1:]:
        S = tree.S(n.id) if variant == "sttnn" else []
        sizes, offs, exts = [], [], []
        for sg in S:
            sizes.append(tree[sg].k), offs.append(0), exts.append(tree[sg].k)
        for m in range(1, tree.d + 1):
            if m in n.modes or any(m in tree[sg].modes for sg in S):
                continue
            sizes.append(dims[m - 1]), offs.append(off[m - 1]), exts.append(ext[m - 1])
        rows = np.zeros(1, dtype=np.int64)
        stride = 1
        for sz, o, e in zip(sizes, offs, exts):
            rows = (rows[:, None] + (np.arange(o, o + e, dtype=np.int64) * stride)[None, :]).reshape(-1, order="F")
            stride *= sz
        X[n.id] = gaussian(seed, n.id, 0, rows[:, None].astype(np.uint64), np.arange(n.rank, dtype=np.uint64)[None, :])
    return {"X": X, "Y": Y}


def sketch_box(block, offset, tree: Tree, seed: int, variant: str, drms=None):
    """Sketch of the tensor equal to `block` on the box at `offset` and zero elsewhere
    (the streaming update of Sec. 4), using only the DRM rows the box touches
    (box_drms).  Same result as sketch() on the zero-padded tensor."""
    block = np.asarray(block, dtype=np.float64)
    ext = block.shape
    off = tuple(int(o) for o in offset)
    if drms is None:
        drms = box_drms(tree, seed, variant, off, ext)
    X, Y = drms["X"], drms["Y"]

    def chain(prefix):
        Z = block
        for pos, s in enumerate(prefix):
            Z = group_product(Z, range(pos, pos + len(tree[s].modes)), Y[s])
        return Z

    R = {}
    for n in tree.nodes[1:]:
        S = tree.S(n.id) if variant == "sttnn" else []
        Z = chain(S)
        first = len(S) if S else n.first - 1
        tax = list(range(first, first + len(n.modes)))
        full = np.zeros((tree.n_of(n.id), n.rank))
        full[_box_rows(tree.dims, n.modes, off, ext)] = unfold(Z, tax) @ X[n.id]
        R[n.id] = full
    Zr = chain(tree[0].children)
    return {"R": R, "Psi_root": Zr.reshape(-1, order="F")}
