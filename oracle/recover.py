"""Recovery phase and reconstruction of the oracle (test infrastructure).

Recovery (Sec. 4, "Recovery phase"; Alg. 2 with its internal-node loop read as
running over every internal level from 1; stabilised least squares of the same
section):
    [Q_t, Rt_t] = economy QR of Omega_t, signs fixed so that diag(Rt_t) >= 0
    Rt_t^{+eps}  = V_1 S_1^{-1} U_1^T over singular values sigma_i > eps_t,
                   eps_t = eps_factor * ||Rt_t||_2, eps_factor = 10 u, u = 2^-52
    leaf      B_t = Psi_t Rt_t^{+eps}                               (n_t x r_t)
    internal  B_t = (Q_cm^T kron ... kron Q_c1^T) Psi_t Rt_t^{+eps} (prod r_c x r_t)
    root      B_0 = (Q_cm^T kron ... kron Q_c1^T) Psi_0             (prod r_c)
    (a free mode of a node takes the identity in place of Q_c^T and its size n_m in
    place of r_c)
Cores are stored column-major with the parent's rank index last.

Reconstruction (Def. 5 and its matricised form): U_leaf = B_leaf,
U_t = (U_cm kron ... kron U_c1) B_t, vec(T_hat) = (U_cm kron ... kron U_c1) B_0.
"""

import numpy as np

from .sketch import group_product
from .tree import Tree

U_DOUBLE = 2.0 ** -52
DEFAULT_EPS_FACTOR = 10.0 * U_DOUBLE


def qr_signed(Om):
    Q, Rt = np.linalg.qr(Om, mode="reduced")
    s = np.sign(np.diag(Rt))
    s[s == 0] = 1.0
    return Q * s[None, :], Rt * s[:, None]


def eps_pinv(M, eps_factor=DEFAULT_EPS_FACTOR):
    """Truncated pseudo-inverse of the stabilised generalised Nystrom method
    (Sec. 2): keep singular values strictly above eps_factor * sigma_1."""
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros(M.T.shape), 0
    keep = s > eps_factor * s[0]
    k = int(keep.sum())
    return (Vt[:k].T / s[:k][None, :]) @ U[:, :k].T, k


def _kron_apply(tree: Tree, t, M, mats):
    """(mats[cm] kron ... kron mats[c1]) applied to the rows of M (child c1 fastest),
    the identity at free-mode positions."""
    pos = tree.positions(t)
    cols = M.shape[1] if M.ndim == 2 else 1
    sizes = [mats[x].shape[1] if kind == "c" else tree.dims[x - 1] for kind, x in pos]
    Z = M.reshape(sizes + [cols], order="F")
    for i, (kind, x) in enumerate(pos):
        if kind == "c":
            Z = group_product(Z, [i], mats[x].T)
    return Z.reshape((-1, cols), order="F")


def assemble(sk, tree: Tree, eps_factor=DEFAULT_EPS_FACTOR):
    """Cores from the sketches.  Returns (cores, info) with info per node:
    Q, Rt, pinv, kept rank."""
    Q, Rt, P, kept = {}, {}, {}, {}
    for n in tree.nodes[1:]:
        Q[n.id], Rt[n.id] = qr_signed(sk["Omega"][n.id])
        P[n.id], kept[n.id] = eps_pinv(Rt[n.id], eps_factor)
    cores = {}
    for n in tree.nodes[1:]:
        if n.is_leaf:
            cores[n.id] = sk["Psi"][n.id] @ P[n.id]
        else:
            cores[n.id] = _kron_apply(tree, n.id, sk["Psi"][n.id], {c: Q[c].T for c in n.children}) @ P[n.id]
    cores[0] = _kron_apply(tree, 0, sk["Psi"][0].reshape(-1, 1), {c: Q[c].T for c in tree[0].children}).ravel()
    return cores, {"Q": Q, "Rt": Rt, "pinv": P, "kept": kept}


def core_shape(tree: Tree, t):
    n = tree[t]
    inner = tuple(tree[x].rank if kind == "c" else tree.dims[x - 1] for kind, x in tree.positions(t))
    if t == 0:
        return inner
    if n.is_leaf:
        return (tree.n_of(t), n.rank)
    return inner + (n.rank,)


def reconstruct(cores, tree: Tree):
    """Dense T_hat (logical indexing, float64) from the cores."""
    U = {}
    for n in reversed(tree.nodes[1:]):          # children before parents
        if n.is_leaf:
            U[n.id] = cores[n.id]
        else:
            B = cores[n.id].reshape((-1, n.rank), order="F")
            U[n.id] = _kron_apply(tree, n.id, B, {c: U[c] for c in n.children})
    v = _kron_apply(tree, 0, cores[0].reshape(-1, 1), {c: U[c] for c in tree[0].children})
    # vec index is column-major over children groups, i.e. over modes 1..d
    return v.reshape(tree.dims, order="F")
