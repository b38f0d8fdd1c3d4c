"""Synthetic tensors shaped like the paper's workloads.

* random tree tensor networks with i.i.d. N(0,1) cores (exact TTN rank);
* the paper's rounding-experiment recipe (Sec. 8): superdiagonal internal cores
  with prescribed decay multiplied by Haar orthogonal matrices on every mode,
  Haar orthonormal leaves;
* additive i.i.d. Gaussian noise of prescribed relative Frobenius norm.

Tensors are returned with logical indexing T[i1, ..., id] and stored so that the
memory order is column-major (mode 1 fastest): `flat_colmajor(T)` is a view.
All randomness comes from numpy.random.Generator(PCG64(seed)).
"""

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _modes(spec):
    if isinstance(spec, int):
        return (spec,)
    if isinstance(spec, frozenset):
        return tuple(sorted(spec))
    out = ()
    for c in spec:
        out += _modes(c)
    return out


def tree_spec_nodes(spec):
    """Breadth-first list of (spec, modes, parent_index, child_specs)."""
    out = []
    queue = [(spec, -1)]
    while queue:
        nxt = []
        for s, par in queue:
            kids = list(s) if isinstance(s, tuple) else []
            out.append((s, _modes(s), par, kids))
            me = len(out) - 1
            for c in kids:
                nxt.append((c, me))
        queue = nxt
    return out


def _nsize(dims, modes):
    p = 1
    for m in modes:
        p *= dims[m - 1]
    return p


def _rank_of(ranks, modes):
    return int(ranks[modes] if isinstance(ranks, dict) else ranks)


def _core_shape(s, modes, kids, dims, ranks, is_root):
    if is_root:
        return tuple(_rank_of(ranks, _modes(c)) for c in kids)
    if not kids:
        return (_nsize(dims, modes), _rank_of(ranks, modes))
    return tuple(_rank_of(ranks, _modes(c)) for c in kids) + (_rank_of(ranks, modes),)


def gaussian_ttn_cores(spec, dims, ranks, seed):
    """Cores with i.i.d. N(0,1) entries, drawn breadth-first, each filled column-major."""
    g = rng(seed)
    cores = {}
    for i, (s, modes, par, kids) in enumerate(tree_spec_nodes(spec)):
        shape = _core_shape(s, modes, kids, dims, ranks, i == 0)
        cores[modes] = g.standard_normal(int(np.prod(shape))).reshape(shape, order="F")
    return cores


def haar(n, k, g):
    """n x k matrix with orthonormal columns, Haar distributed (QR of a Gaussian, sign fixed)."""
    A = g.standard_normal((n, k))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))[None, :]


def decaying_ttn_cores(spec, dims, rank, sigma, seed):
    """Rounding-experiment recipe: Haar leaves; internal cores superdiagonal with
    entries sigma[k] rotated by independent Haar matrices on every mode."""
    g = rng(seed)
    cores = {}
    sigma = np.asarray(sigma, dtype=np.float64)
    for i, (s, modes, par, kids) in enumerate(tree_spec_nodes(spec)):
        shape = _core_shape(s, modes, kids, dims, rank, i == 0)
        if not kids:
            cores[modes] = haar(shape[0], shape[1], g)
            continue
        r = min(shape)
        C = np.zeros(shape)
        for k in range(r):
            C[(k,) * len(shape)] = sigma[k]
        for ax, n in enumerate(shape):
            H = haar(n, n, g)
            C = np.moveaxis(np.tensordot(H, C, axes=([1], [ax])), 0, ax)
        cores[modes] = C
    return cores


def ttn_dense(spec, dims, cores):
    """Dense tensor of a tree tensor network, built with einsum (float64)."""
    letters = iter("abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ")
    mode_letter = {m: next(letters) for m in range(1, len(dims) + 1)}
    nodes = tree_spec_nodes(spec)

    def build(idx):
        s, modes, par, kids = nodes[idx]
        if not kids:
            rl = next(letters)
            shape = [dims[m - 1] for m in modes] + [cores[modes].shape[1]]
            return cores[modes].reshape(shape, order="F"), "".join(mode_letter[m] for m in modes) + rl
        kid_ids = [j for j, n in enumerate(nodes) if n[2] == idx]
        ops, subs, kid_rank_letters = [], [], []
        for j in kid_ids:
            arr, sub = build(j)
            ops.append(arr)
            subs.append(sub)
            kid_rank_letters.append(sub[-1])
        core = cores[modes]
        if idx == 0:
            csub = "".join(kid_rank_letters)
            out = "".join(mode_letter[m] for m in modes)[::-1]
        else:
            rl = next(letters)
            csub = "".join(kid_rank_letters) + rl
            out = "".join(mode_letter[m] for m in modes) + rl
        expr = ",".join(subs + [csub]) + "->" + out
        return np.einsum(expr, *ops, core, optimize=True), out

    T_rev, _ = build(0)          # axes d..1, C-contiguous
    return np.ascontiguousarray(T_rev).T


def flat_colmajor(T):
    """1-D column-major view of a tensor returned by this module (no copy)."""
    return T.T.reshape(-1)


def add_relative_noise(T, rel, seed, unit_rms=False):
    """T <- T * scale + rel * (||T||/||E||) E with E i.i.d. N(0,1), column-major draw order.
    With unit_rms the clean tensor is first scaled to unit RMS and the noise is drawn
    with standard deviation `rel` directly."""
    g = rng(seed)
    Tr = T.T                                # C-contiguous, reversed axes
    if unit_rms:
        Tr = Tr * (np.sqrt(Tr.size) / np.linalg.norm(Tr.reshape(-1)))
        E = g.standard_normal(Tr.shape)
        return np.ascontiguousarray(Tr + rel * E).T
    E = g.standard_normal(Tr.shape)
    scale = rel * np.linalg.norm(Tr.reshape(-1)) / np.linalg.norm(E.reshape(-1))
    return np.ascontiguousarray(Tr + scale * E).T


def config1_tensor(noise=True):
    """16^4 on ((1,2),(3,4)), TTN with all edge ranks 4, N(0,1) cores (seed 0),
    plus Gaussian noise of relative norm 1e-6."""
    spec, dims = ((1, 2), (3, 4)), (16, 16, 16, 16)
    cores = gaussian_ttn_cores(spec, dims, 4, seed=0)
    T = ttn_dense(spec, dims, cores)
    if noise:
        T = add_relative_noise(T, 1e-6, seed=1)
    return T


def config2_tensor(n=128, rank=24, decay=0.8, noise_std=1e-4, seed=0):
    """n^4 on ((1,2),(3,4)): Haar leaves, superdiagonal cores with sigma_k = decay^(k-1)
    rotated by Haar matrices, normalised to unit RMS, plus N(0, noise_std^2) noise."""
    spec, dims = ((1, 2), (3, 4)), (n, n, n, n)
    sigma = decay ** np.arange(rank)
    cores = decaying_ttn_cores(spec, dims, rank, sigma, seed)
    T = ttn_dense(spec, dims, cores)
    return add_relative_noise(T, noise_std, seed=seed + 1, unit_rms=True)


def unbalanced_tensor(dims=(32, 512, 128, 128), rank=24, decay=0.8, noise_std=1e-4, seed=0):
    """The recipe of config2_tensor on ((1,2),(3,4)) with unequal mode sizes (n_1 << n_2),
    where the STTNN visiting order changes the sizes of the maps."""
    spec = ((1, 2), (3, 4))
    sigma = decay ** np.arange(rank)
    cores = decaying_ttn_cores(spec, dims, rank, sigma, seed)
    T = ttn_dense(spec, dims, cores)
    return add_relative_noise(T, noise_std, seed=seed + 1, unit_rms=True)


def small_random_ttn(spec, dims, ranks, seed, noise=0.0):
    cores = gaussian_ttn_cores(spec, dims, ranks, seed)
    T = ttn_dense(spec, dims, cores)
    if noise:
        T = add_relative_noise(T, noise, seed + 7919)
    return T
