"""Pins of the oracle's Khatri-Rao structured sketches of TTN-format tensors (Sec. 7):

* the Khatri-Rao product against its entry formula, by brute force over every row;
* the per-node maps against the product of the per-mode factor entries, by brute force;
* the tree contractions against the dense definition: oracle.sketch of the dense tensor
  with the dense Khatri-Rao maps (Omega_t, Psi_t, leaf R_t and the root Psi) on the
  trees of Fig. 1, ((1,2),(3,4)) and (((1,2),3),(4,5)), with a multi-mode leaf too;
* exact recovery of a TTN whose ranks do not exceed r (Sec. 4 recovery on the
  contracted sketches reproduces the tensor);
* the TTN inner product against the dense one, and the sketch of a sum of two TTNs
  against the sum of their sketches (linearity).
"""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import structured as S
from workloads import synth as W


def test_khatri_rao_entry_formula():
    g = np.random.default_rng(0)
    mats = [g.standard_normal((n, 3)) for n in (2, 4, 3)]
    K = S.khatri_rao(mats)
    assert K.shape == (24, 3)
    for i1, i2, i3 in itertools.product(range(2), range(4), range(3)):
        row = i1 + 2 * i2 + 8 * i3
        np.testing.assert_array_equal(K[row], mats[0][i1] * mats[1][i2] * mats[2][i3])


def test_node_maps_are_products_of_factor_entries():
    dims = (3, 2, 4, 2)
    tree = O.Tree(O.T4, dims, 3, 2)
    X, Y = S.factors(5, dims, 3, 2)
    assert [x.shape for x in X] == [(n, 3) for n in dims]
    assert [y.shape for y in Y] == [(n, 5) for n in dims]
    # factors are the oracle's Gaussians under their own tags
    for mu in range(4):
        for F, kind, k in ((X, 0, 3), (Y, 1, 5)):
            i, j = np.meshgrid(np.arange(dims[mu]), np.arange(k), indexing="ij")
            tag = S.factor_tag(mu, kind)
            np.testing.assert_array_equal(F[mu], O.gaussian(5, tag // 2, tag % 2, i, j))
    D = S.kr_drms(tree, X, Y)
    for n in tree.nodes[1:]:
        outside = [m for m in range(1, 5) if m not in n.modes]
        for j in range(3):
            for idx in itertools.product(*[range(dims[m - 1]) for m in outside]):
                row = np.ravel_multi_index(idx, [dims[m - 1] for m in outside], order="F")
                want = np.prod([X[m - 1][i, j] for m, i in zip(outside, idx)])
                assert D.X[n.id][row, j] == want
        for j in range(5):
            for idx in itertools.product(*[range(dims[m - 1]) for m in n.modes]):
                row = np.ravel_multi_index(idx, [dims[m - 1] for m in n.modes], order="F")
                want = np.prod([Y[m - 1][i, j] for m, i in zip(n.modes, idx)])
                assert D.Y[n.id][row, j] == want


def _close(a, b, tol=1e-12):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    assert np.linalg.norm(a - b) <= tol * max(np.linalg.norm(b), 1e-300), np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    ("toy", O.TOY, (3, 4, 2, 3, 2, 3), 3),
    ("t4", O.T4, (4, 3, 5, 2), 3),
    ("t5", O.T5, (3, 2, 4, 3, 2), 2),
    ("multileaf", ((frozenset({1, 2}), 3), (4, 5)), (3, 2, 4, 3, 2), 2),
]


@pytest.mark.parametrize("name,spec,dims,s", CASES, ids=[c[0] for c in CASES])
def test_tree_contraction_equals_dense_sketch(name, spec, dims, s):
    r, p = 4, 2
    cores = W.gaussian_ttn_cores(spec, dims, s, seed=11)
    T = W.ttn_dense(spec, dims, cores)
    tree = O.Tree(spec, dims, r, p)
    X, Y = S.factors(7, dims, r, p)
    want = O.sketch(T, tree, S.kr_drms(tree, X, Y), "ttnn")
    got = S.ttn_sketch(cores, tree, X, Y)
    for n in tree.nodes[1:]:
        _close(got["Omega"][n.id], want["Omega"][n.id])
        _close(got["Psi"][n.id], want["Psi"][n.id])
        if n.is_leaf:
            _close(got["R"][n.id], want["R"][n.id])
    _close(got["Psi"][0], want["Psi"][0])


@pytest.mark.parametrize("spec,dims", [(O.TOY, (5, 4, 6, 5, 4, 5)), (O.T5, (6, 5, 7, 5, 6))])
def test_exact_recovery_of_low_rank_ttn(spec, dims):
    s, r, p = 2, 3, 2
    cores = W.gaussian_ttn_cores(spec, dims, s, seed=4)
    T = W.ttn_dense(spec, dims, cores)
    tree = O.Tree(spec, dims, r, p)
    X, Y = S.factors(9, dims, r, p)
    oc, _ = O.assemble(S.ttn_sketch(cores, tree, X, Y), tree)
    That = O.reconstruct(oc, tree)
    assert np.linalg.norm(That - T) <= 1e-10 * np.linalg.norm(T)


def _sum_ttn(spec, A, B):
    """Cores of A + B on the same tree: block-diagonal internal cores, stacked leaves,
    and the root as the block sum."""
    out = {}
    for s, modes, par, kids in W.tree_spec_nodes(spec):
        a, b = A[modes], B[modes]
        if not kids:
            out[modes] = np.concatenate([a, b], axis=1)
            continue
        shape = tuple(x + y for x, y in zip(a.shape, b.shape))
        C = np.zeros(shape)
        C[tuple(slice(0, x) for x in a.shape)] = a
        C[tuple(slice(x, None) for x in a.shape)] = b
        out[modes] = C
    return out


def test_ttn_dot_and_linearity():
    spec, dims = O.T5, (4, 3, 5, 3, 4)
    A = W.gaussian_ttn_cores(spec, dims, 2, seed=1)
    B = W.gaussian_ttn_cores(spec, dims, 3, seed=2)
    TA, TB = W.ttn_dense(spec, dims, A), W.ttn_dense(spec, dims, B)
    tr = O.Tree(spec, dims, 3, 0)
    assert abs(S.ttn_dot(tr, A, A) - np.sum(TA * TA)) <= 1e-12 * np.sum(TA * TA)
    assert abs(S.ttn_dot(tr, A, B) - np.sum(TA * TB)) <= 1e-12 * np.linalg.norm(TA) * np.linalg.norm(TB)
    C = _sum_ttn(spec, A, B)
    np.testing.assert_allclose(W.ttn_dense(spec, dims, C), TA + TB, rtol=0, atol=1e-12 * np.abs(TA + TB).max())
    tree = O.Tree(spec, dims, 4, 2)
    X, Y = S.factors(3, dims, 4, 2)
    sa, sb, sc = (S.ttn_sketch(c, tree, X, Y) for c in (A, B, C))
    for key in ("Omega", "Psi"):
        for t in sc[key]:
            _close(sc[key][t], sa[key][t] + sb[key][t], 1e-11)
