"""Pins of the oracle's sketch phase (CPU only).

* Def. 2 unfolding against its index formula, entry by entry;
* every TTNN / STTNN sketch against explicit dense Kronecker products
  (the STTNN form written in the analysis of Sec. 6.3);
* linearity (Sec. 4): sums, scaling, box splits, cancelling rank-1 pairs.
"""
import numpy as np
import pytest

import oracle as O
from oracle import checks as C
from workloads import synth as W

CASES = [
    (O.T4, (3, 2, 4, 3), 2, 1),
    (O.T5, (2, 3, 2, 2, 3), 2, 2),
    (O.TOY, (2, 3, 2, 2, 3, 2), 2, 1),
    (((1, 2, 3),), (3, 2, 2), 2, 1),                       # root with one internal child
    (((1, 2), frozenset({3, 4}), 5), (2, 3, 2, 2, 3), 2, 2),
]


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def test_unfold_matches_index_formula():
    rng = np.random.default_rng(0)
    T = rng.standard_normal((3, 2, 4, 2, 3))
    for modes in ([0], [1], [4], [0, 1], [1, 2], [2, 3, 4], [0, 2], [1, 3, 4], [0, 1, 2, 3, 4]):
        assert np.array_equal(O.unfold(T, modes), C.unfold_explicit(T, modes))
        assert np.array_equal(O.fold(O.unfold(T, modes), T.shape, modes), T)


@pytest.mark.parametrize("spec,dims,r,p", CASES)
@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_sketches_brute_force(spec, dims, r, p, variant):
    tree = O.Tree(spec, dims, r, p)
    rng = np.random.default_rng(1)
    T = rng.standard_normal(dims)
    D = O.DRMs(tree, 3, variant)
    sk = O.sketch(T, tree, D, variant)
    for n in tree.nodes[1:]:
        A = C.contracted_unfolding(T, tree, D, n.id, variant)
        R = A @ D.X[n.id]
        assert rel(sk["R"][n.id], R) < 1e-13
        assert rel(sk["Omega"][n.id], D.Y[n.id].T @ R) < 1e-13
        if n.is_leaf:
            assert rel(sk["Psi"][n.id], R) < 1e-13
        else:
            K = C.kron_rev([D.Y[c].T for c in n.children])
            assert rel(sk["Psi"][n.id], K @ R) < 1e-13
    K0 = C.kron_rev([D.Y[c].T for c in tree[0].children])
    assert rel(sk["Psi"][0], K0 @ C.vec_f(T)) < 1e-13


def test_ttnn_and_sttnn_agree_where_s_is_empty():
    tree = O.Tree(O.T4, (3, 4, 2, 3), 2, 1)
    T = np.random.default_rng(2).standard_normal(tree.dims)
    a = O.sketch(T, tree, O.DRMs(tree, 9, "ttnn"), "ttnn")
    b = O.sketch(T, tree, O.DRMs(tree, 9, "sttnn"), "sttnn")
    for mod in [(1, 2), (1,)]:            # S_t empty: same X_t shape and value
        t = tree.by_modes(mod)
        assert np.array_equal(a["R"][t], b["R"][t])
    assert np.array_equal(a["Psi"][0], b["Psi"][0])


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_linearity(variant):
    tree = O.Tree(O.T5, (3, 4, 2, 3, 2), 2, 2)
    D = O.DRMs(tree, 4, variant)
    g = np.random.default_rng(3)
    T1, T2 = g.standard_normal(tree.dims), g.standard_normal(tree.dims)
    s1, s2 = O.sketch(T1, tree, D, variant), O.sketch(T2, tree, D, variant)
    s12 = O.sketch(2.5 * T1 - 0.75 * T2, tree, D, variant)
    for kind in ("R", "Omega", "Psi"):
        for t in s12[kind]:
            assert rel(s12[kind][t], 2.5 * s1[kind][t] - 0.75 * s2[kind][t]) < 1e-13
    # random box splits of T1: sum of per-box sketches equals the one-shot sketch
    state = None
    cuts = [sorted(set([0, n] + list(g.integers(1, n, size=1)))) if n > 1 else [0, n] for n in tree.dims]
    for idx in np.ndindex(*[len(c) - 1 for c in cuts]):
        off = [cuts[m][i] for m, i in enumerate(idx)]
        end = [cuts[m][i + 1] for m, i in enumerate(idx)]
        blk = T1[tuple(slice(o, e) for o, e in zip(off, end))]
        state = O.sketch_update(state, blk, off, 1.0, tree, D, variant)
    for kind in ("R", "Omega", "Psi"):
        for t in s1[kind]:
            assert rel(state[kind][t], s1[kind][t]) < 1e-13
    # a cancelling pair of rank-1 terms leaves the sketch unchanged
    a = [g.standard_normal(n) for n in tree.dims]
    rank1 = a[0]
    for v in a[1:]:
        rank1 = np.multiply.outer(rank1, v)
    state = O.sketch_update(state, rank1, [0] * 5, 1.0, tree, D, variant)
    state = O.sketch_update(state, rank1, [0] * 5, -1.0, tree, D, variant)
    for kind in ("R", "Omega", "Psi"):
        for t in s1[kind]:
            assert rel(state[kind][t], s1[kind][t]) < 1e-12


def test_storage_rounded_drms():
    tree = O.Tree(O.T4, (3, 2, 2, 3), 2, 1)
    D64, D16 = O.DRMs(tree, 1, "ttnn", "f64"), O.DRMs(tree, 1, "ttnn", "bf16")
    for t in D64.X:
        d = np.abs(D16.X[t] - D64.X[t]) / np.maximum(np.abs(D64.X[t]), 1e-300)
        assert d.max() <= 2.0**-8


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("spec,dims", [(O.T4, (5, 4, 6, 3)), (O.TOY, (3, 4, 2, 3, 4, 2))])
def test_sketch_box_equals_zero_padded(spec, dims, variant):
    from oracle.sketch import sketch_box
    tree = O.Tree(spec, dims, 2, 1)
    D = O.DRMs(tree, 5, variant)
    g = np.random.default_rng(4)
    off = [int(g.integers(0, n)) for n in dims]
    ext = [int(g.integers(1, n - o + 1)) for n, o in zip(dims, off)]
    blk = g.standard_normal(ext)
    full = O.sketch_update(None, blk, off, 1.0, tree, D, variant)
    box = sketch_box(blk, off, tree, 5, variant)
    for t in full["R"]:
        assert rel(box["R"][t], full["R"][t]) < 1e-13
    assert rel(box["Psi_root"], full["Psi"][0]) < 1e-13


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("spec,dims,visit", [
    (O.T4, (5, 4, 3, 6), None), (O.T5, (3, 4, 2, 3, 4), None), (O.TOY, (2, 3, 2, 3, 2, 2), None),
    (O.T4, (5, 4, 3, 6), ((4, 3), (2, 1))), (O.TOY, (2, 3, 2, 3, 2, 2), ((5, 6), (3, (1, 2)), 4))])
def test_sampled_entries_match_full_sketch(spec, dims, visit, variant):
    """The one-entry evaluator used for full-size GPU checks equals the full oracle
    sketch, in the lexicographic order and in orders whose S_t has groups right of t."""
    from oracle.sampled import right_entry, root_entry
    T = np.random.default_rng(3).standard_normal(dims)
    tree = O.Tree(spec, dims, 3, 2, visit=visit)
    sk = O.sketch(T, tree, O.DRMs(tree, 9, variant), variant)
    g = np.random.default_rng(4)
    for n in tree.nodes[1:]:
        ext = [dims[m - 1] for m in n.modes]
        for _ in range(3):
            im = [int(g.integers(e)) for e in ext]
            j = int(g.integers(n.rank))
            i = int(np.ravel_multi_index(im, ext, order="F"))
            want = sk["R"][n.id][i, j]
            assert abs(right_entry(T, tree, 9, variant, n.id, im, j) - want) <= 1e-12 * (1 + abs(want))
    kk = [tree[c].k for c in tree[0].children]
    for _ in range(3):
        km = [int(g.integers(k)) for k in kk]
        want = sk["Psi"][0][int(np.ravel_multi_index(km, kk, order="F"))]
        assert abs(root_entry(T, tree, 9, km) - want) <= 1e-12 * (1 + abs(want))
