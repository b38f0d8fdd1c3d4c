"""Pins of the oracle's STTNN visiting orders (Sec. 5: the order of the nodes is a free
choice; the paper takes the lexicographic one and notes that finding the best is a
combinatorial problem).  A visiting order lists the children of each node in the order
they are visited; S_t = the siblings of t visited before it, together with those of
every ancestor of t.

* reuse sets derived by hand from that rule on T4 and on the tree of Fig. 1;
* relabelling: visiting the children of every node in a chosen order is the
  lexicographic order of the tree whose modes are renumbered in that order.  With the
  maps carried over (rows permuted), the sketches agree and the approximant is the
  lexicographic approximant of the transposed tensor transposed back;
* the projector form of the approximant (Sec. 5) with the reuse sets of the order;
* exact recovery of tensors of TTN rank <= r under non-lexicographic orders;
* malformed visiting orders are refused.
"""
import types

import numpy as np
import pytest

import oracle as O
from oracle.checks import approximant_projector_form

T4 = ((1, 2), (3, 4))
TOY = (((1, 2), 3), 4, (5, 6))


def _S(tree, t_modes):
    return sorted(tree[s].modes for s in tree.S(tree.by_modes(t_modes)))


def test_reuse_sets_by_hand():
    t = O.Tree(T4, (3, 4, 5, 6), 2, 1, visit=((4, 3), (2, 1)))
    want = {(3, 4): [], (1, 2): [(3, 4)], (4,): [], (3,): [(4,)], (2,): [(3, 4)], (1,): [(2,), (3, 4)]}
    for m, s in want.items():
        assert _S(t, m) == s, m
    # only A's children reversed: the root level keeps A before B
    t = O.Tree(T4, (3, 4, 5, 6), 2, 1, visit=((2, 1), (3, 4)))
    want = {(1, 2): [], (3, 4): [(1, 2)], (2,): [], (1,): [(2,)], (3,): [(1, 2)], (4,): [(1, 2), (3,)]}
    for m, s in want.items():
        assert _S(t, m) == s, m
    # Fig. 1 tree, root children visited (5,6), (1,2,3), (4); inside (1,2,3): 3 first
    t = O.Tree(TOY, (2,) * 6, 2, 1, visit=((5, 6), (3, (1, 2)), 4))
    want = {(5, 6): [], (1, 2, 3): [(5, 6)], (4,): [(1, 2, 3), (5, 6)], (3,): [(5, 6)],
            (1, 2): [(3,), (5, 6)], (1,): [(3,), (5, 6)], (2,): [(1,), (3,), (5, 6)],
            (5,): [], (6,): [(5,)]}
    for m, s in want.items():
        assert _S(t, m) == s, m
    # the default is the lexicographic order
    a, b = O.Tree(TOY, (2,) * 6, 2, 1), O.Tree(TOY, (2,) * 6, 2, 1, visit=TOY)
    assert all(a.S(n.id) == b.S(n.id) for n in a.nodes)


def _flat_modes(spec):
    if isinstance(spec, int):
        return [spec] if spec > 0 else []
    if isinstance(spec, frozenset):
        return sorted(spec)
    out = []
    for c in spec:
        out += _flat_modes(c)
    return out


def _relabel(spec, new):
    if isinstance(spec, int):
        return new[spec]
    if isinstance(spec, frozenset):
        return frozenset(new[m] for m in spec)
    return tuple(_relabel(c, new) for c in spec)


def _permute_rows(M, sizes, order):
    """Rows of M run column-major over `sizes`; return them over sizes[order]."""
    c = M.shape[1]
    A = M.reshape(list(sizes) + [c], order="F")
    return A.transpose(list(order) + [len(sizes)]).reshape(-1, c, order="F")


def _x_items(tree, t):
    """Row positions of X_t of STTNN: (position key, size, label), in positional order."""
    node, items, covered = tree[t], [], set()
    for s in tree.S(t):
        items.append((tree[s].first, tree[s].k, ("g", tree[s].modes)))
        covered.update(tree[s].modes)
    for m in range(1, tree.d + 1):
        if m not in node.modes and m not in covered:
            items.append((m, tree.dims[m - 1], ("m", m)))
    return sorted(items)


@pytest.mark.parametrize("spec,visit,dims", [
    (T4, ((4, 3), (2, 1)), (4, 5, 3, 6)),
    (T4, ((3, 4), (1, 2)), (5, 3, 4, 4)),
    (TOY, ((5, 6), (3, (2, 1)), 4), (3, 2, 3, 2, 3, 2)),
    (TOY, (4, ((1, 2), 3), (6, 5)), (2, 3, 2, 3, 2, 3)),
])
def test_relabelling(spec, visit, dims):
    g = np.random.default_rng(1)
    T = g.standard_normal(dims)
    r, p = 2, 1
    tv = O.Tree(spec, dims, r, p, visit=visit)
    D = O.DRMs(tv, 5, "sttnn")
    sigma = _flat_modes(visit)                       # original modes in visiting order
    new = {m: i + 1 for i, m in enumerate(sigma)}
    tl = O.Tree(_relabel(visit, new), [dims[m - 1] for m in sigma], r, p)
    Tl = np.transpose(T, [m - 1 for m in sigma])
    Dl = types.SimpleNamespace(X={}, Y={})
    for n in tv.nodes[1:]:
        nl = tl.by_modes(tuple(sorted(new[m] for m in n.modes)))
        # Y_t: rows over the modes of t, first fastest, in the new numbering
        order = sorted(range(len(n.modes)), key=lambda i: new[n.modes[i]])
        Dl.Y[nl] = _permute_rows(D.Y[n.id], [dims[m - 1] for m in n.modes], order)
        # X_t: rows over the positions of the contracted tensor outside t
        items = _x_items(tv, n.id)
        key = [min(new[m] for m in lab[1]) if lab[0] == "g" else new[lab[1]] for _, _, lab in items]
        order = sorted(range(len(items)), key=lambda i: key[i])
        assert tl.x_shape_sttnn(nl) == [items[i][1] for i in order]
        Dl.X[nl] = _permute_rows(D.X[n.id], [sz for _, sz, _ in items], order)
    sk = O.sketch(T, tv, D, "sttnn")
    skl = O.sketch(Tl, tl, Dl, "sttnn")
    for n in tv.nodes[1:]:
        nl = tl.by_modes(tuple(sorted(new[m] for m in n.modes)))
        assert np.allclose(sk["Omega"][n.id], skl["Omega"][nl], rtol=1e-12, atol=1e-12 * np.abs(sk["Omega"][n.id]).max())
    That = O.reconstruct(O.assemble(sk, tv)[0], tv)
    Thl = O.reconstruct(O.assemble(skl, tl)[0], tl)
    back = np.transpose(Thl, np.argsort([m - 1 for m in sigma]))
    assert np.linalg.norm(That - back) <= 1e-10 * np.linalg.norm(back)
    assert np.linalg.norm(That - T) > 1e-3 * np.linalg.norm(T)        # a real truncation


@pytest.mark.parametrize("spec,visit,dims", [
    (T4, ((4, 3), (2, 1)), (3, 4, 3, 4)),
    (TOY, ((5, 6), (3, (1, 2)), 4), (2, 3, 2, 2, 3, 2)),
    (((1, -2), -3, 4), (4, -3, (1, -2)), (3, 3, 2, 4)),
])
def test_projector_form_with_visiting_order(spec, visit, dims):
    T = np.random.default_rng(2).standard_normal(dims)
    tree = O.Tree(spec, dims, 2, 1, visit=visit)
    D = O.DRMs(tree, 7, "sttnn")
    cores, _ = O.assemble(O.sketch(T, tree, D, "sttnn"), tree)
    ref, _ = approximant_projector_form(T, tree, D, "sttnn")
    assert np.linalg.norm(O.reconstruct(cores, tree) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_exact_recovery_with_visiting_order():
    g = np.random.default_rng(3)
    dims, s = (4, 5, 3, 6), 2
    U = [g.standard_normal((n, s)) for n in dims]
    BA, BB, B0 = g.standard_normal((s, s, s)), g.standard_normal((s, s, s)), g.standard_normal((s, s))
    T = np.einsum("ia,jb,kc,ld,abe,cdf,ef->ijkl", *U, BA, BB, B0, optimize=True)
    for visit in (((4, 3), (2, 1)), ((3, 4), (2, 1))):
        tree = O.Tree(T4, dims, 3, 2, visit=visit)
        cores, _ = O.assemble(O.sketch(T, tree, O.DRMs(tree, 8, "sttnn"), "sttnn"), tree)
        assert np.linalg.norm(O.reconstruct(cores, tree) - T) <= 1e-10 * np.linalg.norm(T)


def test_bad_visiting_orders():
    for bad in (((1, 2), 3, 4),                     # another tree
                ((1, 2, 3), 4),                     # another tree
                ((3, 4), (2, 1), (1, 2))):          # a node twice
        with pytest.raises(O.TreeError):
            O.Tree(T4, (3, 3, 3, 3), 2, 1, visit=bad)
    O.Tree(T4, (3, 3, 3, 3), 2, 1, visit=((frozenset({4}), 3), (2, 1)))    # a leaf as a one-mode group
