"""Pins of the oracle's tree bookkeeping: Fig. 1 labels, Fig. 5 STTNN sets, validation."""
import pytest

from conftest import golden_rows
import oracle as O


def _labels(tree):
    """(level,k) label of every node id, k counted left to right within the level."""
    out, count = {}, {}
    for n in tree.nodes:
        count[n.level] = count.get(n.level, 0) + 1
        out[n.id] = f"{n.level},{count[n.level]}"
    return out


def test_fig1_level_order():
    tree = O.Tree(O.TOY, (2,) * 6, 2, 1)
    lab = _labels(tree)
    want = {row[0]: tuple(int(m) for m in row[1:]) for row in golden_rows("fig1_toy_tree.txt")}
    assert {lab[n.id]: n.modes for n in tree.nodes} == want
    assert tree.depth == 3
    assert [tree[c].modes for c in tree[0].children] == [(1, 2, 3), (4,), (5, 6)]


def test_fig5_sttnn_sets():
    tree = O.Tree(O.TOY, (2,) * 6, 2, 1)
    lab = _labels(tree)
    inv = {v: k for k, v in lab.items()}
    rows = list(golden_rows("fig5_sttnn_sets.txt"))
    assert len(rows) == 9
    for row in rows:
        t = inv[row[0]]
        want = [] if row[1:] == ["-"] else [inv[x] for x in row[1:]]
        assert tree.S(t) == want, row


def test_sttnn_sets_cover_left_modes():
    for spec, d in ((O.T4, 4), (O.T5, 5), (O.TOY, 6)):
        tree = O.Tree(spec, (3,) * d, 2, 1)
        for n in tree.nodes[1:]:
            cov = sorted(m for s in tree.S(n.id) for m in tree[s].modes)
            assert cov == list(range(1, n.first))


def test_t4_sttnn_x_rows():
    n, r, p = 7, 3, 2
    tree = O.Tree(O.T4, (n,) * 4, r, p)
    k = r + p
    want = {(1, 2): n * n, (3, 4): k, (1,): n**3, (2,): k * n * n, (3,): k * n, (4,): k * k}
    for mod, rows in want.items():
        assert tree.x_rows(tree.by_modes(mod), "sttnn") == rows
        assert tree.x_rows(tree.by_modes(mod), "ttnn") == n ** (4 - len(mod))


@pytest.mark.parametrize("spec", [
    ((1, 3), (2, 4)),            # not contiguous
    ((2, 1), (3, 4)),            # children out of order
    ((1, 2), (3,)),              # root misses a mode for d = 4
    ((1, 2), (2, 3, 4)),         # overlapping
])
def test_invalid_trees_rejected(spec):
    with pytest.raises(O.TreeError):
        O.Tree(spec, (2, 2, 2, 2), 1, 0)


def test_mixed_depth_leaves_and_multimode_leaf():
    spec = ((1, 2), frozenset({3, 4}), 5)
    tree = O.Tree(spec, (2, 3, 2, 2, 3), 2, 1)
    leaf = tree.by_modes((3, 4))
    assert tree[leaf].is_leaf and tree.n_of(leaf) == 4
    assert tree.S(tree.by_modes((5,))) == [tree.by_modes((1, 2)), leaf]
