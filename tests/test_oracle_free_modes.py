"""Pins of the oracle on trees with free modes (Def. 3 allows a node to contain more
than the union of its children; a free mode acts as a child whose maps, projector and
core are identities, the convention of the paper for dummy nodes):

* tree parsing: the tensor-train chain of Fig. 4, a free mode between two children,
  a free mode of the root; malformed specs are refused;
* on the tensor-train chain, TTNN is eq. (STTA): T_hat = (P_1 kron I)...(P_{1:d-2} kron
  I) P_{1:d-1} T with P_{1:k} = T^{1:k} X (Y^T T^{1:k} X)^+ Y^T, written out with dense
  projectors (checked against the oracle's cores and reconstruction);
* TTNN and STTNN against the projector form of the approximant with identity factors
  at free modes, on three trees;
* exact recovery of tensors whose TT / TTN ranks do not exceed r.
"""
import numpy as np
import pytest

import oracle as O
from oracle.checks import approximant_projector_form, kron_rev

TT4 = (((1, -2), -3), -4)
TT5 = ((((1, -2), -3), -4), -5)
MID = ((1, -2, 3), 4)                  # free mode 2 between the children {1} and {3}
ROOTF = ((1, 2), -3, (4, 5))           # free mode 3 of the root


def test_parse_free_modes():
    t = O.Tree(TT4, (3, 4, 5, 6), 2, 1)
    assert [n.modes for n in t.nodes] == [(1, 2, 3, 4), (1, 2, 3), (1, 2), (1,)]
    assert [n.free for n in t.nodes] == [(4,), (3,), (2,), ()]
    assert t.positions(0) == [("c", 1), ("f", 4)]
    m = O.Tree(MID, (3, 4, 5, 6), 2, 1)
    assert m.positions(1) == [("c", 3), ("f", 2), ("c", 4)]
    assert O.core_shape(m, 1) == (2, 4, 2, 2)
    assert O.core_shape(O.Tree(ROOTF, (3, 4, 5, 6, 7), 2, 1), 0) == (2, 5, 2)
    assert O.Tree((-1, (2, 3)), (3, 3, 3), 2, 1).positions(0) == [("f", 1), ("c", 1)]
    for bad in (((-1, -2), 3), ((2, -1), 3), ((1, -1), 2)):
        with pytest.raises(O.TreeError):
            O.Tree(bad, (3, 3, 3), 2, 1)


def _tt_dense(dims, s, seed):
    """A tensor of TT ranks s: cores G_k (s_{k-1}, n_k, s_k), contracted left to right."""
    g = np.random.default_rng(seed)
    d = len(dims)
    ranks = [1] + [s] * (d - 1) + [1]
    T = g.standard_normal((dims[0], ranks[1]))
    for k in range(1, d):
        G = g.standard_normal((ranks[k], dims[k], ranks[k + 1]))
        T = np.tensordot(T, G, axes=([T.ndim - 1], [0]))
    return T.reshape(dims)


def _stta(T, tree, D):
    """eq. (STTA) with dense projectors, nodes {1..k} of the chain giving X, Y."""
    dims = T.shape
    d = T.ndim
    v = T.reshape(int(np.prod(dims[:-1])), dims[-1], order="F")
    for k in range(d - 1, 0, -1):
        t = tree.by_modes(tuple(range(1, k + 1)))
        A = T.reshape(int(np.prod(dims[:k])), -1, order="F")
        AX = A @ D.X[t]
        P = AX @ np.linalg.pinv(D.Y[t].T @ AX) @ D.Y[t].T
        v = kron_rev([P, np.eye(int(np.prod(dims[k:d - 1])))]) @ v
    return v.reshape(dims, order="F")


@pytest.mark.parametrize("spec,dims", [(TT4, (4, 5, 3, 6)), (TT5, (3, 4, 3, 5, 4))])
def test_tensor_train_chain_is_stta(spec, dims):
    T = np.random.default_rng(2).standard_normal(dims)
    tree = O.Tree(spec, dims, 2, 1)
    D = O.DRMs(tree, 4, "ttnn")
    cores, _ = O.assemble(O.sketch(T, tree, D, "ttnn"), tree)
    That = O.reconstruct(cores, tree)
    ref = _stta(T, tree, D)
    assert np.linalg.norm(That - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(That - T) > 1e-3 * np.linalg.norm(T)      # a real truncation


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("spec,dims", [(TT4, (3, 4, 3, 4)), (MID, (3, 4, 3, 4)), (ROOTF, (3, 2, 4, 3, 2))])
def test_projector_form_with_free_modes(spec, dims, variant):
    T = np.random.default_rng(5).standard_normal(dims)
    tree = O.Tree(spec, dims, 2, 1)
    D = O.DRMs(tree, 7, variant)
    cores, _ = O.assemble(O.sketch(T, tree, D, variant), tree)
    That = O.reconstruct(cores, tree)
    ref, _ = approximant_projector_form(T, tree, D, variant)
    assert np.linalg.norm(That - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_exact_recovery_with_free_modes(variant):
    dims = (5, 4, 6, 5)
    T = _tt_dense(dims, 2, 3)
    tree = O.Tree(TT4, dims, 3, 2)
    cores, _ = O.assemble(O.sketch(T, tree, O.DRMs(tree, 8, variant), variant), tree)
    assert np.linalg.norm(O.reconstruct(cores, tree) - T) <= 1e-10 * np.linalg.norm(T)
    g = np.random.default_rng(4)
    n1, n2, n3, n4 = dims
    U1, U3, U4 = (g.standard_normal((n, 2)) for n in (n1, n3, n4))
    B = g.standard_normal((2, n2, 2, 2))
    B0 = g.standard_normal((2, 2))
    Tm = np.einsum("ia,kc,ajcd,de,le->ijkl", U1, U3, B, B0, U4, optimize=True)
    tree = O.Tree(MID, dims, 3, 2)
    cores, _ = O.assemble(O.sketch(Tm, tree, O.DRMs(tree, 9, variant), variant), tree)
    assert np.linalg.norm(O.reconstruct(cores, tree) - Tm) <= 1e-10 * np.linalg.norm(Tm)
