"""Pins of the oracle's recovery phase and reconstruction (CPU only).

* projector form of the approximant (Sec. 4 for TTNN, Sec. 5 for STTNN) built
  from explicit n_t x n_t projectors and Kronecker products: equals the
  reconstruction from the cores;
* exact recovery of tensors of TTN rank <= r (projector argument in the proof of
  Lemma 1);
* order-2 tree reduces to the stabilised generalised Nystrom of Sec. 2 and, without
  truncation, to Alg. 1; Tucker tree reduces to MLN (eq. MLN of Sec. 4);
* Lemma 2 and Lemma 3 (Theorems 1 and 3) inequalities; expected bound of Theorem 2.
"""
import numpy as np
import pytest

import oracle as O
from oracle import checks as C
from workloads import synth as W


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


PROJ_CASES = [
    (O.T4, (3, 4, 3, 2), 2, 1, 0),
    (O.T5, (2, 3, 2, 3, 2), 2, 2, 1),
    (O.TOY, (2, 3, 2, 2, 3, 2), 2, 1, 2),
    (((1, 2), frozenset({3, 4}), 5), (2, 3, 2, 2, 3), 2, 2, 3),
]


@pytest.mark.parametrize("spec,dims,r,p,seed", PROJ_CASES)
@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_projector_form_equals_cores(spec, dims, r, p, seed, variant):
    T = W.small_random_ttn(spec, dims, r + 1, seed=seed, noise=0.05)   # not exactly low rank
    tree = O.Tree(spec, dims, r, p)
    D = O.DRMs(tree, 10 + seed, variant)
    sk = O.sketch(T, tree, D, variant)
    cores, info = O.assemble(sk, tree)
    That = O.reconstruct(cores, tree)
    Tp, _ = C.approximant_projector_form(T, tree, D, variant)
    assert rel(That, Tp) < 1e-12
    assert rel(That, T) > 1e-6           # a genuine approximation, not a copy
    for n in tree.nodes:
        assert np.shape(cores[n.id]) == (int(np.prod(O.core_shape(tree, n.id))),) or \
            np.prod(np.shape(cores[n.id])) == np.prod(O.core_shape(tree, n.id))


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_exact_recovery_config1(variant):
    T = W.config1_tensor(noise=False)
    tree = O.Tree(O.T4, T.shape, 6, 3)
    D = O.DRMs(tree, 1, variant)
    cores, info = O.assemble(O.sketch(T, tree, D, variant), tree)
    assert rel(O.reconstruct(cores, tree), T) < 1e-11
    assert all(k == 4 for k in info["kept"].values())   # eps-truncation drops the excess rank


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_exact_recovery_toy_tree(variant):
    dims = (3, 3, 2, 3, 2, 3)
    T = W.small_random_ttn(O.TOY, dims, 2, seed=4)
    tree = O.Tree(O.TOY, dims, 3, 2)
    D = O.DRMs(tree, 2, variant)
    cores, _ = O.assemble(O.sketch(T, tree, D, variant), tree)
    assert rel(O.reconstruct(cores, tree), T) < 1e-11


def test_noisy_config1_error_tracks_noise():
    T = W.config1_tensor(noise=True)
    tree = O.Tree(O.T4, T.shape, 6, 3)
    for v in ("ttnn", "sttnn"):
        cores, _ = O.assemble(O.sketch(T, tree, O.DRMs(tree, 1, v), v), tree)
        e = rel(O.reconstruct(cores, tree), T)
        assert 1e-8 < e < 1e-4          # noise has relative norm 1e-6


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_order2_reduces_to_stabilised_gn(variant):
    g = np.random.default_rng(5)
    A = g.standard_normal((40, 10)) @ g.standard_normal((10, 40))      # rank 10
    ranks = {(1,): 5, (2,): 12}
    over = {(1,): 3, (2,): 3}
    tree = O.Tree((1, 2), A.shape, ranks, over)
    D = O.DRMs(tree, 6, variant)
    sk = O.sketch(A, tree, D, variant)
    cores, _ = O.assemble(sk, tree)
    That = O.reconstruct(cores, tree)
    t1 = tree.by_modes((1,))
    want = C.stab_gn(A, D.X[t1], D.Y[t1])
    assert rel(That, want) < 1e-12
    # no truncation at node 1 (Omega_1 is 8 x 5 of full rank): also Alg. 1 (QR form)
    assert rel(That, C.gn_qr(A, D.X[t1], D.Y[t1])) < 1e-10
    # closed form P1 A P2^T holds for any rank
    B = g.standard_normal((40, 40))
    sk = O.sketch(B, tree, D, variant)
    cores, _ = O.assemble(sk, tree)
    P1 = C.projector(B, tree, D, t1, variant)
    P2 = C.projector(B, tree, D, tree.by_modes((2,)), variant)
    assert rel(O.reconstruct(cores, tree), P1 @ B @ P2.T) < 1e-12


def test_tucker_tree_is_mln():
    dims = (4, 3, 5, 3)
    spec = (1, 2, 3, 4)
    T = W.small_random_ttn(spec, dims, 2, seed=8, noise=0.1)
    tree = O.Tree(spec, dims, 2, 2)
    D = O.DRMs(tree, 3, "ttnn")
    cores, _ = O.assemble(O.sketch(T, tree, D, "ttnn"), tree)
    Z = T
    for mu in range(4):
        P = C.projector(T, tree, D, tree.by_modes((mu + 1,)), "ttnn")
        Z = np.moveaxis(np.tensordot(P, Z, axes=([1], [mu])), 0, mu)
    assert rel(O.reconstruct(cores, tree), Z) < 1e-12


def test_qr_sign_and_eps_pinv():
    g = np.random.default_rng(9)
    Om = g.standard_normal((9, 6))
    Q, R = O.qr_signed(Om)
    assert np.all(np.diag(R) >= 0) and rel(Q @ R, Om) < 1e-14
    assert np.allclose(Q.T @ Q, np.eye(6), atol=1e-14)
    P, k = O.eps_pinv(R)
    assert k == 6 and rel(P, np.linalg.inv(R)) < 1e-12
    Rd = R.copy()
    Rd[:, 4:] = 0.0
    Rd[4:, :] = 0.0
    P, k = O.eps_pinv(Rd)
    assert k == 4 and rel(P, np.linalg.pinv(Rd)) < 1e-12
    # threshold eps = 10 u ||R||_2 with u = 2^-52 (stabilised least squares, Sec. 4):
    # 1e-14 (above 2.2e-15) is kept, 1e-15 (below) is dropped
    Hq, _ = np.linalg.qr(g.standard_normal((5, 5)))
    Hr, _ = np.linalg.qr(g.standard_normal((5, 5)))
    s = np.array([1.0, 1e-8, 1e-14, 1e-15, 1e-17])
    P, k = O.eps_pinv(Hq @ np.diag(s) @ Hr.T)
    assert k == 3
    want = Hr[:, :3] @ np.diag(1.0 / s[:3]) @ Hq[:, :3].T
    assert rel(P, want) < 1e-2           # conditioning 1e14: agreement to a few digits
    assert abs(O.DEFAULT_EPS_FACTOR - 10 * 2.0**-52) == 0.0


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_lemma2_lemma3_theorem_bounds(variant):
    spec, dims = O.TOY, (3, 2, 3, 2, 3, 2)
    T = W.small_random_ttn(spec, dims, 2, seed=11, noise=0.2)
    tree = O.Tree(spec, dims, 2, 2)
    D = O.DRMs(tree, 12, variant)
    That, P = C.approximant_projector_form(T, tree, D, variant)
    err = np.linalg.norm(T - That)
    terms = C.lemma2_terms(T, tree, P)
    assert err <= sum(terms.values()) * (1 + 1e-12)                       # Lemma 2
    bounds, et = C.lemma3_bounds(T, tree, D, P, variant)
    for t in terms:
        assert terms[t] <= bounds[t] * (1 + 1e-10) + 1e-14                 # Lemma 3
    assert all(e >= 1.0 for e in et.values())
    # the telescoping is tight: the terms are not all zero
    assert sum(terms.values()) > 0.5 * err


def test_theorem2_expected_bound():
    spec, dims = O.T4, (6, 5, 6, 5)
    base = W.small_random_ttn(spec, dims, 3, seed=21)
    T = W.add_relative_noise(base, 0.05, seed=22)
    tree = O.Tree(spec, dims, 5, 3)
    errs = []
    for s in range(200):
        D = O.DRMs(tree, 100 + s, "ttnn")
        cores, _ = O.assemble(O.sketch(T, tree, D, "ttnn"), tree)
        errs.append(np.linalg.norm(O.reconstruct(cores, tree) - T))
    bound = C.theorem2_bound(T, tree, rhat=3)
    assert np.mean(errs) <= bound
    # and the spectral tail of every unfolding bounds each GN projection from below
    assert np.mean(errs) > 0
