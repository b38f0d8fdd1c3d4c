"""The 6-D Hilbert tensor of the first accuracy experiment (Sec. 8) and the oracle
on it.  The generator is pinned to the classical Hilbert matrix (scipy) in two
modes, to its closed-form corner entries and to its mode symmetry; the oracle's
approximation of it on the Fig. 1 tree is checked to improve with the rank, as
the error curve of the experiment does, and to be exact where the sketch ranks
reach the ranks of every matricisation."""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
from workloads import hilbert as H
from workloads import synth as W


def test_two_modes_is_the_hilbert_matrix():
    # 1 / (1 + i + j) with 1-based i, j is the classical 1 / (a + b - 1) at a = i + 1, b = j + 1
    n = 9
    assert np.array_equal(H.hilbert_host(n, 2), scipy.linalg.hilbert(n + 1)[1:, 1:])
    assert np.array_equal(H.hilbert_host(n, 1), 1.0 / np.arange(2, n + 2))


def test_corners_and_symmetry():
    n = 5
    T = H.hilbert_host(n)
    assert T.shape == (n,) * 6
    assert T[(0,) * 6] == 1.0 / 7.0
    assert T[(n - 1,) * 6] == 1.0 / (1 + 6 * n)
    assert T[1, 2, 3, 4, 0, 1] == 1.0 / (1 + 2 + 3 + 4 + 5 + 1 + 2)
    for perm in [(1, 0, 2, 3, 4, 5), (5, 4, 3, 2, 1, 0), (2, 0, 4, 1, 5, 3)]:
        assert np.array_equal(T, T.transpose(perm))
    # symmetric, so the column-major flattening is the row-major one
    assert np.array_equal(W.flat_colmajor(T), T.reshape(-1))


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_oracle_error_decays_with_rank(variant):
    n = 8
    T = H.hilbert_host(n)
    errs = []
    for r in (2, 4, 6):
        tree = O.Tree(H.TOY, (n,) * 6, r, H.P_PAPER)
        sk = O.sketch(T, tree, O.DRMs(tree, 11, variant), variant)
        cores, _ = O.assemble(sk, tree)
        errs.append(np.linalg.norm(O.reconstruct(cores, tree) - T) / np.linalg.norm(T))
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs
    assert errs[0] < 1e-2


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_oracle_exact_at_full_rank(variant):
    # n = 2: no node has more than 8 rows in its matricisation (n_t <= 8), so r = 8
    # reaches every matricisation rank and the approximant reproduces the tensor (the
    # rank-deficient Omega_t are handled by the eps-pseudoinverse)
    n = 2
    T = H.hilbert_host(n)
    tree = O.Tree(H.TOY, (n,) * 6, 8, 0)
    sk = O.sketch(T, tree, O.DRMs(tree, 3, variant), variant)
    cores, _ = O.assemble(sk, tree)
    assert np.linalg.norm(O.reconstruct(cores, tree) - T) / np.linalg.norm(T) < 1e-12
