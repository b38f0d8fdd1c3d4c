"""The recovery at the sketch ranks the plans accept, on the GPU through the C ABI,
against the oracle (Sec. 4 recovery phase, Alg. 2):

* the largest ranks at r = 64: p = 91, k = 155, the most that one workgroup's LDS holds
  for the QR and pseudo-inverse of a 155 x 64 Omega_t;
* a tree whose nodes take every form of the recovery kernel at once (k = 256 with
  r = 16, r = 48 with k = 148, r = 64 with k = 96, r = 40 with k = 64): each launch
  sizes its LDS from its own jobs.

Both on a TTN of rank 2 below every r: every sketch element by element, the cores, and
exact recovery (Lemma 1).
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL, errs2, failures, sketch_errors, to_device
from workloads import synth as W

pytestmark = pytest.mark.gpu

MIXED_R = {(1,): 16, (2,): 64, (3,): 40, (4,): 8, (1, 2): 32, (3, 4): 48}
MIXED_P = {(1,): 240, (2,): 32, (3,): 24, (4,): 100, (1, 2): 16, (3, 4): 100}
CASES = [("r64-p91", (12, 10, 9, 11), 64, 91), ("mixed", (20, 18, 16, 14), MIXED_R, MIXED_P)]


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("name,dims,r,p", CASES, ids=[c[0] for c in CASES])
def test_recovery_at_rank_limits(P, name, dims, r, p, variant):
    print(f"rank limits {name} {variant}", flush=True)
    T = W.small_random_ttn(O.T4, dims, 2, seed=6)
    dev, consumed = to_device(T, "f64")
    plan = P.Plan(O.T4, dims, r, p, variant=variant, dtype="f64", seed=9)
    plan.update(dev)
    tree = O.Tree(O.T4, dims, r, p)
    sk = O.sketch(consumed, tree, O.DRMs(tree, 9, variant), variant)
    bad = failures(sketch_errors(plan, tree, sk), TOL["f64"])
    assert not bad, bad
    cores = plan.assemble()
    oc, _ = O.assemble(sk, tree)
    for i, c in enumerate(cores):
        want = oc[tree.by_modes(plan.node_modes[i])].reshape(-1, order="F")
        assert errs2(c.cpu().numpy(), want)[0] <= 1e-9, plan.node_modes[i]
    e2, n2 = P.diff_norms(plan.reconstruct(cores), dev)
    assert np.sqrt(e2 / n2) < 1e-11, np.sqrt(e2 / n2)
    plan.close()
