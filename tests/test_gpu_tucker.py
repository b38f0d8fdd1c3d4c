"""Tucker trees on the GPU (a root whose children are all leaves; with TTNN the
approximation is the multilinear Nystrom method, eq. MLN of Sec. 4, which the oracle's
own tests pin), through the C ABI against the oracle:

* four and five leaves, TTNN and STTNN (the chain of contractions runs over every leaf
  visited before the node), FP64 / FP32 / BF16: every sketch element by element (FP32 /
  BF16 also against the oracle fed the same rounded maps), in FP64 the cores and the
  reconstruction, and exact recovery of a tensor of Tucker rank 2 < r (Lemma 1);
* a whole tensor of 4.4M entries, large enough for the MFMA right-sketch forms: every
  sketch against the oracle in FP32 at the arithmetic tolerance.
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL, TOL_ARITH, errs2, failures, sketch_errors, to_device
from workloads import synth as W

pytestmark = pytest.mark.gpu

CASES = [("star4", (1, 2, 3, 4), (9, 7, 8, 6), 3, 2), ("star5", (1, 2, 3, 4, 5), (5, 6, 4, 7, 5), 3, 1)]


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("name,spec,dims,r,p", CASES, ids=[c[0] for c in CASES])
def test_tucker_tree(P, name, spec, dims, r, p, variant, dtype):
    seed = 12
    print(f"tucker {name} {variant} {dtype}", flush=True)
    T = W.small_random_ttn(spec, dims, 2, seed=4, noise=0.05)
    dev, consumed = to_device(T, dtype)
    plan = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=seed)
    plan.update(dev)
    tree = O.Tree(spec, dims, r, p)
    sk = O.sketch(consumed, tree, O.DRMs(tree, seed, variant), variant)
    bad = failures(sketch_errors(plan, tree, sk), TOL[dtype])
    assert not bad, bad
    if dtype != "f64":
        skr = O.sketch(consumed, tree, O.DRMs(tree, seed, variant, dtype), variant)
        bad = failures(sketch_errors(plan, tree, skr), TOL_ARITH[dtype])
        assert not bad, bad
        plan.close()
        return
    cores = plan.assemble()
    oc, _ = O.assemble(sk, tree)
    for i, c in enumerate(cores):
        want = oc[tree.by_modes(plan.node_modes[i])].reshape(-1, order="F")
        assert errs2(c.cpu().numpy(), want)[0] <= 1e-10, plan.node_modes[i]
    That = plan.reconstruct(cores).cpu().numpy()
    ref = W.flat_colmajor(O.reconstruct(oc, tree))
    assert np.linalg.norm(That - ref) <= 1e-10 * np.linalg.norm(ref)
    plan.close()
    # exact recovery at Tucker rank 2 < r
    E = W.small_random_ttn(spec, dims, 2, seed=5)
    edev, _ = to_device(E, "f64")
    plan = P.Plan(spec, dims, r, p, variant=variant, dtype="f64", seed=seed)
    plan.update(edev)
    e2, n2 = P.diff_norms(plan.reconstruct(plan.assemble()), edev)
    assert np.sqrt(e2 / n2) < 1e-11, np.sqrt(e2 / n2)
    plan.close()


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_tucker_tree_mfma_sizes(P, variant):
    spec, dims, r, p, seed = (1, 2, 3, 4), (64, 48, 40, 36), 8, 4, 13
    print(f"tucker large {variant}", flush=True)
    g = np.random.default_rng(31)
    T = g.standard_normal(dims)
    dev, consumed = to_device(T, "f32")
    plan = P.Plan(spec, dims, r, p, variant=variant, dtype="f32", seed=seed)
    plan.update(dev)
    tree = O.Tree(spec, dims, r, p)
    sk = O.sketch(consumed, tree, O.DRMs(tree, seed, variant, "f32"), variant)
    bad = failures(sketch_errors(plan, tree, sk), TOL_ARITH["f32"])
    assert not bad, bad
    plan.close()
