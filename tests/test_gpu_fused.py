"""GPU parity of the fused one-pass kernel (first root child ({1},{2}), n_1 = 128;
STTNN, and TTNN mode for roots with two children) and of the whole-tensor MFMA
right sketches, against the oracle and against the generic HIP path, through the
C ABI.  The (128, 16, 64, 32) shape is large enough (2^22 entries) for the TTNN
leaves right of A to take the MFMA right-sketch kernel."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL, TOL_ARITH, errs2, failures, sketch_errors, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    return P


_DRM_CACHE = {}


def drms(spec, dims, r, p, seed, variant, dtype="f64"):
    """Oracle DRMs (FP64, or rounded to a plan dtype), generated once per problem."""
    key = (repr(spec), tuple(dims), r, p, seed, variant, dtype)
    if key not in _DRM_CACHE:
        _DRM_CACHE[key] = O.DRMs(O.Tree(spec, dims, r, p), seed, variant, dtype)
    return _DRM_CACHE[key]


def generic_plan(P, *args, **kw):
    os.environ["TTNN_DISABLE_FUSED"] = "1"
    try:
        return P.Plan(*args, **kw)
    finally:
        del os.environ["TTNN_DISABLE_FUSED"]


SHAPES = [
    (O.T4, (128, 16, 8, 32)),
    (O.T4, (128, 8, 16, 16)),
    (((1, 2), (3, (4, 5))), (128, 8, 4, 8, 8)),
    (O.T4, (128, 16, 64, 32)),
]


@pytest.mark.parametrize("shape", SHAPES, ids=["t4a", "t4b", "deep", "t4big"])
@pytest.mark.parametrize("r", [16, 32, 64])
@pytest.mark.parametrize("dtype", ["bf16", "f32", "f64"])
@pytest.mark.parametrize("variant", ["sttnn", "ttnn"])
def test_fused_parity(P, shape, r, dtype, variant):
    spec, dims = shape
    p = r // 2
    T = np.random.default_rng(11).standard_normal(dims)
    dev, consumed = to_device(T, dtype)
    plan = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=4)
    plan.update(dev)
    tree = O.Tree(spec, dims, r, p)
    sk = O.sketch(consumed, tree, drms(spec, dims, r, p, 4, variant), variant)
    errs = sketch_errors(plan, tree, sk)
    bad = failures(errs, TOL[dtype])
    assert not bad, bad
    # the same rounded DRMs on both sides: arithmetic error alone
    if dtype != "f64":
        skr = O.sketch(consumed, tree, drms(spec, dims, r, p, 4, variant, dtype), variant)
        bad = failures(sketch_errors(plan, tree, skr), TOL_ARITH[dtype])
        assert not bad, bad
    gen = generic_plan(P, spec, dims, r, p, variant=variant, dtype=dtype, seed=4)
    gen.update(dev)
    cmp = {}
    for n in tree.nodes:
        for kind in ((0, 1, 2) if n.id else (2,)):
            a = plan.read_sketch(plan.node(n.modes), kind).cpu().numpy()
            b = gen.read_sketch(gen.node(n.modes), kind).cpu().numpy()
            cmp[(n.modes, kind)] = errs2(a, b)
    bad = failures(cmp, TOL_ARITH[dtype])
    assert not bad, bad


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
@pytest.mark.parametrize("variant", ["sttnn", "ttnn"])
def test_fused_streaming_mix(P, dtype, variant):
    """Whole-tensor updates take the fused path, boxes the generic one; the sum of
    both kinds equals the one-shot sketch of the summed tensor."""
    spec, dims, r, p = O.T4, (128, 16, 64, 32), 32, 16
    g = np.random.default_rng(12)
    T1, T2 = g.standard_normal(dims), g.standard_normal(dims)
    d1, c1 = to_device(T1, dtype)
    box = T2[10:90, 3:12, 2:7, 5:30]
    db, cb = to_device(box, dtype)
    plan = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=5)
    plan.update(d1, alpha=2.0)
    plan.update(db, extent=box.shape, offset=(10, 3, 2, 5), alpha=-1.0)
    full = 2.0 * c1
    full[10:90, 3:12, 2:7, 5:30] -= cb
    tree = O.Tree(spec, dims, r, p)
    sk = O.sketch(full, tree, O.DRMs(tree, 5, variant), variant)
    errs = sketch_errors(plan, tree, sk)
    assert not failures(errs, TOL[dtype]), errs
