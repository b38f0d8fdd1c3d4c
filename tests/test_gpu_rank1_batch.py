"""Batched rank-1 updates on the GPU (streaming by linearity, Sec. 4), through the C ABI:
ttnn_sketch_update_rank1_batched with 1, 3, 8, 16 and 19 terms (one and two launches of
up to 16 terms) is bitwise equal to the same terms applied one by one with
ttnn_sketch_update_rank1, for TTNN and STTNN (a non-lexicographic order, a free mode) in
FP64 / FP32 / BF16, and the accumulated sketches match the oracle's sketch of the sum
of the terms at the dtype tolerance."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL, failures, sketch_errors

pytestmark = pytest.mark.gpu

T4 = ((1, 2), (3, 4))
T5 = (((1, 2), 3), (4, 5))
TOY = (((1, 2), 3), 4, (5, 6))
FREE = (((1, -2), 3), -4, (5, 6))
CASES = [("t5-ttnn-f32", T5, None, (9, 10, 8, 11, 7), "ttnn", "f32"),
         ("t4-ttnn-f64", T4, None, (12, 40, 10, 9), "ttnn", "f64"),
         ("toy-sttnn-f64-order", TOY, ((5, 6), (3, (1, 2)), 4), (5, 4, 6, 3, 5, 4), "sttnn", "f64"),
         ("free-sttnn-bf16", FREE, None, (5, 4, 6, 3, 5, 4), "sttnn", "bf16")]


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    assert torch.cuda.is_available()
    return P


def _sketches(P, plan, tree):
    out = []
    for n in tree.nodes:
        cid = plan.node(n.modes)
        if n.id == 0:
            out.append(plan.read_sketch(cid, P.SK_PSI).cpu().numpy())
            continue
        for kind in (P.SK_R, P.SK_OMEGA, P.SK_PSI):
            out.append(plan.read_sketch(cid, kind).cpu().numpy())
    return out


@pytest.mark.parametrize("m", [1, 3, 8, 16, 19])
@pytest.mark.parametrize("name,spec,visit,dims,variant,dtype", CASES, ids=[c[0] for c in CASES])
def test_rank1_batched_equals_sequential(P, name, spec, visit, dims, variant, dtype, m):
    print(f"rank1 batch {name} m={m}", flush=True)
    r, p = 4, 2
    g = np.random.default_rng(30 + m)
    vecs = [[g.standard_normal(n) for n in dims] for _ in range(m)]
    alphas = [float(a) for a in g.uniform(-2, 2, size=m)]
    dev = [[torch.from_numpy(v).cuda() for v in term] for term in vecs]
    one = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=4, visit=visit)
    many = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=4, visit=visit)
    for term, a in zip(dev, alphas):
        one.update_rank1(term, alpha=a)
    many.update_rank1_batched(dev, alphas)
    torch.cuda.synchronize()
    tree = O.Tree(spec, dims, r, p, visit=visit)
    for a, b in zip(_sketches(P, one, tree), _sketches(P, many, tree)):
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    T = np.zeros(dims)
    for term, a in zip(vecs, alphas):
        outer = term[0]
        for v in term[1:]:
            outer = np.multiply.outer(outer, v)
        T += a * outer
    sk = O.sketch(T, tree, O.DRMs(tree, 4, variant, dtype), variant)
    bad = failures(sketch_errors(many, tree, sk), TOL["f64"])
    assert not bad, bad
    one.close()
    many.close()


def test_rank1_batched_empty_is_noop(P):
    plan = P.Plan(T4, (6, 7, 5, 4), 3, 2, variant="sttnn", dtype="f64", seed=2)
    plan.update_rank1_batched([], [])
    torch.cuda.synchronize()
    tree = O.Tree(T4, (6, 7, 5, 4), 3, 2)
    assert all(not np.any(s) for s in _sketches(P, plan, tree))
    plan.close()


# leaf maps of 16^5 rows over five factor positions of 16, plans in the grouped rank-1
# form: the two fastest positions contracted on the FP64 MFMA (4,096 blocks of 256
# rows; the maps of 65,536 rows of (1,2) and (5,6), 256 blocks, each block split over
# two workgroups); FP32 and BF16 maps,
# TTNN and STTNN (whose chained nodes' positions are the short contracted groups and
# take the other form), against the oracle on the same rounded maps at FP64 accuracy
MFMA_CASES = [("ttnn-f32", "ttnn", "f32"), ("sttnn-f32", "sttnn", "f32"), ("ttnn-bf16", "ttnn", "bf16")]


@pytest.mark.parametrize("m", [1, 16])
@pytest.mark.parametrize("name,variant,dtype", MFMA_CASES, ids=[c[0] for c in MFMA_CASES])
def test_rank1_mfma_form(P, name, variant, dtype, m):
    dims, r, p = (16,) * 6, 8, 4
    print(f"rank1 mfma {name} m={m}", flush=True)
    g = np.random.default_rng(60 + m)
    vecs = [[g.standard_normal(n) for n in dims] for _ in range(m)]
    alphas = [float(a) for a in g.uniform(-2, 2, size=m)]
    dev = [[torch.from_numpy(v).cuda() for v in term] for term in vecs]
    one = P.Plan(TOY, dims, r, p, variant=variant, dtype=dtype, seed=6)
    many = P.Plan(TOY, dims, r, p, variant=variant, dtype=dtype, seed=6)
    one.set_rank1_form("grouped")
    many.set_rank1_form("grouped")
    for term, a in zip(dev, alphas):
        one.update_rank1(term, alpha=a)
    many.update_rank1_batched(dev, alphas)
    torch.cuda.synchronize()
    tree = O.Tree(TOY, dims, r, p)
    for a, b in zip(_sketches(P, one, tree), _sketches(P, many, tree)):
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    T = np.zeros(dims)
    for term, a in zip(vecs, alphas):
        outer = term[0]
        for v in term[1:]:
            outer = np.multiply.outer(outer, v)
        T += a * outer
    sk = O.sketch(T, tree, O.DRMs(tree, 6, variant, dtype), variant)
    bad = failures(sketch_errors(many, tree, sk), 1e-10)
    assert not bad, bad
    one.close()
    many.close()
