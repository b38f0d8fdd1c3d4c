"""The measurement hook (ttnn_set_timing): events around the sweep of a whole-tensor
update, from which the side stream of the Z1-writing form also forks.  With timing on,
every sketch is bitwise the same as with timing off, over two updates in a row, and the
sweep time is positive; the one-pass forms are the ones the bench times (STTNN writing
Z1, TTNN mode)."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

DIMS = (128, 32, 64, 64)          # 16.8M entries: the one-pass kernel with n_1 = 128


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    assert torch.cuda.is_available()
    return P


def sketches(P, plan, tree):
    out = []
    for n in tree.nodes:
        for kind in ((P.SK_R, P.SK_OMEGA, P.SK_PSI) if n.id else (P.SK_PSI,)):
            out.append(plan.read_sketch(plan.node(n.modes), kind).cpu().numpy())
    return out


@pytest.mark.parametrize("variant,kind", [("sttnn", 2), ("ttnn", 3)])
def test_timing_leaves_results_bitwise(P, variant, kind):
    print(f"timing {variant}", flush=True)
    g = torch.Generator(device="cuda").manual_seed(5)
    T = torch.randn(int(np.prod(DIMS)), generator=g, device="cuda", dtype=torch.float32)
    tree = O.Tree(O.T4, DIMS, 32, 16)
    res = {}
    for timed in (False, True):
        plan = P.Plan(O.T4, DIMS, 32, 16, variant=variant, dtype="f32", seed=4)
        plan.set_timing(timed)
        plan.update(T)
        plan.update(T, alpha=-0.25)
        assert plan.sweep_kind() == kind
        if timed:
            ms = plan.sweep_time_ms()
            assert np.isfinite(ms) and ms > 0.0, ms
        res[timed] = sketches(P, plan, tree)
        plan.close()
    for a, b in zip(res[False], res[True]):
        assert np.array_equal(a, b)
