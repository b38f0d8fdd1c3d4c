"""Streamed updates at full size on the order-5 serving shape: 64^5 on
(((1,2),3),(4,5)), r = 24, p = 12, FP32, delivered as the boxes of a random tiling of
the tensor plus a cancelling pair of rank-1 terms (the sketches are linear, Sec. 4,
so the sum of the update sketches is the sketch of the tensor).  Every sketch the plan
holds (R_t, Omega_t, Psi_t, root Psi) is compared element by element with the full
oracle sketch of the tensor, the oracle fed the same FP32-rounded DRMs, at the
arithmetic tolerance (FP32 tensor values, FP32 sums within a chunk, FP64 beyond)."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL_ARITH, failures, sketch_errors
from workloads import serving as WS
from workloads import synth as W

pytestmark = pytest.mark.gpu

DIMS, R, P_OVER, SEED = (64, 64, 64, 64, 64), 24, 12, 5


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    return P


@pytest.fixture(scope="module")
def tensor():
    """Seeded N(0,1) FP32 tensor on the device (flat, column-major) and the FP64 host
    copy of exactly those values, as a logical [i1, .., i5] array."""
    g = torch.Generator(device="cuda").manual_seed(123)
    n = int(np.prod(DIMS))
    dev = torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    host = dev.double().cpu().numpy().reshape(DIMS[::-1]).T
    return dev, host


def boxes_of(dev, offs_exts):
    """Device blocks (column-major copies) of the boxes of the flat tensor."""
    V = dev.view(*DIMS[::-1])                      # [i5, i4, i3, i2, i1]
    for off, ext in offs_exts:
        sl = tuple(slice(o, o + e) for o, e in zip(off[::-1], ext[::-1]))
        yield off, ext, V[sl].contiguous().reshape(-1)


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_stream64_parity(P, tensor, variant):
    dev, host = tensor
    print(f"order-5 streamed parity {variant}", flush=True)
    tree = O.Tree(O.T5, DIMS, R, P_OVER)
    plan = P.Plan(O.T5, DIMS, R, P_OVER, variant=variant, dtype="f32", seed=SEED)
    g = W.rng(31)
    bx = WS.boxes(DIMS, g, lo=24, hi=40)
    for off, ext, blk in boxes_of(dev, bx):
        plan.update(blk, extent=ext, offset=off)
    for fac, a in WS.rank1_pairs(DIMS, 1, seed=17):
        plan.update_rank1([torch.from_numpy(v).cuda() for v in fac], alpha=a)
    torch.cuda.synchronize()
    sk = O.sketch(host, tree, O.DRMs(tree, SEED, variant, "f32"), variant)
    errs = sketch_errors(plan, tree, sk)
    plan.close()
    bad = failures(errs, TOL_ARITH["f32"])
    assert not bad, bad
