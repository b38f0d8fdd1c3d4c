"""Streamed updates at full size on the order-5 serving shape: 64^5 on
(((1,2),3),(4,5)), r = 24, p = 12, FP32, delivered as the boxes of a random tiling of
the tensor plus a cancelling pair of rank-1 terms (the sketches are linear, Sec. 4,
so the sum of the update sketches is the sketch of the tensor).  Sampled entries of
the node sketches are checked against the oracle's one-entry evaluator of the tensor
(oracle.sampled) within the FP32 tolerance relative to the RMS entry of the GPU
sketch.  The oracle regenerates a whole DRM column per sampled entry (16.7M rows for
a leaf), so the samples are few: every internal node, and two leaves (TTNN) or one
(STTNN)."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.sampled import right_entry
from gpu_util import TOL
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


@pytest.mark.parametrize("variant,leaves", [("ttnn", 2), ("sttnn", 1)])
def test_stream64_sampled_parity(P, tensor, variant, leaves):
    dev, host = tensor
    tree = O.Tree(O.T5, DIMS, R, P_OVER)
    plan = P.Plan(O.T5, DIMS, R, P_OVER, variant=variant, dtype="f32", seed=SEED)
    g = W.rng(31)
    bx = WS.boxes(DIMS, g, lo=24, hi=40)
    for off, ext, blk in boxes_of(dev, bx):
        plan.update(blk, extent=ext, offset=off)
    for fac, a in WS.rank1_pairs(DIMS, 1, seed=17):
        plan.update_rank1([torch.from_numpy(v).cuda() for v in fac], alpha=a)
    torch.cuda.synchronize()

    internal = [n for n in tree.nodes[1:] if n.children]
    leaf = [n for n in tree.nodes[1:] if not n.children]
    picked = internal + [leaf[int(i)] for i in g.choice(len(leaf), leaves, replace=False)]
    worst = {}
    for n in picked:
        Rg = plan.read_sketch(plan.node(n.modes), P.SK_R).cpu().numpy()
        scale = np.sqrt(np.mean(Rg ** 2))
        ext = [DIMS[m - 1] for m in n.modes]
        j = int(g.integers(R))
        im = [int(g.integers(e)) for e in ext]
        i = int(np.ravel_multi_index(im, ext, order="F"))
        want = right_entry(host, tree, SEED, variant, n.id, im, j)
        worst[n.modes] = abs(Rg[i, j] - want) / scale
    plan.close()
    bad = {k: v for k, v in worst.items() if not v <= TOL["f32"]}
    assert not bad, (bad, worst)
