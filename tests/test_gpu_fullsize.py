"""Parity at the full benchmark size (128^4 on ((1,2),(3,4)), r = 32, p = 16), in the
launch configuration the benchmark times (one whole-tensor update: the fused sweep,
plus the MFMA right sketches for TTNN), on sampled outputs that the oracle evaluates
one at a time (oracle.sampled).  Each sampled entry of R_t and of the root sketch
must agree within the dtype tolerance relative to the RMS entry of the GPU result."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.sampled import right_entry, root_entry
from gpu_util import TOL, to_device

pytestmark = pytest.mark.gpu

DIMS, R, P_OVER, SEED = (128, 128, 128, 128), 32, 16, 1


@pytest.fixture(scope="module")
def T():
    # logical T[i1, i2, i3, i4] stored column-major (mode 1 fastest)
    return np.random.default_rng(0).standard_normal(DIMS[::-1]).T


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    return P


_DEV = {}


def device_copy(T, dtype):
    """The tensor on the device in `dtype` and the values it holds (one dtype kept)."""
    if dtype not in _DEV:
        _DEV.clear()
        _DEV[dtype] = to_device(T, dtype)
    return _DEV[dtype]


@pytest.mark.parametrize("variant", ["sttnn", "ttnn"])
@pytest.mark.parametrize("dtype", ["bf16", "f32", "f64"])
def test_fullsize_sampled_parity(P, T, variant, dtype):
    dev, consumed = device_copy(T, dtype)
    plan = P.Plan(O.T4, DIMS, R, P_OVER, variant=variant, dtype=dtype, seed=SEED)
    plan.update(dev)
    torch.cuda.synchronize()
    tree = O.Tree(O.T4, DIMS, R, P_OVER)
    g = np.random.default_rng(7)
    worst = {}
    for n in tree.nodes[1:]:
        Rg = plan.read_sketch(plan.node(n.modes), P.SK_R).cpu().numpy()
        scale = np.sqrt(np.mean(Rg ** 2))
        ext = [DIMS[m - 1] for m in n.modes]
        for j in g.choice(R, 2, replace=False):
            for _ in range(2):
                im = [int(g.integers(e)) for e in ext]
                i = int(np.ravel_multi_index(im, ext, order="F"))
                want = right_entry(consumed, tree, SEED, variant, n.id, im, int(j))
                err = abs(Rg[i, j] - want) / scale
                worst[n.modes] = max(worst.get(n.modes, 0.0), err)
    psi = plan.read_sketch(plan.node(tree[0].modes), P.SK_PSI).cpu().numpy()
    scale = np.sqrt(np.mean(psi ** 2))
    kk = [tree[c].k for c in tree[0].children]
    for _ in range(3):
        km = [int(g.integers(k)) for k in kk]
        want = root_entry(consumed, tree, SEED, km)
        err = abs(psi[int(np.ravel_multi_index(km, kk, order="F"))] - want) / scale
        worst["root"] = max(worst.get("root", 0.0), err)
    plan.close()
    bad = {k: v for k, v in worst.items() if not v <= TOL[dtype]}
    assert not bad, (bad, worst)
