"""The boundary through the C ABI: plans built in a caller-owned workspace (ttnn_plan)
against plans from the library's pool (ttnn_plan_create), and box updates read in place
from strided views of a resident tensor against packed copies of the same boxes (single
and batched calls).  The arithmetic and its order do not depend on where the plan lives
or on how the block is addressed, so the results must agree bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL, failures, sketch_errors, to_device
from workloads import serving as WS
from workloads import synth as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    return P


def read_all(P, plan, tree):
    out = []
    for n in tree.nodes:
        for kind in ((P.SK_R, P.SK_OMEGA, P.SK_PSI) if n.id else (P.SK_PSI,)):
            out.append(plan.read_sketch(plan.node(n.modes), kind).cpu())
    return out


def same_bits(a, b):
    return all(torch.equal(x.view(torch.int64), y.view(torch.int64)) for x, y in zip(a, b))


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_workspace_plan_equals_pool_plan(P, variant, dtype):
    spec, dims = O.T4, (128, 16, 12, 20)             # large enough for the one-pass kernel
    T = W.small_random_ttn(spec, dims, 4, seed=3, noise=1e-2)
    dev, consumed = to_device(T, dtype)
    tree = O.Tree(spec, dims, 16, 8)
    ws = torch.empty(P.workspace_bytes(spec, dims, 16, 8, variant, dtype), dtype=torch.uint8, device="cuda")
    a = P.Plan(spec, dims, 16, 8, variant=variant, dtype=dtype, seed=6, workspace=ws)
    b = P.Plan(spec, dims, 16, 8, variant=variant, dtype=dtype, seed=6, pool=True)
    assert a.footprint() == b.footprint() == ws.numel()
    for pl in (a, b):
        pl.update(dev)
    assert same_bits(read_all(P, a, tree), read_all(P, b, tree))
    ca, cb = a.assemble(), b.assemble()
    assert all(torch.equal(x, y) for x, y in zip(ca, cb))
    sk = O.sketch(consumed, tree, O.DRMs(tree, 6, variant), variant)
    assert not failures(sketch_errors(a, tree, sk), TOL[dtype])
    a.close()
    b.close()
    del ws


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_strided_boxes_equal_packed_boxes(P, variant, dtype):
    """Boxes of a random tiling given as views of the resident tensor (read in place
    with their strides) give bitwise the sketches of the same boxes copied packed, one
    by one and batched; a whole tensor that is itself a strided view (a slice of a
    larger array) matches the packed whole tensor within the dtype tolerance (it takes
    the generic kernels, the packed one the one-pass kernels)."""
    spec, dims, r, p = O.T5, (9, 12, 7, 10, 8), 4, 2
    T = np.random.default_rng(6).standard_normal(dims)
    dev, consumed = to_device(T, dtype)
    V = dev.view(*dims[::-1])                                 # [i5, .., i1]
    bx = WS.boxes(dims, W.rng(4), lo=2, hi=5)
    packed = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=2)
    strided = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=2)
    batched = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=2)
    items = []
    for off, ext in bx:
        view = V[tuple(slice(o, o + e) for o, e in zip(off[::-1], ext[::-1]))]
        packed.update(view.contiguous().reshape(-1), extent=ext, offset=off, alpha=0.5)
        strided.update(view, extent=ext, offset=off, alpha=0.5)
        items.append((batched, view, ext, off, 0.5))
    P.update_batched(items)
    torch.cuda.synchronize()
    tree = O.Tree(spec, dims, r, p)
    want = read_all(P, packed, tree)
    assert same_bits(read_all(P, strided, tree), want)
    assert same_bits(read_all(P, batched, tree), want)
    # the whole tensor as a slice of a larger array (every mode strided)
    big = torch.zeros(dims[4] + 1, dims[3] + 2, dims[2] + 1, dims[1] + 3, dims[0] + 2, dtype=dev.dtype, device="cuda")
    big[1:, 2:, 1:, 3:, 2:] = V
    whole = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=2)
    whole.update(big[1:, 2:, 1:, 3:, 2:])
    sk = O.sketch(consumed, tree, O.DRMs(tree, 2, variant), variant)
    assert not failures(sketch_errors(whole, tree, sk), TOL[dtype])
    for pl in (packed, strided, batched, whole):
        pl.close()
