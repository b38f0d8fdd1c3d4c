"""Trees with free modes on the GPU (Def. 3: a node may contain more than the union of
its children; each free mode behaves as a child with identity maps, projector and core),
through the C ABI, against the oracle:

* the tensor-train chain of Fig. 4 (orders 4 and 5), a free mode between two children,
  a free mode of the root; TTNN and STTNN; FP64 / FP32 / BF16: maps bit for bit, every
  sketch element by element (the dtype tolerances, and the rounded-map oracle at the
  arithmetic tolerance), the cores and the reconstruction in FP64;
* streaming: the boxes of a random tiling plus a cancelling pair of rank-1 terms
  against the oracle's whole-tensor sketch;
* exact recovery of a tensor of TT rank <= r.
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL, TOL_ARITH, errs2, failures, sketch_errors, to_device
from workloads import serving as WS
from workloads import synth as W

pytestmark = pytest.mark.gpu

TT4 = (((1, -2), -3), -4)
TT5 = ((((1, -2), -3), -4), -5)
MID = ((1, -2, 3), 4)
ROOTF = ((1, 2), -3, (4, 5))
CASES = [("tt4", TT4, (20, 24, 18, 22)), ("tt5", TT5, (9, 12, 10, 11, 8)),
         ("mid", MID, (20, 17, 24, 19)), ("rootf", ROOTF, (9, 10, 12, 11, 9))]


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    return P


def gpu_cores_by_modes(plan, cores):
    return {plan.node_modes[i]: c.cpu().numpy() for i, c in enumerate(cores)}


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name,spec,dims", CASES, ids=[c[0] for c in CASES])
def test_free_mode_parity(P, name, spec, dims, dtype, variant):
    r, p = 4, 2
    print(f"free modes {name} {variant} {dtype}", flush=True)
    T = np.random.default_rng(11).standard_normal(dims)
    dev, consumed = to_device(T, dtype)
    plan = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=3)
    plan.update(dev)
    tree = O.Tree(spec, dims, r, p)
    D = O.DRMs(tree, 3, variant)
    Dr = O.DRMs(tree, 3, variant, dtype)              # the one rounded map a plan of this dtype keeps
    for n in tree.nodes[1:]:                          # maps bit for bit
        cid = plan.node(n.modes)
        assert np.array_equal(plan.read_drm(cid, 0).cpu().numpy(), Dr.X[n.id])
        assert np.array_equal(plan.read_drm(cid, 1).cpu().numpy(), Dr.Y[n.id])
    sk = O.sketch(consumed, tree, D, variant)
    bad = failures(sketch_errors(plan, tree, sk), TOL[dtype])
    assert not bad, bad
    if dtype != "f64":
        skr = O.sketch(consumed, tree, Dr, variant)
        bad = failures(sketch_errors(plan, tree, skr), TOL_ARITH[dtype])
        assert not bad, bad
        return
    cores = plan.assemble()
    oc, _ = O.assemble(sk, tree)
    gc = gpu_cores_by_modes(plan, cores)
    for n in tree.nodes:
        want = oc[n.id].reshape(-1, order="F")
        e = errs2(gc[n.modes], want)
        assert e[0] <= 1e-10, (n.modes, e)
    That = plan.reconstruct(cores).cpu().numpy()
    ref = W.flat_colmajor(O.reconstruct(oc, tree))
    assert np.linalg.norm(That - ref) <= 1e-10 * np.linalg.norm(ref)
    plan.close()


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("name,spec,dims", CASES[1:3], ids=[c[0] for c in CASES[1:3]])
def test_free_mode_streaming(P, name, spec, dims, variant):
    """Boxes of a tiling, read in place, plus a cancelling pair of rank-1 terms: the
    oracle's sketch of the whole tensor (linearity, Sec. 4)."""
    r, p = 4, 2
    T = np.random.default_rng(12).standard_normal(dims)
    dev, consumed = to_device(T, "f64")
    V = dev.view(*dims[::-1])
    plan = P.Plan(spec, dims, r, p, variant=variant, dtype="f64", seed=5)
    for off, ext in WS.boxes(dims, W.rng(3), lo=2, hi=6):
        view = V[tuple(slice(o, o + e) for o, e in zip(off[::-1], ext[::-1]))]
        plan.update(view, extent=ext, offset=off)
    g = np.random.default_rng(13)
    fac = [torch.from_numpy(g.standard_normal(n)).cuda() for n in dims]
    plan.update_rank1(fac, alpha=0.75)
    plan.update_rank1(fac, alpha=-0.75)
    torch.cuda.synchronize()
    tree = O.Tree(spec, dims, r, p)
    sk = O.sketch(consumed, tree, O.DRMs(tree, 5, variant), variant)
    bad = failures(sketch_errors(plan, tree, sk), TOL["f64"])
    assert not bad, bad
    plan.close()


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
def test_free_mode_exact_recovery(P, variant):
    dims, s = (16, 12, 14, 10), 3
    g = np.random.default_rng(4)
    ranks = [1, s, s, s, 1]
    T = g.standard_normal((dims[0], s))
    for k in range(1, 4):
        T = np.tensordot(T, g.standard_normal((ranks[k], dims[k], ranks[k + 1])), axes=([T.ndim - 1], [0]))
    T = T.reshape(dims)
    dev, _ = to_device(T, "f64")
    plan = P.Plan(TT4, dims, 4, 2, variant=variant, dtype="f64", seed=9)
    plan.update(dev)
    That = plan.reconstruct(plan.assemble()).cpu().numpy()
    ref = W.flat_colmajor(T)
    assert np.linalg.norm(That - ref) <= 1e-10 * np.linalg.norm(ref)
    plan.close()
