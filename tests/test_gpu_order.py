"""STTNN in non-lexicographic visiting orders on the GPU (Sec. 5: the order of the
nodes is free; node t reuses the contractions of the siblings visited before it and
before each of its ancestors), through the C ABI, against the oracle in the same order:

* several trees and orders (contracted groups on both sides of a node, a free mode);
  FP64 / FP32 / BF16: maps bit for bit (their shapes follow the order), the reuse sets,
  every sketch element by element (the dtype tolerances, and the rounded-map oracle at
  the arithmetic tolerance), the cores and the reconstruction in FP64;
* streaming: the boxes of a tiling plus a cancelling pair of rank-1 terms against the
  oracle's whole-tensor sketch;
* whole tensors large enough for the MFMA and batched paths (((1,2),(3,4)) with
  n_1 << n_2, in the order the search picks; the 6-D Hilbert tensor of the paper on the
  tree of Fig. 1 in its searched order): sampled entries of every R_t against the
  one-entry oracle, and the accuracy of the approximation.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.sampled import right_entry, root_entry
from gpu_util import TOL, TOL_ARITH, errs2, failures, sketch_errors, to_device
from workloads import hilbert as H
from workloads import serving as WS
from workloads import synth as W

pytestmark = pytest.mark.gpu

T4 = ((1, 2), (3, 4))
TOY = (((1, 2), 3), 4, (5, 6))
T5 = (((1, 2), 3), (4, 5))
FREE = (((1, -2), 3), -4, (5, 6))
CASES = [("t4-a", T4, ((2, 1), (3, 4)), (12, 40, 10, 9)),
         ("t4-rev", T4, ((4, 3), (2, 1)), (9, 14, 11, 13)),
         ("toy", TOY, ((5, 6), (3, (1, 2)), 4), (5, 4, 6, 3, 5, 4)),
         ("t5", T5, ((4, 5), (3, (2, 1))), (8, 11, 6, 9, 7)),
         ("free", FREE, ((5, 6), (3, (1, -2)), -4), (5, 4, 6, 3, 5, 4))]


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("name,spec,visit,dims", CASES, ids=[c[0] for c in CASES])
def test_order_parity(P, name, spec, visit, dims, dtype):
    r, p = 4, 2
    print(f"order {name} {dtype}", flush=True)
    T = np.random.default_rng(21).standard_normal(dims)
    dev, consumed = to_device(T, dtype)
    plan = P.Plan(spec, dims, r, p, variant="sttnn", dtype=dtype, seed=3, visit=visit)
    plan.update(dev)
    tree = O.Tree(spec, dims, r, p, visit=visit)
    D = O.DRMs(tree, 3, "sttnn")
    Dr = O.DRMs(tree, 3, "sttnn", dtype)
    for n in tree.nodes[1:]:
        cid = plan.node(n.modes)
        assert sorted(plan.node_modes[c] for c in plan.reuse_set(cid)) == sorted(tree[s].modes for s in tree.S(n.id))
        assert np.array_equal(plan.read_drm(cid, 0).cpu().numpy(), Dr.X[n.id])
        assert np.array_equal(plan.read_drm(cid, 1).cpu().numpy(), Dr.Y[n.id])
    sk = O.sketch(consumed, tree, D, "sttnn")
    bad = failures(sketch_errors(plan, tree, sk), TOL[dtype])
    assert not bad, bad
    if dtype != "f64":
        skr = O.sketch(consumed, tree, Dr, "sttnn")
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


@pytest.mark.parametrize("name,spec,visit,dims", [CASES[1], CASES[2], CASES[4]], ids=["t4-rev", "toy", "free"])
def test_order_streaming(P, name, spec, visit, dims):
    """Boxes of a tiling, read in place, plus a cancelling pair of rank-1 terms: the
    oracle's sketch of the whole tensor (linearity, Sec. 4)."""
    r, p = 4, 2
    T = np.random.default_rng(22).standard_normal(dims)
    dev, consumed = to_device(T, "f64")
    V = dev.view(*dims[::-1])
    plan = P.Plan(spec, dims, r, p, variant="sttnn", dtype="f64", seed=5, visit=visit)
    for off, ext in WS.boxes(dims, W.rng(4), lo=2, hi=6):
        view = V[tuple(slice(o, o + e) for o, e in zip(off[::-1], ext[::-1]))]
        plan.update(view, extent=ext, offset=off)
    g = np.random.default_rng(23)
    fac = [torch.from_numpy(g.standard_normal(n)).cuda() for n in dims]
    plan.update_rank1(fac, alpha=0.5)
    plan.update_rank1(fac, alpha=-0.5)
    torch.cuda.synchronize()
    tree = O.Tree(spec, dims, r, p, visit=visit)
    sk = O.sketch(consumed, tree, O.DRMs(tree, 5, "sttnn"), "sttnn")
    bad = failures(sketch_errors(plan, tree, sk), TOL["f64"])
    assert not bad, bad
    plan.close()


def test_rank1_in_order(P):
    """A rank-1 update alone equals the oracle's sketch of the outer product."""
    spec, visit, dims = CASES[3][1:]
    g = np.random.default_rng(24)
    vecs = [g.standard_normal(n) for n in dims]
    T = vecs[0]
    for v in vecs[1:]:
        T = np.multiply.outer(T, v)
    plan = P.Plan(spec, dims, 4, 2, variant="sttnn", dtype="f64", seed=6, visit=visit)
    plan.update_rank1([torch.from_numpy(v).cuda() for v in vecs], alpha=1.25)
    tree = O.Tree(spec, dims, 4, 2, visit=visit)
    sk = O.sketch(1.25 * T, tree, O.DRMs(tree, 6, "sttnn"), "sttnn")
    bad = failures(sketch_errors(plan, tree, sk), TOL["f64"])
    assert not bad, bad
    plan.close()


# first contraction of the chain at mode 2 of the raw tensor with L = n_1 > 1: the
# streaming MFMA mode product (at least 32768 rows L Q; rows, contraction and columns
# ragged against its 128-row tiles, 32 / 16-value steps and 16-column blocks)
MID = [("f32-ragged", (8, 20, 70, 59), 9, 4, "f32"), ("f32-wide", (8, 16, 64, 64), 30, 10, "f32"),
       ("f64-l2", (2, 12, 128, 160), 9, 4, "f64"), ("f64-ragged", (4, 37, 90, 100), 20, 8, "f64")]


@pytest.mark.parametrize("name,dims,r,p,dtype", MID, ids=[c[0] for c in MID])
def test_order_mode_product_at_mode2(P, name, dims, r, p, dtype):
    visit = ((2, 1), (3, 4))
    print(f"order mid {name}", flush=True)
    T = np.random.default_rng(27).standard_normal(dims)
    dev, consumed = to_device(T, dtype)
    plan = P.Plan(T4, dims, r, p, variant="sttnn", dtype=dtype, seed=8, visit=visit)
    plan.update(dev)
    tree = O.Tree(T4, dims, r, p, visit=visit)
    sk = O.sketch(consumed, tree, O.DRMs(tree, 8, "sttnn", dtype), "sttnn")
    bad = failures(sketch_errors(plan, tree, sk), TOL_ARITH[dtype])
    assert not bad, bad
    plan.close()


def _sampled(P, plan, host, tree, seed, tol, g, per_node=3):
    worst = {}
    for t in tree.nodes[1:]:
        Rg = plan.read_sketch(plan.node(t.modes), P.SK_R).cpu().numpy()
        scale = np.sqrt(np.mean(Rg ** 2))
        ext = [tree.dims[m - 1] for m in t.modes]
        for _ in range(per_node):
            im = [int(g.integers(e)) for e in ext]
            j = int(g.integers(t.rank))
            i = int(np.ravel_multi_index(im, ext, order="F"))
            want = right_entry(host, tree, seed, "sttnn", t.id, im, j)
            worst[t.modes] = max(worst.get(t.modes, 0.0), abs(Rg[i, j] - want) / scale)
    psi = plan.read_sketch(plan.node(tree[0].modes), P.SK_PSI).cpu().numpy()
    kk = [tree[c].k for c in tree[0].children]
    for _ in range(per_node):
        km = [int(g.integers(k)) for k in kk]
        want = root_entry(host, tree, seed, km)
        got = psi[int(np.ravel_multi_index(km, kk, order="F"))]
        worst["root"] = max(worst.get("root", 0.0), abs(got - want) / np.sqrt(np.mean(psi ** 2)))
    return {k: v for k, v in worst.items() if not v <= tol}, worst


def test_order_large_unbalanced(P):
    """((1,2),(3,4)) with n_1 = 32 << n_2 = 512, FP32, 268M entries (the benchmark's
    visiting-order workload, in its launch configuration), in the searched order (mode 2
    before mode 1: the lexicographic X_1 would hold as many entries as the tensor): the
    MFMA right sketches, the streaming mode product at mode 2 and the batched FP64 jobs,
    sampled against the one-entry oracle."""
    dims, r, p, seed = (32, 512, 128, 128), 32, 16, 7
    visit, _ = P.order_search(T4, dims, r, p)
    assert visit == ((2, 1), (3, 4))
    print("order large t4 f32", flush=True)
    g = np.random.default_rng(25)
    host = g.standard_normal(dims, dtype=np.float32).astype(np.float64)
    dev = torch.from_numpy(np.ascontiguousarray(W.flat_colmajor(host)).astype(np.float32)).cuda()
    plan = P.Plan(T4, dims, r, p, variant="sttnn", dtype="f32", seed=seed, visit=visit)
    plan.update(dev)
    torch.cuda.synchronize()
    tree = O.Tree(T4, dims, r, p, visit=visit)
    bad, worst = _sampled(P, plan, host, tree, seed, TOL["f32"], g)
    plan.close()
    assert not bad, (bad, worst)


def test_order_hilbert_full_size(P):
    """The 6-D Hilbert tensor (n = 20, 64M entries) on the tree of Fig. 1 in its searched
    order at r = 13 (the benchmark's configuration): sampled sketch entries against the
    one-entry oracle, and the accuracy of the approximation in both orders."""
    n, r, seed = H.N_PAPER, 13, 5
    dims = (n,) * 6
    visit, _ = P.order_search(H.TOY, dims, r, H.P_PAPER)
    assert visit != H.TOY
    print(f"order hilbert {visit}", flush=True)
    dev = H.hilbert_device(n)
    host = H.hilbert_host(n)
    errs = {}
    for v in (visit, None):
        plan = P.Plan(H.TOY, dims, r, H.P_PAPER, variant="sttnn", dtype="f64", seed=seed, visit=v)
        plan.update(dev)
        e2, n2 = P.diff_norms(plan.reconstruct(plan.assemble()), dev)
        errs[v] = np.sqrt(e2 / n2)
        if v is not None:
            tree = O.Tree(H.TOY, dims, r, H.P_PAPER, visit=v)
            bad, worst = _sampled(P, plan, host, tree, seed, TOL["f64"], np.random.default_rng(26), per_node=2)
            assert not bad, (bad, worst)
        plan.close()
    # at r = 13 both orders reach the tensor's FP64 floor (the oracle gives ~1e-12)
    assert errs[visit] < 1e-10 and errs[None] < 1e-10, errs
