"""GPU tests of the streaming / serving path, through the C ABI.

* rank-1 updates: the sketches of a_1 o ... o a_d match the oracle's sketches of the
  dense outer product, the oracle fed the plan's (rounded) DRMs: the factors are FP64
  and every product and sum is FP64, so FP64 accuracy is asked of every dtype (the
  quantization of the maps themselves is not an error of the path; on these 2..9-wide
  modes it alone moves BF16 sketches by a few percent from FP64-map sketches);
* batched updates (ttnn_sketch_update_batched): bitwise equal to the same updates
  applied one by one, for plans of different sizes and boxes, with several updates
  of one plan in the same call;
* the serving loop: every stream's sketches are bitwise the same alone and in the
  mix, streams admitted under an HBM budget all finish, and the final sketches match
  the oracle's sketches of each stream's whole tensor.
"""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import serving as WS
from workloads import synth as W
from gpu_util import rel, failures, sketch_errors, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    assert torch.cuda.is_available()
    return P


def read_all(P, plan):
    """Every accumulator of a plan as float64 numpy arrays (for bitwise checks)."""
    out = {}
    for cid in range(plan.num_nodes):
        if plan.level_id(cid) == 0:
            out[(cid, "psi")] = plan.read_sketch(cid, P.SK_PSI).cpu().numpy()
        else:
            out[(cid, "R")] = plan.read_sketch(cid, P.SK_R).cpu().numpy()
    return out


def same_bits(a, b):
    return all(np.array_equal(a[k].view(np.uint64), b[k].view(np.uint64)) for k in a)


RANK1_CASES = [
    ("t4", O.T4, (9, 7, 6, 8), 4, 2),
    ("t5", O.T5, (5, 6, 4, 3, 5), 3, 2),
    ("toy", O.TOY, (3, 4, 3, 2, 3, 2), 2, 2),
]


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", RANK1_CASES, ids=lambda c: c[0])
def test_rank1_matches_oracle(P, case, variant, dtype):
    name, spec, dims, r, p = case
    g = W.rng(5)
    f = [g.standard_normal(n) for n in dims]
    plan = P.Plan(spec, dims, r, p, variant=variant, dtype=dtype, seed=3)
    plan.update_rank1([torch.from_numpy(v).cuda() for v in f], alpha=0.75)
    torch.cuda.synchronize()
    T = 0.75 * np.einsum(",".join("abcdefgh"[i] for i in range(len(dims))) + "->" + "abcdefgh"[:len(dims)], *f)
    tree = O.Tree(spec, dims, r, p)
    sk = O.sketch(T, tree, O.DRMs(tree, 3, variant, dtype), variant)
    errs = sketch_errors(plan, tree, sk)
    bad = failures(errs, 1e-10)
    assert not bad, bad
    plan.close()


def test_rank1_pairs_cancel_and_mix_with_boxes(P):
    """Boxes of a tiling plus cancelling rank-1 pairs add up to the sketch of the
    tensor (f64, STTNN)."""
    spec, dims, r, p = O.T4, (13, 11, 9, 10), 4, 3
    T = W.small_random_ttn(spec, dims, 3, seed=4, noise=1e-3)
    plan = P.Plan(spec, dims, r, p, variant="sttnn", dtype="f64", seed=2)
    g = W.rng(8)
    for off, ext in WS.boxes(dims, g, lo=3, hi=6):
        sl = tuple(slice(o, o + e) for o, e in zip(off, ext))
        blk, _ = to_device(T[sl], "f64")
        plan.update(blk, extent=ext, offset=off)
    for fac, a in WS.rank1_pairs(dims, 3, seed=9):
        plan.update_rank1([torch.from_numpy(v).cuda() for v in fac], alpha=a)
    torch.cuda.synchronize()
    tree = O.Tree(spec, dims, r, p)
    sk = O.sketch(T, tree, O.DRMs(tree, 2, "sttnn"), "sttnn")
    errs = sketch_errors(plan, tree, sk)
    assert not failures(errs, 1e-10), errs


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_batched_equals_sequential_bitwise(P, variant, dtype):
    spec = O.T4
    dims_list = [(17, 9, 12, 10), (9, 14, 8, 13), (20, 6, 7, 11)]
    g = W.rng(11)
    work = []            # (plan index, offset, extent, block)
    tensors = [W.small_random_ttn(spec, d, 3, seed=20 + i) for i, d in enumerate(dims_list)]
    for i, d in enumerate(dims_list):
        for off, ext in WS.boxes(d, g, lo=4, hi=9)[:5]:
            sl = tuple(slice(o, o + e) for o, e in zip(off, ext))
            blk, _ = to_device(tensors[i][sl], dtype)
            work.append((i, off, ext, blk))
    perm = g.permutation(len(work))
    work = [work[k] for k in perm]

    def plans():
        return [P.Plan(spec, d, 5, 3, variant=variant, dtype=dtype, seed=40 + i) for i, d in enumerate(dims_list)]

    seq = plans()
    for i, off, ext, blk in work:
        seq[i].update(blk, extent=ext, offset=off, alpha=0.5)
    bat = plans()
    P.update_batched([(bat[i], blk, ext, off, 0.5) for i, off, ext, blk in work])
    torch.cuda.synchronize()
    for a, b in zip(seq, bat):
        assert same_bits(read_all(P, a), read_all(P, b))


def _stream_updates(P, prob, T, dtype):
    ups = []
    for off, ext, blk in WS.box_updates(T, prob, lo=4, hi=12):
        dev, _ = to_device(T[tuple(slice(o, o + e) for o, e in zip(off, ext))], dtype)
        ups.append((off, ext, dev))
    return ups


def test_serving_alone_vs_mix_bitwise(P):
    from paper_2412_06111_amd import serve as S
    dtype = "f32"
    probs = [WS.stream_problem(s, nlo=14, nhi=26, rlo=2, rhi=5, ranks=(4, 6)) for s in range(4)]
    tens = [WS.stream_tensor(pr) for pr in probs]
    ups = [_stream_updates(P, pr, T, dtype) for pr, T in zip(probs, tens)]
    specs = [S.StreamSpec(O.T4, pr["dims"], pr["r"], pr["p"], variant="sttnn", dtype=dtype, seed=pr["seed"])
             for pr in probs]

    # mixed: all streams through the batching server (budget fits them all)
    srv = S.Server(budget_bytes=1 << 40, max_batch=8, keep_plans=True)
    arrivals = []
    for s, u in enumerate(ups):
        srv.open_stream(s, specs[s])
        for k, (off, ext, dev) in enumerate(u):
            arrivals.append(S.Update(s, "box", block=dev, offset=off, extent=ext, arrival=0.0))
    st = srv.run(arrivals)
    assert st["updates"] == sum(len(u) for u in ups)
    assert max(srv.batches) > 1
    mixed = {s: read_all(P, srv.plans[s]) for s in range(4)}

    # alone: one plan per stream, updates one by one in the same order
    for s, u in enumerate(ups):
        plan = P.Plan(O.T4, probs[s]["dims"], probs[s]["r"], probs[s]["p"], variant="sttnn", dtype=dtype,
                      seed=probs[s]["seed"])
        for off, ext, dev in u:
            plan.update(dev, extent=ext, offset=off)
        torch.cuda.synchronize()
        assert same_bits(read_all(P, plan), mixed[s]), s
        plan.close()


def test_serving_budget_admission_and_parity(P):
    from paper_2412_06111_amd import serve as S
    dtype = "f32"
    probs = [WS.stream_problem(s, nlo=16, nhi=30, rlo=2, rhi=5, ranks=(4, 6)) for s in range(5)]
    tens = [WS.stream_tensor(pr) for pr in probs]
    specs = [S.StreamSpec(O.T4, pr["dims"], pr["r"], pr["p"], variant="ttnn", dtype=dtype, seed=pr["seed"])
             for pr in probs]
    fps = [P.footprint_estimate(sp.spec, sp.dims, sp.rank, sp.over, sp.variant, sp.dtype) for sp in specs]
    budget = max(fps) + sum(sorted(fps)[:1])          # about two streams at a time
    recon = {}

    def on_close(sid, plan, cores):
        recon[sid] = plan.reconstruct(cores).cpu().numpy()

    srv = S.Server(budget_bytes=budget, max_batch=8, keep_plans=False, on_close=on_close)
    arrivals = []
    times = WS.poisson_arrivals(10_000, 2000.0, seed=3)
    k = 0
    for s, (pr, T) in enumerate(zip(probs, tens)):
        srv.open_stream(s, specs[s])
        for off, ext, dev in _stream_updates(P, pr, T, dtype):
            arrivals.append(S.Update(s, "box", block=dev, offset=off, extent=ext, arrival=float(times[k]),
                                     nbytes=dev.numel() * 4))
            k += 1
    arrivals.sort(key=lambda u: u.arrival)
    st = srv.run(arrivals)
    assert st["updates"] == len(arrivals)
    assert st["p99_ms"] >= st["p50_ms"] > 0
    assert srv.used == 0 and not srv.streams
    assert len(srv.closed) == 5
    # admission in arrival order, and the admitted footprint never exceeded the budget
    assert srv.admit_order == list(range(5))
    assert 0 < st["peak_used_bytes"] <= budget and srv.peak_used <= budget
    # final cores of every stream reconstruct its tensor like the oracle's cores do
    for s, (pr, T) in enumerate(zip(probs, tens)):
        tree = O.Tree(O.T4, pr["dims"], pr["r"], pr["p"])
        sk = O.sketch(T, tree, O.DRMs(tree, pr["seed"], "ttnn"), "ttnn")
        oc, _ = O.assemble(sk, tree)
        want = O.reconstruct(oc, tree)
        e_gpu = rel(recon[s], W.flat_colmajor(T))
        e_orc = rel(W.flat_colmajor(want), W.flat_colmajor(T))
        assert abs(e_gpu - e_orc) <= 0.1 * e_orc + 1e-6, (s, e_gpu, e_orc)


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_persistent_round_equals_per_level_launches(P, variant, dtype):
    """With TTNN_PERSISTENT=1 a batched round runs as one persistent cooperative launch
    (every level's contractions, folds and reductions, grid-wide barriers between them);
    by default the same tiles run as one launch per level and kind.  The two must agree
    bit for bit, for plans of different sizes and several rounds per call."""
    import os
    spec = O.T5 if variant == "sttnn" else O.T4
    dims_list = [(9, 8, 7, 6, 5), (6, 9, 5, 8, 7)] if variant == "sttnn" else [(17, 9, 12, 10), (9, 14, 8, 13)]
    tensors = [W.small_random_ttn(spec, d, 3, seed=40 + i) for i, d in enumerate(dims_list)]
    g = W.rng(19)
    work = []
    for i, d in enumerate(dims_list):
        for off, ext in WS.boxes(d, g, lo=2, hi=5)[:12]:
            blk, _ = to_device(tensors[i][tuple(slice(o, o + e) for o, e in zip(off, ext))], dtype)
            work.append((i, off, ext, blk))
    results = []
    for persistent in ("1", "0"):
        os.environ["TTNN_PERSISTENT"] = persistent
        try:
            plans = [P.Plan(spec, d, 4, 2, variant=variant, dtype=dtype, seed=3) for d in dims_list]
            P.update_batched([(plans[i], blk, ext, off, 0.5 + i) for i, off, ext, blk in work])
            torch.cuda.synchronize()
            results.append([read_all(P, pl) for pl in plans])
            for pl in plans:
                pl.close()
        finally:
            del os.environ["TTNN_PERSISTENT"]
    for a, b in zip(*results):
        assert same_bits(a, b)
