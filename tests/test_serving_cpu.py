"""Scheduling rules of the serving loop and the serving workload generator, on the
CPU (a stand-in engine records what the server asks the device to do)."""
import numpy as np
import pytest

from paper_2412_06111_amd import serve as S
from workloads import serving as WS


class FakeEngine:
    """Records launches; an event completes after it has been polled `lag` times
    (or waited for)."""

    def __init__(self, footprints, lag=1):
        self.fp = footprints
        self.lag = lag
        self.launches = []
        self.live = set()
        self.peak_live = 0
        self.assembled = []
        self.n_ev = 0
        self.clock = 0.0

    def footprint(self, spec):
        return self.fp[spec.seed]

    def create(self, spec):
        h = ("plan", spec.seed)
        self.live.add(h)
        self.peak_live = max(self.peak_live, sum(self.fp[x[1]] for x in self.live))
        return h

    def launch(self, items):
        plans = [p for p, _ in items]
        assert len(plans) == len(set(plans)), "two updates of one plan in a batch"
        self.launches.append([(p[1], u) for p, u in items])

    def assemble(self, plan):
        self.assembled.append(plan[1])
        return ("cores", plan[1])

    assemble_async = assemble

    def status_async(self, plan):
        return 0

    def status_value(self, h):
        return h

    def destroy(self, plan):
        self.live.remove(plan)

    def event(self):
        self.n_ev += 1
        return {"id": self.n_ev, "polls": 0}

    def done(self, ev):
        ev["polls"] += 1
        return ev["polls"] > self.lag

    def wait(self, ev):
        ev["polls"] = self.lag + 1

    def elapsed_ms(self, a, b):
        return 1.0 + b["id"]

    def sync(self):
        pass


def spec(seed):
    return S.StreamSpec(((1, 2), (3, 4)), (8, 8, 8, 8), 4, 2, seed=seed)


def test_admission_respects_budget_and_frees_memory():
    fp = {0: 60, 1: 50, 2: 30, 3: 70}
    eng = FakeEngine(fp)
    srv = S.Server(budget_bytes=100, max_batch=4, engine=eng)
    for s in range(4):
        srv.open_stream(s, spec(s))
    arr = []
    for s in range(4):
        for k in range(3):
            arr.append(S.Update(s, arrival=0.0, nbytes=10))
    st = srv.run(arr)
    assert eng.peak_live <= 100
    assert st["peak_used_bytes"] == srv.peak_used <= 100 and srv.peak_used >= 60
    assert srv.admit_order == [0, 1, 2, 3]          # FIFO admission
    assert st["wait_p99_ms"] >= 0 and st["gpu_p99_ms"] >= 0
    assert sorted(eng.assembled) == [0, 1, 2, 3]
    assert srv.used == 0 and not eng.live
    assert len(srv.completed) == 12


def test_batches_one_update_per_stream_in_order():
    fp = {s: 1 for s in range(5)}
    eng = FakeEngine(fp, lag=2)
    srv = S.Server(budget_bytes=10, max_batch=3, max_inflight=2, engine=eng)
    for s in range(5):
        srv.open_stream(s, spec(s))
    arr = [S.Update(s, arrival=0.0) for k in range(4) for s in range(5)]
    for i, u in enumerate(arr):
        u.offset = i                                   # submission order tag
    srv.run(arr)
    assert all(len(b) <= 3 for b in eng.launches)
    seen = {}
    for b in eng.launches:
        for sid, u in b:
            assert seen.get(sid, -1) < u.offset        # per-stream order preserved
            seen[sid] = u.offset
    assert sum(len(b) for b in eng.launches) == 20
    assert max(len(b) for b in eng.launches) == 3


def test_oversized_stream_rejected():
    eng = FakeEngine({0: 500})
    srv = S.Server(budget_bytes=100, engine=eng)
    with pytest.raises(ValueError):
        srv.open_stream(0, spec(0))


def test_assemble_every():
    eng = FakeEngine({0: 1})
    srv = S.Server(budget_bytes=10, assemble_every=2, engine=eng)
    srv.open_stream(0, spec(0))
    srv.run([S.Update(0, arrival=0.0) for _ in range(5)])
    assert eng.assembled == [0, 0, 0]                   # after 2, after 4, at close


def test_stats_percentiles():
    ups = []
    for i in range(100):
        u = S.Update(0, arrival=0.0, nbytes=1000)
        u.t_done = (i + 1) * 1e-3
        ups.append(u)
    st = S.stats(ups, 1.0)
    assert st["updates"] == 100 and abs(st["p50_ms"] - 50.5) < 1e-9 and st["p99_ms"] > 99
    assert st["ingest_GBps"] == pytest.approx(1e-4)


def test_tiling_and_boxes_partition_the_tensor():
    g = np.random.default_rng(0)
    for n in (4, 30, 49, 160):
        segs = WS.tiling(n, g)
        assert sum(segs) == n and all(s >= 1 for s in segs)
        assert all(4 <= s <= 48 for s in segs[:-1])
    dims = (17, 23, 9, 30)
    cover = np.zeros(dims, dtype=int)
    for off, ext in WS.boxes(dims, np.random.default_rng(1), lo=3, hi=8):
        cover[tuple(slice(o, o + e) for o, e in zip(off, ext))] += 1
    assert (cover == 1).all()


def test_stream_problem_ranges():
    for s in range(20):
        pr = WS.stream_problem(s)
        assert all(32 <= n <= 160 for n in pr["dims"])
        assert pr["r"] in (16, 32) and pr["p"] == pr["r"] // 2
        for m, r in pr["ttn_ranks"].items():
            assert 1 <= r <= 32


def test_rank1_pairs_cancel():
    pairs = WS.rank1_pairs((3, 4, 5), 2, seed=1)
    assert len(pairs) == 4
    for (f1, a1), (f2, a2) in zip(pairs[0::2], pairs[1::2]):
        assert a1 == -a2 and all(np.array_equal(x, y) for x, y in zip(f1, f2))


def test_order5_tensor_matches_dense_ttn():
    """The order-5 serving tensor built by the device contraction (run here on the
    CPU) equals the einsum contraction of the same seeded cores, scaled to unit RMS."""
    from workloads import synth as W
    n, rank, seed = 5, 3, 11
    flat = WS.order5_tensor_device(n=n, rank=rank, seed=seed, noise=0.0, device="cpu").numpy()
    dims = (n,) * 5
    T = W.ttn_dense(WS.T5, dims, W.gaussian_ttn_cores(WS.T5, dims, rank, seed))
    ref = np.asarray(W.flat_colmajor(T), dtype=np.float64)
    ref = ref * np.sqrt(ref.size) / np.linalg.norm(ref)
    assert flat.shape == ref.shape
    assert np.allclose(flat, ref, rtol=1e-12, atol=1e-12)


def _group_sizes(eng):
    out = []
    for b in eng.launches:
        for _, u in b:
            out.append(len(u.group) if u.group else 1)
    return out


def _flat_order(eng):
    out = []
    for b in eng.launches:
        for _, u in b:
            out += [x.offset for x in (u.group or [u])]
    return out


def test_rank1_updates_grouped_in_order():
    """Consecutive queued rank-1 updates of a stream go out as one group (at most
    rank1_batch, boxes never grouped), in submission order."""
    eng = FakeEngine({0: 1})
    srv = S.Server(budget_bytes=10, engine=eng, rank1_batch=4)
    srv.open_stream(0, spec(0))
    kinds = ["box", "rank1", "rank1", "rank1", "box"] + ["rank1"] * 10
    arr = [S.Update(0, kind=k, arrival=0.0) for k in kinds]
    for i, u in enumerate(arr):
        u.offset = i
    srv.run(arr)
    assert _group_sizes(eng) == [1, 3, 1, 4, 4, 2]
    assert _flat_order(eng) == list(range(len(kinds)))
    assert len(srv.completed) == len(kinds)


def test_rank1_groups_stop_at_assembly_points():
    """A group never crosses a point where the cores are assembled, so the cores after
    k updates hold exactly the first k."""
    eng = FakeEngine({0: 1})
    srv = S.Server(budget_bytes=10, engine=eng, rank1_batch=4, assemble_every=5)
    srv.open_stream(0, spec(0))
    kinds = ["box", "rank1", "rank1", "rank1", "box"] + ["rank1"] * 10
    arr = [S.Update(0, kind=k, arrival=0.0) for k in kinds]
    for i, u in enumerate(arr):
        u.offset = i
    srv.run(arr)
    assert _group_sizes(eng) == [1, 3, 1, 4, 1, 4, 1]
    assert eng.assembled == [0, 0, 0, 0]               # after 5, 10, 15, and at close
    assert _flat_order(eng) == list(range(len(kinds)))


def test_rank1_batch_one_launches_singly():
    eng = FakeEngine({0: 1})
    srv = S.Server(budget_bytes=10, engine=eng, rank1_batch=1)
    srv.open_stream(0, spec(0))
    srv.run([S.Update(0, kind="rank1", arrival=0.0) for _ in range(5)])
    assert _group_sizes(eng) == [1] * 5
