"""Continuous-batching serving loop for streamed sketch updates.

Sketches are linear in the tensor (Sec. 4: the sketches of a sum of updates are the
sums of their sketches), so a stream's tensor can arrive as additive pieces in any
order: boxes (slices, sub-blocks) and rank-1 terms.  The server keeps every admitted
stream's plan (DRMs + FP64 sketch accumulators) resident on the device and

* admits streams in arrival order while their footprint (ttnn_footprint_estimate)
  fits the HBM budget; a stream that finishes releases its plan, and waiting streams
  are admitted as memory frees up;
* forms a batch whenever fewer than `max_inflight` batches are on the GPU: the
  oldest pending update of every admitted stream, up to `max_batch` updates;
  updates that arrive while earlier batches run join the next batch (continuous
  batching);
* launches each batch through ttnn_sketch_update_batched, which runs every step of
  the box updates of same-shaped plans as one launch, so a stream's result is bitwise
  the same alone and in the mix (fixed reduction orders);
* assembles cores on demand (every `assemble_every` updates of a stream, and when a
  stream closes), enqueued without draining the GPU; a closing stream is retired
  once an event after its final assembly has completed: the numerical status of all
  its assemblies (copied to pinned memory in stream order) is checked, `on_close`
  runs and the plan's memory is released in stream order;
* records a HIP event per batch and reports per-update latency (arrival to the end
  of its batch on the GPU) as p50/p99, beside throughput.

All device work is done by libttnn.so; this module schedules.  `engine` exists so
the scheduling rules can be exercised without a device.
"""

import collections
import time

import numpy as np


class Update:
    """One additive piece of a stream's tensor.

    kind 'box': `block` (device tensor, plan dtype, column-major box), `offset`,
    `extent`; kind 'rank1': `factors` (one FP64 device vector per mode)."""

    __slots__ = ("sid", "kind", "block", "offset", "extent", "factors", "alpha", "arrival", "nbytes",
                 "t_done", "t_launch", "t_gpu", "batch", "group")

    def __init__(self, sid, kind="box", block=None, offset=None, extent=None, factors=None, alpha=1.0,
                 arrival=0.0, nbytes=0):
        self.sid, self.kind, self.block, self.offset, self.extent = sid, kind, block, offset, extent
        self.factors, self.alpha, self.arrival, self.nbytes = factors, alpha, arrival, nbytes
        self.t_done = None
        self.group = None                       # rank-1: the terms launched with it (itself first)
        self.t_launch = None                    # host time its batch was launched
        self.t_gpu = None                       # device time of its batch (s)
        self.batch = None


class StreamSpec:
    """The problem of one stream (tree, dims, ranks, variant, dtype, DRM seed)."""

    def __init__(self, spec, dims, rank, over, variant="ttnn", dtype="f32", seed=1):
        self.spec, self.dims, self.rank, self.over = spec, tuple(dims), rank, over
        self.variant, self.dtype, self.seed = variant, dtype, seed


class LibEngine:
    """The device engine: plans, batched updates and events of libttnn.so."""

    def __init__(self, stream=None):
        import torch
        from . import _lib as L
        self.torch, self.L = torch, L
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.rank1_form = "termwise"            # the server sets "grouped" when it batches terms
        # pinned status words, reused (a pinned allocation costs milliseconds)
        self._pinned = [torch.zeros(1, dtype=torch.int32, pin_memory=True) for _ in range(16)]

    def footprint(self, s):
        return self.L.footprint_estimate(s.spec, s.dims, s.rank, s.over, s.variant, s.dtype)

    def create(self, s):
        plan = self.L.Plan(s.spec, s.dims, s.rank, s.over, variant=s.variant, dtype=s.dtype, seed=s.seed,
                           stream=self.stream)
        plan.set_rank1_form(self.rank1_form)
        return plan

    def launch(self, items):
        """items: list of (plan, Update) with at most one update per plan."""
        boxes = [(p, u.block, u.extent, u.offset, u.alpha) for p, u in items if u.kind == "box"]
        if boxes:
            self.L.update_batched(boxes, stream=self.stream)
        for p, u in items:
            if u.kind == "rank1":
                if u.group and len(u.group) > 1:          # one read of each map for the group
                    p.update_rank1_batched([x.factors for x in u.group], [x.alpha for x in u.group],
                                           stream=self.stream)
                else:
                    p.update_rank1(u.factors, u.alpha, stream=self.stream)

    def assemble(self, plan):
        """Cores of the plan; reads back the status of every assembly since the last
        query (synchronises the stream)."""
        cores = plan.assemble_async(stream=self.stream)
        plan.assemble_status(stream=self.stream)
        return cores

    def assemble_async(self, plan):
        """On-demand cores without draining the stream (status checked at close)."""
        return plan.assemble_async(stream=self.stream)

    def status_async(self, plan):
        """Enqueue the plan's sticky numerical status into pinned host memory; read it
        with status_value once an event recorded after this call has completed."""
        h = self._pinned.pop() if self._pinned else self.torch.zeros(1, dtype=self.torch.int32, pin_memory=True)
        plan.assemble_status_async(h, stream=self.stream)
        return h

    def status_value(self, h):
        v = int(h[0])
        self._pinned.append(h)
        return v

    def destroy(self, plan):
        """Release in stream order (no device synchronisation)."""
        plan.close_async(stream=self.stream)

    def event(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        return e

    def done(self, ev):
        return ev.query()

    def wait(self, ev):
        ev.synchronize()

    def elapsed_ms(self, ev0, ev1):
        return ev0.elapsed_time(ev1)

    def sync(self):
        self.torch.cuda.synchronize()


class _Stream:
    __slots__ = ("sid", "spec", "plan", "queue", "footprint", "closing", "n_done", "n_total", "cores",
                 "inflight", "admitted_at", "close_ev", "close_status")

    def __init__(self, sid, spec, footprint):
        self.sid, self.spec, self.footprint = sid, spec, footprint
        self.plan = None
        self.queue = collections.deque()
        self.closing = False
        self.n_done = 0
        self.n_total = 0
        self.cores = None
        self.inflight = 0
        self.admitted_at = None
        self.close_ev = None                    # event after the final assembly
        self.close_status = None


class Server:
    def __init__(self, budget_bytes, max_batch=64, max_inflight=2, assemble_every=0, engine=None,
                 keep_plans=False, on_close=None, rank1_batch=16):
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        # consecutive queued rank-1 updates of one stream launched together (up to this
        # many, never across an assembly point); the library applies them in order,
        # bitwise as one by one, reading each map once for the group
        self.rank1_batch = max(1, int(rank1_batch))
        self.max_inflight = int(max_inflight)
        self.assemble_every = int(assemble_every)
        self.keep_plans = keep_plans
        self.on_close = on_close                # on_close(sid, plan, cores) before the plan is released
        self.engine = engine if engine is not None else LibEngine()
        if self.rank1_batch > 1 and hasattr(self.engine, "rank1_form"):
            self.engine.rank1_form = "grouped"  # terms come in groups: the group form
        self.used = 0
        self.peak_used = 0                      # largest admitted footprint at any time
        self.create_s = []                      # host time of each plan creation (admission)
        self.streams = {}
        self.waiting = collections.deque()      # sids not yet admitted, arrival order
        self.admit_order = []
        self.inflight = collections.deque()     # (event, [updates], [sids], event before launch)
        self.completed = []
        self.batches = []                       # sizes of launched batches
        self.closed = {}                        # sid -> cores of finished streams
        self.plans = {}                         # sid -> plan of finished streams (keep_plans)
        self._ref = None
        self._t_ref = 0.0

    # ---------------------------------------------------------------- clock
    def start_clock(self):
        """Reference point shared by the host clock and the GPU events."""
        self.engine.sync()
        self._ref = self.engine.event()
        self.engine.wait(self._ref)
        self._t_ref = time.perf_counter()

    def now(self):
        return time.perf_counter() - self._t_ref

    # ---------------------------------------------------------------- streams
    def open_stream(self, sid, spec):
        if sid in self.streams:
            raise ValueError(f"stream {sid} is already open")
        fp = self.engine.footprint(spec)
        if fp > self.budget:
            raise ValueError(f"stream {sid} needs {fp} bytes, more than the whole budget {self.budget}")
        self.streams[sid] = _Stream(sid, spec, fp)
        self.waiting.append(sid)

    def submit(self, u):
        st = self.streams[u.sid]
        if st.closing:
            raise ValueError(f"stream {u.sid} is already closed")
        st.queue.append(u)
        st.n_total += 1

    def close_stream(self, sid):
        self.streams[sid].closing = True

    def _admit(self):
        while self.waiting:
            sid = self.waiting[0]
            st = self.streams[sid]
            if self.used + st.footprint > self.budget:
                break
            self.waiting.popleft()
            t0 = time.perf_counter()
            st.plan = self.engine.create(st.spec)
            self.create_s.append(time.perf_counter() - t0)
            self.used += st.footprint
            self.peak_used = max(self.peak_used, self.used)
            st.admitted_at = self.now() if self._ref is not None else 0.0
            self.admit_order.append(sid)

    def _retire(self, block=False):
        for sid in list(self.streams):
            st = self.streams[sid]
            if st.plan is None or not st.closing or st.queue or st.inflight:
                continue
            if st.close_ev is None:             # enqueue the final assembly, retire later
                st.cores = self.engine.assemble_async(st.plan)
                st.close_status = self.engine.status_async(st.plan)
                st.close_ev = self.engine.event()
                if not block:
                    continue
            if block:
                self.engine.wait(st.close_ev)
            elif not self.engine.done(st.close_ev):
                continue
            if self.engine.status_value(st.close_status) != 0:
                raise RuntimeError(f"stream {sid}: an assembly met a non-finite sketch or a rank-0 node")
            self.closed[sid] = st.cores
            if self.on_close is not None:
                self.on_close(sid, st.plan, st.cores)
            if self.keep_plans:                 # kept for inspection: its memory stays in use
                self.plans[sid] = st.plan
            else:
                self.engine.destroy(st.plan)
                self.used -= st.footprint
            st.plan = None
            del self.streams[sid]

    # ---------------------------------------------------------------- scheduling
    def _form_batch(self):
        ready = [st for st in self.streams.values() if st.plan is not None and st.queue]
        ready.sort(key=lambda st: st.queue[0].arrival)          # oldest pending update first
        return ready[: self.max_batch]

    def step(self):
        """Admit, launch at most one batch, retire finished streams.  Returns the
        number of updates launched."""
        self.poll()
        self._retire()
        self._admit()
        if len(self.inflight) >= self.max_inflight:
            return 0
        chosen = self._form_batch()
        if not chosen:
            return 0
        items, ups, counts = [], [], []
        for st in chosen:
            u = st.queue.popleft()
            group = [u]
            if u.kind == "rank1" and self.rank1_batch > 1:
                room = self.rank1_batch
                if self.assemble_every:
                    room = min(room, self.assemble_every - st.n_done % self.assemble_every)
                while len(group) < room and st.queue and st.queue[0].kind == "rank1":
                    group.append(st.queue.popleft())
            u.group = group if len(group) > 1 else None
            for x in group:
                x.batch = len(self.batches)
                ups.append(x)
            items.append((st.plan, u))
            counts.append(len(group))
            st.inflight += 1
        t_launch = self.now()
        for u in ups:
            u.t_launch = t_launch
        ev0 = self.engine.event()               # the batch's device span: ev0 .. ev
        self.engine.launch(items)
        for st, cnt in zip(chosen, counts):
            st.n_done += cnt                    # a group never crosses an assembly point
            if self.assemble_every and st.n_done % self.assemble_every == 0:
                st.cores = self.engine.assemble_async(st.plan)
        ev = self.engine.event()
        self.inflight.append((ev, ups, [st.sid for st in chosen], ev0))
        self.batches.append(len(ups))
        return len(ups)

    def poll(self, block=False):
        while self.inflight:
            ev, ups, sids, ev0 = self.inflight[0]
            if block:
                self.engine.wait(ev)
            elif not self.engine.done(ev):
                break
            self.inflight.popleft()
            t = self.engine.elapsed_ms(self._ref, ev) * 1e-3      # seconds on the server clock
            t_gpu = self.engine.elapsed_ms(ev0, ev) * 1e-3
            for u in ups:
                u.t_done = t
                u.t_gpu = t_gpu
                self.completed.append(u)
            for sid in sids:
                if sid in self.streams:
                    self.streams[sid].inflight -= 1

    def drain(self):
        """Run until no admitted stream has pending work and nothing is in flight
        (streams that were never closed stay admitted)."""
        while True:
            if self.step():
                continue
            if self.inflight:
                self.poll(block=True)
                continue
            self._retire(block=True)
            self._admit()
            if any(st.plan is not None and st.queue for st in self.streams.values()):
                continue
            break

    # ---------------------------------------------------------------- driver
    def run(self, arrivals):
        """arrivals: list of Update with `arrival` (seconds from start), sorted.  The
        caller has opened every stream; streams close after their last update."""
        self.start_clock()
        last = {}
        for u in arrivals:
            last[u.sid] = u
        i = 0
        n = len(arrivals)
        while i < n or self.inflight or any(st.queue for st in self.streams.values()):
            now = self.now()
            while i < n and arrivals[i].arrival <= now:
                u = arrivals[i]
                self.submit(u)
                if last[u.sid] is u:
                    self.close_stream(u.sid)
                i += 1
            launched = self.step()
            if launched == 0 and i >= n and not self.inflight and self.waiting and \
                    not any(st.plan is not None for st in self.streams.values()):
                raise RuntimeError("streams wait for admission but no admitted stream holds memory it can free")
            if launched == 0 and (i >= n or arrivals[i].arrival > self.now()):
                if self.inflight and not self.engine.done(self.inflight[0][0]):
                    time.sleep(20e-6)
                elif not self.inflight and i < n:
                    time.sleep(min(50e-6, max(0.0, arrivals[i].arrival - self.now())))
        self.drain()
        out = stats(self.completed, self.now())
        out["peak_used_bytes"] = self.peak_used
        out["plan_create_ms_max"] = max(self.create_s) * 1e3 if self.create_s else 0.0
        out["plan_create_ms_total"] = sum(self.create_s) * 1e3
        return out


def stats(completed, wall_s):
    lat = np.array([(u.t_done - u.arrival) * 1e3 for u in completed]) if completed else np.zeros(1)
    nbytes = sum(u.nbytes for u in completed)
    out = {
        "updates": len(completed),
        "wall_s": wall_s,
        "updates_per_s": len(completed) / wall_s if wall_s > 0 else 0.0,
        "ingest_GBps": nbytes / wall_s / 1e9 if wall_s > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
    }
    # latency = waiting (arrival to the launch of its batch: admission of its stream,
    # earlier updates of the stream, batches in flight) + on the GPU (launch to the end
    # of its batch)
    timed = [u for u in completed if u.t_launch is not None]
    if timed:
        wait = [(u.t_launch - u.arrival) * 1e3 for u in timed]
        gpu = [(u.t_done - u.t_launch) * 1e3 for u in timed]
        out["wait_p50_ms"], out["wait_p99_ms"] = float(np.percentile(wait, 50)), float(np.percentile(wait, 99))
        out["gpu_p50_ms"], out["gpu_p99_ms"] = float(np.percentile(gpu, 50)), float(np.percentile(gpu, 99))
    # device time of the batch that carried each update (from an event before its launch
    # to one after it: the batch's own span on the stream)
    dev = [u.t_gpu * 1e3 for u in completed if u.t_gpu is not None]
    if dev:
        out["device_p50_ms"], out["device_p99_ms"] = float(np.percentile(dev, 50)), float(np.percentile(dev, 99))
    for kind in ("box", "rank1"):
        lk = [(u.t_done - u.arrival) * 1e3 for u in completed if u.kind == kind]
        if lk:
            out[f"{kind}_p50_ms"] = float(np.percentile(lk, 50))
            out[f"{kind}_p99_ms"] = float(np.percentile(lk, 99))
        dk = [u.t_gpu * 1e3 for u in completed if u.kind == kind and u.t_gpu is not None]
        if dk:
            out[f"{kind}_device_p50_ms"] = float(np.percentile(dk, 50))
            out[f"{kind}_device_p99_ms"] = float(np.percentile(dk, 99))
            out[f"{kind}_updates"] = len(dk)
    return out
