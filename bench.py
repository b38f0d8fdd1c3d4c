"""Benchmark of the TTNN / STTNN sketch phase on one MI355X.

Workload: order-4 tensor 128^4 (268,435,456 entries) on the balanced binary tree
((1,2),(3,4)), built as a tree tensor network with edge ranks 24 and singular values
0.8^k on every edge, normalised to unit RMS plus N(0, 1e-4^2) noise; Gaussian DRMs,
sketch rank r = 32, oversampling p = 16; the whole tensor resident in HBM is
sketched in one pass and the TTN cores are assembled in FP64.

One step = sketch update of the whole tensor (fused one-pass kernel + deterministic
reduction) + FP64 epilogue + recovery phase (QR, Jacobi SVD, eps-pseudoinverse,
cores).  DRM generation happens once per plan, before timing.  The default warm-up
(40 steps, about 50 ms of FP32 work) brings the GPU to its sustained clock before the
timed steps; after a few steps from idle the sweep still runs about 10% slower.

    python bench.py [--steps K] [--warmup W] [--variants ttnn,sttnn] [--dtypes f32,f64,bf16]

Prints one compact JSON line last on stdout; the full results go to --detail.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sketch ingest GB/s (% HBM roofline) + p50/p99 update latency, bf16/fp32 vs fp64"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2516.6, "f32": 157.3, "f64": 78.6}
ESIZE = {"f64": 8, "f32": 4, "bf16": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--over", type=int, default=16)
    ap.add_argument("--variants", default="ttnn,sttnn")
    ap.add_argument("--dtypes", default="f32,f64,bf16")
    ap.add_argument("--headline", default="sttnn:f32")
    ap.add_argument("--precision-ranks", default="16,64",
                    help="extra STTNN BF16 and FP64 runs at these sketch ranks (p = r/2)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving runs")
    ap.add_argument("--single-n", type=int, default=64, help="mode size of the single-stream serving run")
    ap.add_argument("--config4-tilings", type=int, default=1,
                    help="two-piece tilings of the single-stream run (32 boxes each); 112 in the full recipe")
    ap.add_argument("--config4-pairs", type=int, default=256, help="cancelling rank-1 pairs of the single-stream run")
    ap.add_argument("--serve-streams", type=int, default=64)
    ap.add_argument("--serve-nmax", type=int, default=160)
    ap.add_argument("--no-hilbert", action="store_true", help="skip the 6-D Hilbert accuracy curves")
    ap.add_argument("--hilbert-only", action="store_true",
                    help="run only the Hilbert curves and print them as one JSON line")
    ap.add_argument("--hilbert-n", type=int, default=20)
    ap.add_argument("--hilbert-trials", type=int, default=3, help="DRM seeds per rank (the paper averages 30)")
    ap.add_argument("--hilbert-ranks", default="2,3,4,5,6,7,8,9,10,11,12,13")
    ap.add_argument("--hilbert-dtypes", default="f64,f32")
    ap.add_argument("--detail", default="bench_detail.json",
                    help="file for the full per-configuration, serving and Hilbert results ('' = none)")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="the Poisson load (a fraction of the batched path's closed-loop rate) summarised in the record")
    ap.add_argument("--serve-loads", default="0.25,0.5,0.8", help="Poisson loads run (fractions of the closed-loop rate)")
    ap.add_argument("--no-rounding", action="store_true", help="skip the TTN rounding runs (Khatri-Rao maps)")
    ap.add_argument("--no-pipeline", action="store_true", help="skip the two-plan throughput runs")
    ap.add_argument("--no-order", action="store_true", help="skip the STTNN visiting-order runs")
    ap.add_argument("--order-only", action="store_true",
                    help="only the STTNN visiting-order runs (lexicographic against searched)")
    ap.add_argument("--order-cases", default="t4,hilbert", help="visiting-order workloads run (t4, hilbert)")
    ap.add_argument("--rank1-only", action="store_true",
                    help="only the rank-1 groups on the streaming configuration's plan")
    ap.add_argument("--order-visits", default="lexicographic,searched", help="visiting orders run")
    ap.add_argument("--rounding-only", action="store_true",
                    help="run only the TTN rounding runs and print them as one JSON line")
    ap.add_argument("--round-n", type=int, default=500)
    ap.add_argument("--round-ranks", default="16,32,48")
    ap.add_argument("--round-trials", type=int, default=3, help="map seeds per rank (the paper averages 30)")
    return ap.parse_args()


# ---------------------------------------------------------------- work counts
# Node list of ((1,2),(3,4)) in level order (root, A, B, {1}, {2}, {3}, {4}) and the
# STTNN reuse sets of Sec. 5 / Fig. 5 on it: S_A = S_1 = {} , S_B = {A}, S_2 = {{1}},
# S_3 = {A}, S_4 = {A, {3}}.
T4_MODES = [(1, 2, 3, 4), (1, 2), (3, 4), (1,), (2,), (3,), (4,)]


def work_counts(dims, r, p, variant):
    """Leading-order flops and DRM entries of one sketch pass over the whole tensor on
    ((1,2),(3,4)), every node with rank r and oversampling p (k = r + p).

    Flops: every contraction of the sketch phase, 2 * (entries of its input) * (columns
    of its DRM), including the root chain T x_A Y_A^T x_B Y_B^T.  DRM entries: every
    X_t, and every Y_s that some contraction of the tensor (or of an intermediate) uses,
    once.  Returns (flops, drm_entries, N)."""
    n1, n2, n3, n4 = dims
    N = n1 * n2 * n3 * n4
    nA, nB = n1 * n2, n3 * n4
    k = r + p
    if variant == "ttnn":
        flops = 2 * N * (6 * r + k) + 2 * k * nB * k           # six R_t, root chain
        x_rows = nB + nA + N // n1 + N // n2 + N // n3 + N // n4
        y_used = nA + nB                                       # Y_A, Y_B (root)
    else:
        flops = (2 * N * k                      # T x_A Y_A^T (S_B, S_3, S_4, root)
                 + 2 * N * k                    # T x_1 Y_1^T (S_2)
                 + 2 * (k * n3 * n4) * k        # (T x_A Y_A^T) x_3 Y_3^T (S_4)
                 + 2 * (k * nB) * k             # root: x_B Y_B^T
                 + 2 * N * r                    # R_A
                 + 2 * (k * nB) * r             # R_B
                 + 2 * N * r                    # R_1
                 + 2 * (k * n2 * n3 * n4) * r   # R_2
                 + 2 * (k * n3 * n4) * r        # R_3
                 + 2 * (k * k * n4) * r)        # R_4
        x_rows = nB + k + N // n1 + k * n3 * n4 + k * n4 + k * k
        y_used = nA + nB + n1 + n3                             # Y_A, Y_B, Y_1, Y_3
    return flops, x_rows * r + y_used * k, N


def sweep_counts(dims, r, p, variant, dtype, kind):
    """Algorithmic flops and bytes of the timed sweep kernel alone (`kind` as reported
    by the library, ttnn_sweep_kind), on ((1,2),(3,4)).

    1: the one-pass STTNN kernel reads the tensor once and the DRMs X_A, X_1, X_2, Y_A,
       Y_1 once, and writes R_A, Z_A = Y_A^T T^{A}, R_1, R_2 once (FP32; FP64 for an
       FP64 plan); the remaining nodes are formed from Z_A afterwards.
    2: the same kernel without R_2: it writes Z1 = Y_1^T T^{(1)} (k x N / n_1, in the
       plan dtype, FP32 for a BF16 plan) and reads no X_2; R_2 is a separate streaming
       contraction.
    3: the TTNN-mode kernel: tensor once, X_A, X_1, Y_A, X_B once; R_A, Z_A, R_1, R_B out.
    0: the sweep is the whole update and its counts are those of the pass."""
    flops, drm, N = work_counts(dims, r, p, variant)
    s = ESIZE[dtype]
    if kind == 0:
        return flops, N * s + drm * s
    n1, n2, n3, n4 = dims
    nA, nB = n1 * n2, n3 * n4
    k = r + p
    acc = 8 if dtype == "f64" else 4
    if kind == 3:
        drm_k = nB * r + (N // n1) * r + nA * k + nA * r        # X_A, X_1, Y_A, X_B
        out = nA * r + k * nB + n1 * r + nB * r
        return 2 * N * (3 * r + k), N * s + drm_k * s + out * acc
    drm_k = nB * r + (N // n1) * r + nA * k + n1 * k              # X_A, X_1, Y_A, Y_1
    out = nA * r + k * nB + n1 * r
    kflops = 2 * N * (2 * r + 2 * k)
    if kind == 1:
        drm_k += k * n3 * n4 * r                                 # X_2
        out += n2 * r
        kflops += 2 * (N // n1) * k * r
        return kflops, N * s + drm_k * s + out * acc
    zs = 4 if dtype == "bf16" else s               # a BF16 plan writes Z1 in FP32
    return kflops, N * s + drm_k * s + out * acc + k * (N // n1) * zs


def measured_traffic(key):
    """HBM bytes per launch of the fused sweep kernel, from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs summarised under profiles/ (scaled by a plain 1 GiB copy), if the
    kernel sources still hash to what was measured; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sttnn_t4_kernel_traffic.json")
    if not key.startswith("sttnn:") or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2412_06111_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest()[:16] != rec["hash"] or key not in rec["traffic"]:
        return None
    return rec["traffic"][key]["bytes"]


def copy_rate(nbytes=1 << 30, reps=10):
    """A plain device-to-device copy of known size: the calibration kernel for the
    HBM byte counters and a measured streaming ceiling (read + write bytes / time)."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        y.copy_(x)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": ms, "GBps_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}


# ---------------------------------------------------------------- GPU run
def read_sketches(plan):
    """Every node sketch of the plan's last update (R, Omega, Psi; Psi only at the root),
    as FP64 host arrays keyed by (node modes, kind)."""
    import paper_2412_06111_amd as P
    out = {}
    for i, modes in enumerate(T4_MODES):
        cid = plan.node(modes)
        for kind in ((P.SK_PSI,) if i == 0 else (P.SK_R, P.SK_OMEGA, P.SK_PSI)):
            out[(modes, kind)] = plan.read_sketch(cid, kind).cpu().numpy()
    return out


def sketch_rel_errors(sk, ref):
    """Per node, the largest relative Frobenius error of its sketches against `ref`."""
    import numpy as np
    per = {}
    for (modes, kind), a in sk.items():
        b = ref[(modes, kind)]
        e = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        key = ",".join(str(m) for m in modes)
        per[key] = max(per.get(key, 0.0), e)
    return per


def run_gpu(args, T_dev64, variant, dtype, rank=None, over=None, keep_sketches=False):
    import torch
    import paper_2412_06111_amd as P
    from workloads.serving import T4

    rank = args.rank if rank is None else rank
    over = args.over if over is None else over
    dims = (args.n,) * 4
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    plan = P.Plan(T4, dims, rank, over, variant=variant, dtype=dtype, seed=1)
    t1.record()
    torch.cuda.synchronize()
    drm_ms = t0.elapsed_time(t1)
    if dtype == "f64":
        X = T_dev64
    elif dtype == "f32":
        X = T_dev64.to(torch.float32)
    else:
        X = T_dev64.to(torch.float32).to(torch.bfloat16)
    cores = plan.alloc_cores()

    sweep_ms = []

    def step(ev=None):
        plan.reset()
        if ev is not None:
            ev[0].record(stream)
        plan.update(X)
        if ev is not None:
            ev[1].record(stream)
        plan.assemble_async(cores)    # enqueued; the numerical status is read once per timed run
        if ev is not None:
            sweep_ms.append(plan.sweep_time_ms())

    plan.set_timing(True)             # HIP events on the launch stream around the sweep kernel
    for _ in range(args.warmup):
        step()
    plan.assemble_status()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    tic = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    plan.assemble_status()            # every timed assembly was numerically sound
    torch.cuda.synchronize()
    toc = time.perf_counter()
    ms_step = (toc - tic) * 1e3 / args.steps
    sketch_ms = [a.elapsed_time(b) for a, b in evs]
    res = {"ms_per_step": ms_step, "sketch_ms_avg": sum(sketch_ms) / len(sketch_ms),
           "sketch_ms_min": min(sketch_ms), "sweep_kernel_ms_avg": sum(sweep_ms) / len(sweep_ms),
           "sweep_kernel_ms_min": min(sweep_ms), "drm_generation_ms": drm_ms, "footprint_bytes": plan.footprint(),
           "sweep_kind": plan.sweep_kind()}
    if not args.no_error:
        That = plan.reconstruct(cores)
        e2, n2 = P.diff_norms(That, T_dev64)
        res["approx_rel_error"] = (e2 / n2) ** 0.5
        del That
    if keep_sketches:
        res["_sketches"] = read_sketches(plan)
    del X
    plan.close()
    torch.cuda.empty_cache()
    return res


def run_pipelined(args, T_dev64, variant, dtype, nplans=2):
    """Throughput with `nplans` plans of the same problem taking the steps in turn, each on
    a stream of its own (reset + whole-tensor update + enqueued assembly, as in run_gpu),
    so that one step's FP64 tail runs while the next step's sweep starts: ms per step =
    wall time over the timed steps.  Every step does the whole work of a step."""
    import torch
    import paper_2412_06111_amd as P
    from workloads.serving import T4

    dims = (args.n,) * 4
    X = T_dev64 if dtype == "f64" else T_dev64.to(torch.float32)
    if dtype == "bf16":
        X = X.to(torch.bfloat16)
    streams = [torch.cuda.Stream() for _ in range(nplans)]
    plans, cores = [], []
    for k in range(nplans):
        with torch.cuda.stream(streams[k]):
            plans.append(P.Plan(T4, dims, args.rank, args.over, variant=variant, dtype=dtype, seed=1,
                                stream=streams[k]))
            cores.append(plans[-1].alloc_cores())
    torch.cuda.synchronize()

    def run(n):
        for i in range(n):
            k = i % nplans
            with torch.cuda.stream(streams[k]):
                plans[k].reset(stream=streams[k])
                plans[k].update(X, stream=streams[k])
                plans[k].assemble_async(cores[k], stream=streams[k])

    run(args.warmup)
    torch.cuda.synchronize()
    tic = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - tic) * 1e3 / args.steps
    for k in range(nplans):
        plans[k].assemble_status(stream=streams[k])      # every assembly was numerically sound
        plans[k].close()
    del X
    torch.cuda.empty_cache()
    return ms


# ---------------------------------------------------------------- 6-D Hilbert curves
# pseudo-inverse thresholds: the library default (10 * 2^-52) for FP64 sketches, the FP32
# noise level for FP32 sketches (a threshold set for FP64 keeps noise directions there)
EPS_HILBERT = {"f64": 0.0, "f32": 10.0 * 2.0 ** -23, "bf16": 0.0}
def hilbert_bench(args):
    """The first accuracy experiment of Sec. 8: the 6-D Hilbert tensor
    1 / (1 + i_1 + .. + i_6) (mode size 20, 64M entries, resident in HBM) on the index
    tree of Fig. 1, equal ranks r, p = 3, TTNN and STTNN.  Per rank: the mean relative
    Frobenius error over `--hilbert-trials` DRM seeds (the paper averages 30) and the
    time of one approximation (reset + sketch update of the whole tensor + assembly of
    the cores), from events on the stream, averaged over 5 timed repeats with the first
    seed's plan after 2 untimed ones.  The FP32 rows sketch the FP32 rounding of the
    tensor, with the pseudo-inverse threshold at the FP32 noise level; their errors are
    against the FP64 tensor."""
    import torch
    import paper_2412_06111_amd as P
    from workloads import hilbert as H

    n = args.hilbert_n
    dims = (n,) * 6
    T64 = H.hilbert_device(n)
    ranks = [int(x) for x in args.hilbert_ranks.split(",") if x]
    out = {"workload": f"6-D Hilbert tensor, {n}^6 on the Fig. 1 tree (((1,2),3),4,(5,6)), p = {H.P_PAPER}",
           "trials": args.hilbert_trials, "eps_factor": EPS_HILBERT, "curves": {}}
    stream = torch.cuda.current_stream()
    for dtype in args.hilbert_dtypes.split(","):
        X = T64 if dtype == "f64" else T64.to(torch.float32)
        for variant in ("ttnn", "sttnn"):
            rows = []
            for r in ranks:
                errs, ms = [], None
                for trial in range(args.hilbert_trials):
                    plan = P.Plan(H.TOY, dims, r, H.P_PAPER, variant=variant, dtype=dtype, seed=100 + trial,
                                  eps_factor=EPS_HILBERT[dtype])
                    cores = plan.alloc_cores()
                    if trial == 0:
                        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                               for _ in range(7)]
                        for a, b in evs:
                            a.record(stream)
                            plan.reset()
                            plan.update(X)
                            plan.assemble_async(cores)
                            b.record(stream)
                        plan.assemble_status()
                        torch.cuda.synchronize()
                        t = [a.elapsed_time(b) for a, b in evs[2:]]
                        ms = sum(t) / len(t)
                    else:
                        plan.update(X)
                        plan.assemble(cores)
                    e2, n2 = P.diff_norms(plan.reconstruct(cores), T64)
                    errs.append((e2 / n2) ** 0.5)
                    plan.close()
                rows.append({"rank": r, "mean_rel_error": sum(errs) / len(errs), "max_rel_error": max(errs),
                             "ms_per_approximation": ms,
                             "ingest_GBps": X.numel() * X.element_size() / (ms * 1e-3) / 1e9})
            out["curves"][f"{variant}:{dtype}"] = rows
            print(f"# hilbert {variant}:{dtype}: r={rows[-1]['rank']} error {rows[-1]['mean_rel_error']:.2e}",
                  file=sys.stderr, flush=True)
        del X
    del T64
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- TTN rounding
ROUND_TTN_RANK, ROUND_P = 70, 10
ROUND_DECAYS = {"quadratic": lambda i: 1.0 / i ** 2, "cubic": lambda i: 1.0 / i ** 3, "exponential": lambda i: 0.5 ** i}


def order_bench(args):
    """STTNN in the lexicographic visiting order of Sec. 5 and in the order of least
    modelled cost (ttnn_order_search), on workloads where the order matters: T4 with
    n_1 << n_2 (FP32) and the 6-D Hilbert tensor on the tree of Fig. 1 (FP64, r = 13,
    the largest rank of the experiment).  Per order: ms per step (reset + whole-tensor
    update + assembly, as the headline), sketch ms (HIP events around the update),
    the model's flops and map entries, the plan footprint, the approximation error."""
    import numpy as np
    import torch
    import paper_2412_06111_amd as P
    from workloads import hilbert as H
    from workloads import synth as W

    T4 = ((1, 2), (3, 4))
    out = {}
    cases = [("t4", "t4_32x512x128x128_r32_f32", T4, (32, 512, 128, 128), 32, 16, "f32"),
             ("hilbert", "hilbert6d_n20_fig1tree_r13_f64", H.TOY, (20,) * 6, 13, H.P_PAPER, "f64")]
    wanted, visits = args.order_cases.split(","), args.order_visits.split(",")
    stream = torch.cuda.current_stream()
    for short, name, spec, dims, r, p, dtype in cases:
        if short not in wanted:
            continue
        if name.startswith("hilbert"):
            X64 = H.hilbert_device(dims[0]).reshape(-1)
        else:
            X64 = torch.from_numpy(np.ascontiguousarray(W.flat_colmajor(W.unbalanced_tensor(dims)))).cuda()
        X = X64 if dtype == "f64" else X64.to(torch.float32)
        best, _ = P.order_search(spec, dims, r, p)
        rec = {"searched_order": repr(best)}
        for label, visit in (("lexicographic", None), ("searched", best)):
            if label not in visits:
                continue
            plan = P.Plan(spec, dims, r, p, variant="sttnn", dtype=dtype, seed=1, visit=visit)
            cores = plan.alloc_cores()

            def step(ev=None):
                plan.reset()
                if ev is not None:
                    ev[0].record(stream)
                plan.update(X)
                if ev is not None:
                    ev[1].record(stream)
                plan.assemble_async(cores)

            for _ in range(args.warmup):
                step()
            plan.assemble_status()
            torch.cuda.synchronize()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            tic = time.perf_counter()
            for i in range(args.steps):
                step(evs[i])
            plan.assemble_status()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - tic) * 1e3 / args.steps
            e2, n2 = P.diff_norms(plan.reconstruct(cores), X64)
            rec[label] = {"ms_per_step": ms,
                          "sketch_ms_avg": sum(a.elapsed_time(b) for a, b in evs) / len(evs),
                          "model_gflop": P.order_cost(spec, dims, r, p, visit=visit) / 1e9,
                          "model_map_entries": P.order_cost(spec, dims, r, p, visit=visit, objective="maps"),
                          "footprint_bytes": plan.footprint(), "approx_rel_error": (e2 / n2) ** 0.5}
            plan.close()
            del cores
            torch.cuda.empty_cache()
            print(f"# order {name} {label}: {rec[label]['ms_per_step']:.3f} ms/step, "
                  f"{rec[label]['model_gflop']:.1f} GFLOP (model)", file=sys.stderr, flush=True)
        if "lexicographic" in rec and "searched" in rec:
            rec["speedup"] = rec["lexicographic"]["ms_per_step"] / rec["searched"]["ms_per_step"]
        out[name] = rec
        del X, X64
        torch.cuda.empty_cache()
    return out


def rank1_bench(args):
    """Rank-1 updates on the streaming configuration's plan: 64^5 on (((1,2),3),(4,5)),
    TTNN, r = 24, p = 12, FP32 maps, in groups of 1, 2, 4 and 8 terms
    (ttnn_sketch_update_rank1_batched, bitwise equal to the terms one by one).  Per group
    size: ms a group and a term (stream events), and the maps' bytes a term over its
    time (every row of every X_t is read once per group)."""
    import numpy as np
    import torch
    import paper_2412_06111_amd as P
    from workloads.serving import T5

    n = args.single_n
    dims = (n,) * 5
    g = np.random.default_rng(5)
    terms = [[torch.from_numpy(g.standard_normal(k)).cuda() for k in dims] for _ in range(16)]
    stream = torch.cuda.current_stream()
    out = {"workload": f"{n}^5 on (((1,2),3),(4,5)), TTNN, r=24, p=12, FP32 maps"}
    for form in ("termwise", "grouped"):
        plan = P.Plan(T5, dims, 24, 12, variant="ttnn", dtype="f32", seed=1)
        plan.set_rank1_form(form)
        map_bytes = 0
        for i in range(1, plan.num_nodes):
            rows, cols = plan.drm_shape(i, 0)
            map_bytes += rows * cols * 4
        out["map_bytes"] = map_bytes
        for m in (1, 2, 4, 8, 16):
            for _ in range(2):
                plan.update_rank1_batched(terms[:m], [1.0] * m)
            torch.cuda.synchronize()
            reps = max(2, args.steps // 2)
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(reps):
                plan.update_rank1_batched(terms[:m], [1.0] * m)
            t1.record(stream)
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / reps
            out[f"{form}_group{m}"] = {"ms_per_group": ms, "ms_per_term": ms / m,
                                       "map_GBps_per_group": map_bytes / (ms * 1e-3) / 1e9}
            print(f"# rank-1 {form} group of {m}: {ms:.3f} ms, {ms / m:.3f} ms a term, maps "
                  f"{map_bytes / (ms * 1e-3) / 1e9:.0f} GB/s", file=sys.stderr, flush=True)
        plan.close()
    return out


def rounding_counts(spec, dims, r, p, s):
    """Flops of one structured sketch (Khatri-Rao maps) of a TTN with ranks s on `spec`,
    every node with rank r and oversampling p (k = r + p), as the path computes it: down
    vectors (each core entry times r + k columns), up vectors (r columns per child),
    Omega_t = dy^T u, leaf R_t = U u, and the Psi chains (parent index with u, then each
    child with dy; the root's children only).  2 flops per multiply-add."""
    from workloads import synth as W
    k = r + p
    fma = 0
    for i, (sp, modes, par, kids) in enumerate(W.tree_spec_nodes(spec)):
        root = i == 0
        if not kids:
            nt = 1
            for m in modes:
                nt *= dims[m - 1]
            core = nt * s
            fma += core * (r + k) + s * k * r + nt * s * r
            continue
        m = len(kids)
        core = s ** m * (1 if root else s)
        if not root:
            fma += core * (r + k) + s * k * r
        fma += core * r * m                                   # up vectors of the children
        sizes = [s] * m + ([] if root else [s])
        if not root:                                          # parent index with u
            fma += core * r
            sizes[-1] = r
        for q in range(m):                                    # each child index with dy
            cur = 1
            for x in sizes:
                cur *= x
            fma += cur * k
            sizes[q] = k
    return 2 * fma


def rounding_bench(args):
    """The second experiment of Sec. 8: rounding of order-6 tensors given in TTN format
    on the tree of Fig. 1, mode size 500, TTN ranks 70, internal cores superdiagonal with
    entries sigma_i (quadratic, cubic, exponential decay) rotated by Haar matrices, Haar
    leaves; TTNN with Khatri-Rao maps (Sec. 7), equal ranks r, p = 10.  Per decay and
    rank: the mean relative error ||T - T_r|| / ||T|| over `--round-trials` map seeds,
    from TTN inner products on the GPU, and the time of one rounding (reset + structured
    sketch of the TTN + FP64 assembly of the cores), from events on the stream,
    averaged over 10 timed repeats after 3 untimed ones."""
    import numpy as np
    import torch
    import paper_2412_06111_amd as P
    from workloads import synth as W

    spec = ((((1, 2), 3), 4, (5, 6)))
    n = args.round_n
    dims = (n,) * 6
    s = ROUND_TTN_RANK
    ranks = [int(x) for x in args.round_ranks.split(",") if x]
    out = {"workload": f"TTN rounding, order 6, n={n}, TTN ranks {s}, Fig. 1 tree, Khatri-Rao maps, p={ROUND_P}",
           "trials": args.round_trials, "rows": {}}
    stream = torch.cuda.current_stream()
    for name, f in ROUND_DECAYS.items():
        sigma = np.array([f(i) for i in range(1, s + 1)])
        host = W.decaying_ttn_cores(spec, dims, s, sigma, seed=7)
        dc = {m: torch.from_numpy(np.ascontiguousarray(c.reshape(-1, order="F"))).cuda() for m, c in host.items()}
        for r in ranks:
            errs, ms = [], None
            for trial in range(args.round_trials):
                plan = P.Plan(spec, dims, r, ROUND_P, variant="kr", seed=300 + trial)
                cores = plan.alloc_cores()
                work = torch.empty(plan.update_ttn_work_bytes(s), dtype=torch.uint8, device="cuda")
                if trial == 0:
                    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                           for _ in range(13)]
                    for a, b in evs:
                        a.record(stream)
                        plan.reset()
                        plan.update_ttn(dc, s, work=work)
                        plan.assemble_async(cores)
                        b.record(stream)
                    plan.assemble_status()
                    torch.cuda.synchronize()
                    t = [a.elapsed_time(b) for a, b in evs[3:]]
                    ms = sum(t) / len(t)
                else:
                    plan.update_ttn(dc, s, work=work)
                    plan.assemble(cores)
                rr = plan.core_ranks()
                tt = plan.ttn_dot(dc, s, dc, s)
                e2 = tt - 2 * plan.ttn_dot(dc, s, cores, rr) + plan.ttn_dot(cores, rr, cores, rr)
                errs.append(float(np.sqrt(max(e2, 0.0) / tt)))
                plan.close()
            flops = rounding_counts(spec, dims, r, ROUND_P, s)
            out["rows"][f"{name}:r{r}"] = {"rank": r, "mean_rel_error": sum(errs) / len(errs),
                                          "max_rel_error": max(errs), "ms_per_rounding": ms,
                                          "sketch_flops": flops,
                                          "TFLOPs_whole_rounding": flops / (ms * 1e-3) / 1e12}
            print(f"# rounding {name} r={r}: {ms:.3f} ms, error {sum(errs) / len(errs):.3e}",
                  file=sys.stderr, flush=True)
        del dc
    torch.cuda.empty_cache()
    return out


def cpu_baseline_rounding(args, r=48):
    """The oracle (plain NumPy FP64 tree contractions and recovery) on one rounding of
    the quadratic-decay TTN of the rounding runs, same sizes: the CPU reference time."""
    import numpy as np
    import oracle as O
    from oracle import structured as S
    from workloads import synth as W

    spec = ((((1, 2), 3), 4, (5, 6)))
    dims = (args.round_n,) * 6
    s = ROUND_TTN_RANK
    sigma = np.array([ROUND_DECAYS["quadratic"](i) for i in range(1, s + 1)])
    cores = W.decaying_ttn_cores(spec, dims, s, sigma, seed=7)
    tree = O.Tree(spec, dims, r, ROUND_P)
    X, Y = S.factors(300, dims, r, ROUND_P)
    reps, t0 = 0, time.perf_counter()
    while True:
        O.assemble(S.ttn_sketch(cores, tree, X, Y), tree)
        reps += 1
        if time.perf_counter() - t0 > 3.0 or reps >= 50:
            break
    sec = (time.perf_counter() - t0) / reps
    return {"value": sec * 1e3, "unit": "ms per rounding", "kind": "oracle", "rank": r,
            "sample": f"{reps} roundings (structured sketch + assembly, maps drawn once)"}


# ---------------------------------------------------------------- serving
def _brief(name, st):
    print(f"# serving {name}: {st['updates_per_s']:.0f} updates/s, p50 {st['p50_ms']:.3f} ms, "
          f"p99 {st['p99_ms']:.3f} ms", file=sys.stderr, flush=True)


def serving_bench(args):
    """Many streams of box updates (mode sizes U{32..nmax}, TTN ranks 8..32 + 1e-5
    noise, r in {16, 32}, p = r/2, TTNN on ((1,2),(3,4))).  Batched FP32 server vs the
    plain FP64 path with one update per launch, each closed-loop (all updates at t=0,
    admission at 50% of the streams' total footprint) and under Poisson arrivals at
    `serve_load` x the batched closed-loop rate (budget = total footprint: every
    stream's updates interleave over the whole run).  Update payloads are resident in
    HBM before the clock starts."""
    import numpy as np
    import torch
    import paper_2412_06111_amd as P
    from paper_2412_06111_amd import serve as S
    from workloads import serving as WS

    probs = [WS.stream_problem(s, nhi=args.serve_nmax) for s in range(args.serve_streams)]
    tens, boxes = [], []
    for pr in probs:
        tens.append(WS.stream_tensor_device(pr))
        boxes.append(WS.boxes(pr["dims"], WS.rng(pr["seed"] + 31)))
    n_updates = sum(len(b) for b in boxes)

    def make_updates(dtype):
        tdt = {"f32": torch.float32, "f64": torch.float64}[dtype]
        per = []
        for s, (pr, T, bx) in enumerate(zip(probs, tens, boxes)):
            n1, n2, n3, n4 = pr["dims"]
            V = T.view(n4, n3, n2, n1)
            ups = []
            for off, ext in bx:
                blk = V[off[3]:off[3] + ext[3], off[2]:off[2] + ext[2], off[1]:off[1] + ext[1],
                        off[0]:off[0] + ext[0]].to(tdt).contiguous().reshape(-1)
                ups.append(S.Update(s, "box", block=blk, offset=off, extent=ext, nbytes=blk.numel() * blk.element_size()))
            per.append(ups)
        return per

    def specs(dtype):
        return [S.StreamSpec(WS.T4, pr["dims"], pr["r"], pr["p"], variant="ttnn", dtype=dtype, seed=pr["seed"])
                for pr in probs]

    def one_run(dtype, max_batch, rate, per):
        sp = specs(dtype)
        fps = [P.footprint_estimate(x.spec, x.dims, x.rank, x.over, x.variant, x.dtype) for x in sp]
        # closed loop: half the streams' footprint (admission as memory frees up);
        # Poisson: every stream admitted (their updates interleave over the whole run)
        budget = max(max(fps), sum(fps) // 2) if not rate else sum(fps)
        final = {}

        def on_close(sid, plan, cores):   # keep the cores; errors are measured after the run
            final[sid] = cores

        srv = S.Server(budget_bytes=budget, max_batch=max_batch, max_inflight=2, on_close=on_close)
        for s in range(len(probs)):
            srv.open_stream(s, sp[s])
        # arrival order: a random interleaving of the streams (each stream's boxes in its own order)
        g = WS.rng(7)
        order = g.permutation(np.repeat(np.arange(len(probs)), [len(u) for u in per]))
        nxt = [0] * len(probs)
        arrivals = []
        times = WS.poisson_arrivals(len(order), rate, seed=11) if rate else np.zeros(len(order))
        for t, sid in zip(times, order):
            u = per[sid][nxt[sid]]
            nxt[sid] += 1
            u.arrival, u.t_done = float(t), None
            arrivals.append(u)
        st = srv.run(arrivals)
        errs = {}
        for sid, cores in final.items():  # outside the timed run: reconstruct with a plan of the same tree
            x = sp[sid]
            pl = P.Plan(x.spec, x.dims, x.rank, x.over, variant=x.variant, dtype=x.dtype, seed=x.seed)
            That = pl.reconstruct(cores)
            e2, n2 = P.diff_norms(That, tens[sid])
            errs[sid] = (e2 / n2) ** 0.5
            del That
            pl.close()
        st["budget_bytes"] = budget
        st["total_footprint_bytes"] = sum(fps)
        st["mean_batch"] = float(np.mean(srv.batches)) if srv.batches else 0.0
        st["approx_rel_error_median"] = float(np.median(list(errs.values())))
        st["approx_rel_error_max"] = float(np.max(list(errs.values())))
        # streams whose sketch rank is below a TTN edge rank cannot capture their tensor:
        # their errors are reported apart
        low = [s for s in errs if probs[s]["r"] < max(probs[s]["ttn_ranks"].values())]
        ok = [s for s in errs if s not in low]
        st["streams_r_below_ttn_rank"] = len(low)
        if ok:
            st["approx_rel_error_max_r_at_least_ttn_rank"] = float(max(errs[s] for s in ok))
        if low:
            st["approx_rel_error_median_r_below_ttn_rank"] = float(np.median([errs[s] for s in low]))
        return st

    out = {"streams": len(probs), "updates": n_updates,
           "workload": f"{len(probs)} streams, TTNN on ((1,2),(3,4)), n ~ U{{32..{args.serve_nmax}}}, "
                       "TTN ranks 8..32 + 1e-5 noise, r in {16,32}, p=r/2, sub-blocks 4..48 per mode; "
                       "closed loop: admission at 50% of the total footprint; Poisson: all streams admitted"}
    per32 = make_updates("f32")
    closed = one_run("f32", 64, 0.0, per32)
    out["batched_f32_closed_loop"] = closed
    _brief("batched f32 closed loop", closed)
    per64 = make_updates("f64")
    out["fp64_one_per_launch_closed_loop"] = one_run("f64", 1, 0.0, per64)
    _brief("fp64 closed loop", out["fp64_one_per_launch_closed_loop"])
    # Poisson arrivals at fractions of the batched path's closed-loop rate, both paths on
    # the same arrival trace
    out["poisson"] = {}
    for load in [float(x) for x in args.serve_loads.split(",") if x]:
        rate = load * closed["updates_per_s"]
        b = one_run("f32", 64, rate, per32)
        f = one_run("f64", 1, rate, per64)
        out["poisson"][f"{load:g}"] = {"rate_per_s": rate, "batched_f32": b, "fp64_one_per_launch": f}
        _brief(f"batched f32 poisson {load:g}", b)
        _brief(f"fp64 poisson {load:g}", f)
    hi = out["poisson"].get(f"{args.serve_load:g}")
    if hi:
        out["poisson_rate_per_s"] = hi["rate_per_s"]
        out["batched_f32_poisson"] = hi["batched_f32"]
        out["fp64_one_per_launch_poisson"] = hi["fp64_one_per_launch"]
    del per64, tens
    torch.cuda.empty_cache()
    return out


def serving_single(args):
    """Single stream of the order-5 serving workload through the batching server: the
    64^5 FP32 TTN on (((1,2),3),(4,5)) with every edge rank 16 (N(0,1) cores, seeded,
    unit RMS), r = 24, p = 12, TTNN.  Updates: the 32 boxes of each of `config4_tilings`
    two-piece tilings (one cut per mode at U{8..56}), each the resident tensor over the
    box read in place (strided) with alpha = 1 / tilings, plus `config4_pairs` cancelling
    pairs of rank-1 terms with N(0,1) factors; all in a random order, submitted at once
    (closed loop); cores enqueued every 256 updates.  Per update: the device time of its
    launch (p50 / p99, overall and by kind); ingest rate (payload bytes: box entries
    read and rank-1 factor bytes, over wall time); approximation error of the final
    cores against the tensor (the pairs cancel, the tilings sum to it)."""
    import numpy as np
    import torch
    import paper_2412_06111_amd as P
    from paper_2412_06111_amd import serve as S
    from workloads import serving as WS

    n = args.single_n
    dims = (n,) * 5
    T64 = WS.order5_tensor_device(n=n, rank=16, seed=0, noise=0.0)
    X = T64.to(torch.float32)
    V = X.view(*dims[::-1])                                   # [i5, .., i1]
    k = args.config4_tilings
    ups = []
    for off, ext in WS.cut_tilings(dims, k, seed=3, lo=8, hi=56):
        view = V[tuple(slice(o, o + e) for o, e in zip(off[::-1], ext[::-1]))]
        nb = int(np.prod(ext)) * 4
        ups.append(S.Update(0, "box", block=view, offset=off, extent=ext, alpha=1.0 / k, nbytes=nb))
    for fac, a in WS.rank1_pairs(dims, args.config4_pairs, seed=43):
        f = [torch.from_numpy(v).cuda() for v in fac]
        ups.append(S.Update(0, "rank1", factors=f, alpha=a, nbytes=sum(v.size * 8 for v in fac)))
    order = WS.rng(1).permutation(len(ups))
    ups = [ups[i] for i in order]
    for u in ups:
        u.arrival = 0.0
    spec = S.StreamSpec(WS.T5, dims, 24, 12, variant="ttnn", dtype="f32", seed=7)
    final = {}

    def on_close(sid, plan, cores):
        That = plan.reconstruct(cores)
        final["err"] = P.diff_norms(That, T64)
        del That

    srv = S.Server(budget_bytes=1 << 40, max_batch=1, max_inflight=2, assemble_every=256, on_close=on_close)
    srv.open_stream(0, spec)
    st = srv.run(ups)
    e2, n2 = final["err"]
    boxes = sum(1 for u in ups if u.kind == "box")
    keep = ("updates", "wall_s", "updates_per_s", "ingest_GBps", "device_p50_ms", "device_p99_ms",
            "box_device_p50_ms", "box_device_p99_ms", "rank1_device_p50_ms", "rank1_device_p99_ms",
            "plan_create_ms_max")
    out = {"workload": f"{n}^5 FP32 TTN (edge ranks 16) on (((1,2),3),(4,5)), TTNN, r=24, p=12; {boxes} boxes of "
                       f"{k} two-piece tilings (8..56 per mode, read in place, alpha 1/{k}) + {len(ups) - boxes} "
                       "rank-1 terms (cancelling pairs), random order, cores every 256 updates, via the server",
           **{f: st[f] for f in keep if f in st}, "approx_rel_error": (e2 / n2) ** 0.5}
    out["update_p50_ms"], out["update_p99_ms"] = out.get("device_p50_ms"), out.get("device_p99_ms")
    del ups, X, V, T64
    torch.cuda.empty_cache()
    return out


def host_info():
    """CPU model, usable cores and the BLAS libraries NumPy runs on (with their threads)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        for p in threadpool_info():
            if p.get("user_api") == "blas":
                blas.append(f"{p.get('internal_api')} {p.get('version')} x{p.get('num_threads')}")
    except Exception:                      # threadpoolctl missing or failing: report nothing
        pass
    return {"cpu_model": model, "cores": len(os.sched_getaffinity(0)), "blas": ", ".join(blas) or "unknown"}


def cpu_baseline(T, variant, rank, over, seed=1):
    """The FP64 oracle, as it stands, on the whole headline workload (the 128^4 tensor,
    one sketch of the whole tensor and its recovery), phases timed separately: DRM
    generation, the sketch phase (every R_t and the root sketch), the epilogue plus
    recovery phase (Omega_t, Psi_t, QR, eps-pseudo-inverse, cores), and the dense
    reconstruction.  `value` is the tensor's FP64 bytes over the sketch time."""
    import numpy as np
    import oracle as O
    tree = O.Tree(O.T4, T.shape, rank, over)
    ph = {}
    tic = time.perf_counter()
    D = O.DRMs(tree, seed, variant)
    ph["drm_s"] = time.perf_counter() - tic
    tic = time.perf_counter()
    sk = O.sketch(T, tree, D, variant)
    ph["sketch_s"] = time.perf_counter() - tic
    tic = time.perf_counter()
    cores, _ = O.assemble(sk, tree)
    ph["assemble_s"] = time.perf_counter() - tic
    tic = time.perf_counter()
    That = O.reconstruct(cores, tree)
    ph["reconstruct_s"] = time.perf_counter() - tic
    err = float(np.linalg.norm(That - T) / np.linalg.norm(T))
    info = host_info()
    return {"value": T.size * 8 / ph["sketch_s"] / 1e9, "unit": "GB/s", "cores": info["cores"],
            "kind": "oracle",
            "sample": f"whole workload: {variant} r={rank} p={over} on the 128^4 tensor, FP64 NumPy (DRM entries "
                      f"in C); value = tensor bytes / sketch time; approximation error {err:.3g}",
            "phases_s": {k[:-2]: round(v, 3) for k, v in ph.items()},
            "cpu_model": info["cpu_model"], "blas": info["blas"]}


# per-configuration summary in the final record: one list per configuration, in this order
SUMMARY_FIELDS = ("ms_per_step", "sweep_kernel_ms_avg", "sweep_roofline_frac", "approx_rel_error",
                  "sketch_rel_error_vs_fp64_path_max")


def roofline_of(flops, nbytes, ms, dtype):
    """Bound (the larger of the HBM and MFMA times at peak), achieved rate and fraction."""
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = flops / (MFMA_PEAK_TFLOPS[dtype] * 1e12)
    if t_mfma > t_hbm:
        ach = flops / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": MFMA_PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
                "frac": ach / MFMA_PEAK_TFLOPS[dtype]}
    ach = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}


def compact_line(args, key, results, cpu=None, serving=None, hilbert=None, copy=None, traffic=None, rounding=None,
                 pipelined=None, orders=None):
    """The one JSON record the benchmark prints last (kept well under 4 KB): headline
    value, the sweep kernel's roofline and a step-level one, the CPU baseline and a
    short summary of every other measured configuration."""
    hv, hd = key.split(":")[:2]
    head = results[key]
    kind_name = {0: "whole update", 1: "sttnn_t4_kernel (one-pass STTNN sweep)",
                 2: "sttnn_t4_kernel (one-pass STTNN sweep writing Z1; R_2 by a streaming kernel)",
                 3: "sttnn_t4_kernel in TTNN mode (R_A, Z_A, R_1, R_B)"}[head["sweep_kind"]]
    roof = roofline_of(head["sweep_flops"], head["sweep_algorithmic_bytes"], head["sweep_kernel_ms_avg"], hd)
    roof["traffic"] = traffic
    roof["kernel"] = f"{kind_name}; HIP events on the launch stream"
    roof["algorithmic_bytes_per_launch"] = head["sweep_algorithmic_bytes"]
    roof["flops_per_launch"] = head["sweep_flops"]
    step = roofline_of(head["flops"], head["algorithmic_bytes"], head["ms_per_step"], hd)
    step["what"] = "whole step (sketch update + FP64 epilogue + assembly) vs all sketch-phase flops and compulsory bytes"
    roof["step"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in step.items()}
    for k in ("achieved", "frac"):
        roof[k] = round(roof[k], 4)
    summary = {"fields": list(SUMMARY_FIELDS)}
    for k, r in results.items():
        summary[k] = [float(f"{r[s]:.3g}") if r.get(s) is not None else None for s in SUMMARY_FIELDS]
    line = {
        "metric": METRIC,
        "value": round(head["ingest_GBps"], 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hd,
        "data": "synthetic",
        "config": {"workload": f"{hv.upper()} one-pass sketch + FP64 assembly, {args.n}^4 on ((1,2),(3,4)), "
                               f"TTN ranks 24, 0.8^k spectra, 1e-4 noise, r={args.rank}, p={args.over}",
                   "variant": hv, "n": args.n, "rank": args.rank, "oversample": args.over},
        "roofline": roof,
        "cpu_baseline": cpu,
        "results": summary,
    }
    if copy is not None:
        line["copy_GBps_read_plus_write"] = round(copy["GBps_read_plus_write"], 1)
    if serving is not None:
        fields = ("updates_per_s", "ingest_GBps", "p50_ms", "p99_ms", "box_device_p99_ms", "rank1_device_p99_ms",
                  "approx_rel_error")
        sv = {"fields": list(fields)}
        for name in ("batched_f32_closed_loop", "batched_f32_poisson", "fp64_one_per_launch_closed_loop",
                     "fp64_one_per_launch_poisson", "single_stream_f32"):
            s = serving.get(name)
            if s:
                sv[name] = [float(f"{s[f]:.4g}") if s.get(f) is not None else None for f in fields]
        line["serving"] = sv
    if hilbert is not None:
        line["hilbert_6d"] = {c: f"r{rows[-1]['rank']} err {rows[-1]['mean_rel_error']:.2g}"
                              for c, rows in hilbert["curves"].items()}
    if rounding is not None:
        rr = {"workload": rounding["workload"]}
        for k, v in rounding["rows"].items():
            rr[k] = f"{v['ms_per_rounding']:.3g} ms, err {v['mean_rel_error']:.2g}"
        if rounding.get("cpu_baseline"):
            rr["cpu_oracle_ms"] = round(rounding["cpu_baseline"]["value"], 1)
        line["ttn_rounding"] = rr
    if pipelined:
        line["two_plans_in_turn_ms_per_step"] = {k: round(v, 4) for k, v in pipelined.items()}
    if orders:
        # ms per step, [lexicographic, searched] visiting order
        line["sttnn_order_ms"] = {k.split("_r")[0]: [round(v[o]["ms_per_step"], 3) if o in v else None
                                                   for o in ("lexicographic", "searched")]
                                  for k, v in orders.items()}
    return line


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the sketch path runs on a single GPU", file=sys.stderr)
        sys.exit(2)

    if args.hilbert_only:
        print(json.dumps(hilbert_bench(args)))
        return
    if args.rounding_only:
        print(json.dumps(rounding_bench(args)))
        return
    if args.order_only:
        print(json.dumps(order_bench(args)))
        return
    if args.rank1_only:
        print(json.dumps(rank1_bench(args)))
        return

    import numpy as np
    import torch
    from workloads import synth as W

    t_gen = time.perf_counter()
    T = W.config2_tensor(n=args.n)
    T_dev64 = torch.from_numpy(np.ascontiguousarray(W.flat_colmajor(T))).cuda()
    t_gen = time.perf_counter() - t_gen
    dims = T.shape
    results = {}

    def measure(variant, dtype, rank, over, key, ref=None):
        """One configuration; keeps its sketches when it is the FP64 reference (ref is
        None and dtype f64), else reports their errors against `ref`."""
        r = run_gpu(args, T_dev64, variant, dtype, rank, over, keep_sketches=True)
        sk = r.pop("_sketches")
        if ref is not None:
            per = sketch_rel_errors(sk, ref)
            r["sketch_rel_error_vs_fp64_path"] = per
            r["sketch_rel_error_vs_fp64_path_max"] = max(per.values())
        flops, drm_entries, N = work_counts(dims, rank, over, variant)
        r["rank"], r["oversample"] = rank, over
        r["flops"] = flops
        r["algorithmic_bytes"] = N * ESIZE[dtype] + drm_entries * ESIZE[dtype]
        r["ingest_GBps"] = N * ESIZE[dtype] / (r["ms_per_step"] * 1e-3) / 1e9
        r["sketch_GBps_algorithmic"] = r["algorithmic_bytes"] / (r["sketch_ms_avg"] * 1e-3) / 1e9
        r["sketch_TFLOPs"] = flops / (r["sketch_ms_avg"] * 1e-3) / 1e12
        kf, kb = sweep_counts(dims, rank, over, variant, dtype, r["sweep_kind"])
        r["sweep_flops"] = kf
        r["sweep_algorithmic_bytes"] = kb
        r["sweep_GBps"] = kb / (r["sweep_kernel_ms_avg"] * 1e-3) / 1e9
        r["sweep_TFLOPs"] = kf / (r["sweep_kernel_ms_avg"] * 1e-3) / 1e12
        rf = roofline_of(kf, kb, r["sweep_kernel_ms_avg"], dtype)
        r["sweep_roofline_frac"] = rf["frac"]
        results[key] = r
        print(f"# {key}: {r['ms_per_step']:.3f} ms/step, sweep {r['sweep_kernel_ms_avg']:.3f} ms "
              f"({rf['bound']} frac {rf['frac']:.3f})", file=sys.stderr, flush=True)
        return sk

    # FP64 first in each variant: its sketches are the reference the other dtypes'
    # sketch errors are reported against (the FP64 path is itself held to 1e-10 of the
    # FP64 oracle by the GPU parity tests; the oracle is too slow at this size)
    dtypes = args.dtypes.split(",")
    dtypes = (["f64"] if "f64" in dtypes else []) + [d for d in dtypes if d != "f64"]
    for variant in args.variants.split(","):
        ref = None
        for dtype in dtypes:
            sk = measure(variant, dtype, args.rank, args.over, f"{variant}:{dtype}", ref)
            if dtype == "f64":
                ref = sk
    # the precision workload's other sketch ranks: STTNN BF16 against FP64, p = r/2
    for rr in [int(x) for x in args.precision_ranks.split(",") if x]:
        ref = measure("sttnn", "f64", rr, rr // 2, f"sttnn:f64:r{rr}")
        measure("sttnn", "bf16", rr, rr // 2, f"sttnn:bf16:r{rr}", ref)

    key = args.headline if args.headline in results else next(iter(results))
    pipelined = {}
    if not args.no_pipeline:
        for k in ("sttnn:f32", "sttnn:bf16"):
            if k in results:
                v, d = k.split(":")
                pipelined[k] = run_pipelined(args, T_dev64, v, d)
                print(f"# {k} two plans in turn: {pipelined[k]:.3f} ms/step", file=sys.stderr, flush=True)
    copy = copy_rate()

    hilbert = None
    if not args.no_hilbert:
        hilbert = hilbert_bench(args)
    orders = None
    if not args.no_order:
        orders = order_bench(args)
    rounding = None
    if not args.no_rounding:
        rounding = rounding_bench(args)
        if not args.no_cpu:
            rounding["cpu_baseline"] = cpu_baseline_rounding(args)
    serving = None
    if not args.no_serve:
        del T_dev64
        torch.cuda.empty_cache()
        serving = serving_bench(args)
        serving["single_stream_f32"] = serving_single(args)
        print(f"# serving single stream: {serving['single_stream_f32']['updates_per_s']:.0f} updates/s",
              file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        hv = key.split(":")[0]
        cpu = cpu_baseline(T, hv, args.rank, args.over)
        print(f"# cpu baseline: {json.dumps(cpu['phases_s'])}", file=sys.stderr, flush=True)

    line = compact_line(args, key, results, cpu=cpu, serving=serving, hilbert=hilbert, copy=copy,
                        traffic=measured_traffic(key), rounding=rounding, pipelined=pipelined, orders=orders)
    detail = {"line": line, "results": results, "copy_calibration": copy, "serving": serving,
              "hilbert_6d": hilbert, "ttn_rounding": rounding, "two_plans_in_turn_ms_per_step": pipelined,
              "sttnn_visiting_order": orders,
              "input_generation_s": t_gen}
    if args.detail:
        d = os.path.dirname(os.path.abspath(args.detail))
        os.makedirs(d, exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump(detail, f, indent=1, default=float)
    sys.stdout.flush()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
