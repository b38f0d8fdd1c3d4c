"""The benchmark's final stdout record: valid JSON, under 4 KB, with the fields the
measurement contract asks for, for a recorded set of results as large as the default
run produces (both variants in three dtypes, the extra sketch ranks, serving, the
Hilbert curves and the CPU baseline).  No GPU needed."""
import json
import os
import sys
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _result(variant, dtype, r, kind):
    p = r // 2
    flops, drm, N = bench.work_counts((128,) * 4, r, p, variant)
    kf, kb = bench.sweep_counts((128,) * 4, r, p, variant, dtype, kind)
    ms = 1.1234567891234
    return {"ms_per_step": ms, "sketch_ms_avg": 0.912345678, "sketch_ms_min": 0.9, "sweep_kernel_ms_avg": 0.7312345,
            "sweep_kernel_ms_min": 0.72, "drm_generation_ms": 12.3456, "footprint_bytes": 2123456789,
            "sweep_kind": kind, "approx_rel_error": 1.0412345e-3, "rank": r, "oversample": p, "flops": flops,
            "algorithmic_bytes": N * bench.ESIZE[dtype] + drm * bench.ESIZE[dtype],
            "ingest_GBps": N * bench.ESIZE[dtype] / (ms * 1e-3) / 1e9, "sweep_flops": kf,
            "sweep_algorithmic_bytes": kb, "sketch_rel_error_vs_fp64_path_max": 3.41234e-3,
            "sweep_roofline_frac": 0.7471234,
            "sketch_rel_error_vs_fp64_path": {"1,2": 1e-3, "3,4": 2e-3}}


def _recorded():
    res = {}
    for v, kind in (("ttnn", 3), ("sttnn", 2)):
        for dt in ("f64", "f32", "bf16"):
            res[f"{v}:{dt}"] = _result(v, dt, 32, kind)
    for rr in (16, 64):
        res[f"sttnn:f64:r{rr}"] = _result("sttnn", "f64", rr, 2)
        res[f"sttnn:bf16:r{rr}"] = _result("sttnn", "bf16", rr, 2)
    st = {"updates": 6614, "wall_s": 0.3456789, "updates_per_s": 19123.456789, "ingest_GBps": 56.123456,
          "p50_ms": 0.71234567, "p99_ms": 83.1234567, "mean_batch": 40.1234, "box_device_p99_ms": 0.1234567,
          "rank1_device_p99_ms": 0.01234567, "approx_rel_error": 2.51234e-4}
    serving = {k: dict(st) for k in ("batched_f32_closed_loop", "batched_f32_poisson",
                                     "fp64_one_per_launch_closed_loop", "fp64_one_per_launch_poisson")}
    serving["single_stream_f32"] = {"updates_per_s": 3712.3456, "ingest_GBps": 4.2345678, "update_p50_ms": 0.1234567,
                                    "update_p99_ms": 0.1712345}
    rows = [{"rank": r, "mean_rel_error": 10.0 ** -r, "max_rel_error": 10.0 ** -r, "ms_per_approximation": 1.5,
             "ingest_GBps": 300.0} for r in range(2, 14)]
    hilbert = {"curves": {f"{v}:{d}": rows for v in ("ttnn", "sttnn") for d in ("f64", "f32")}}
    cpu = {"value": 0.0761234567, "unit": "GB/s", "cores": 16, "kind": "oracle",
           "sample": "whole workload: sttnn r=32 p=16 on the 128^4 tensor, FP64 NumPy (DRM entries in C); "
                     "value = tensor bytes / sketch time; approximation error 0.00103",
           "phases_s": {"drm": 12.345, "sketch": 6.789, "assemble": 0.012, "reconstruct": 0.345},
           "cpu_model": "AMD EPYC 9575F 64-Core Processor with a long marketing name",
           "blas": "openblas 0.3.27 x16, openblas 0.3.27 x16"}
    rounding = {"workload": "order-6 TTN, n = 500, TTN ranks 70 on the Fig. 1 tree, Khatri-Rao maps, p = 10",
                "rows": {f"{d}:r{r}": {"ms_per_rounding": 1.1912345, "mean_rel_error": 1.2345e-3}
                         for d in ("quadratic", "cubic", "exponential") for r in (16, 32, 48)},
                "cpu_baseline": {"value": 21.123456}}
    pipelined = {"sttnn:f32": 0.98512345, "sttnn:bf16": 0.62712345}
    orders = {"t4_32x512x128x128_r32_f32": {"lexicographic": {"ms_per_step": 2.82212345},
                                            "searched": {"ms_per_step": 1.62012345}},
              "hilbert6d_n20_fig1tree_r13_f64": {"lexicographic": {"ms_per_step": 1.32112345},
                                                 "searched": {"ms_per_step": 1.13212345}}}
    return res, serving, hilbert, cpu, rounding, pipelined, orders


def test_compact_line_parses_and_fits():
    res, serving, hilbert, cpu, rounding, pipelined, orders = _recorded()
    args = SimpleNamespace(steps=20, warmup=40, n=128, rank=32, over=16)
    line = bench.compact_line(args, "sttnn:f32", res, cpu=cpu, serving=serving, hilbert=hilbert,
                              copy={"GBps_read_plus_write": 4567.891}, traffic=1980000000, rounding=rounding,
                              pipelined=pipelined, orders=orders)
    text = json.dumps(line)
    assert "\n" not in text
    assert len(text) < 4096, len(text)
    back = json.loads(text)
    for f in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert f in back, f
    assert back["n_gpus"] == 1 and back["dtype"] == "f32" and back["config"]["workload"]
    roof = back["roofline"]
    for f in ("bound", "achieved", "peak", "unit", "frac", "traffic", "step"):
        assert f in roof, f
    # FP32 STTNN at r = 32 is bound by the FP32 MFMA rate, both for the kernel and the step
    assert roof["bound"] == "mfma" and roof["step"]["bound"] == "mfma"
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert set(back["cpu_baseline"]["phases_s"]) == {"drm", "sketch", "assemble", "reconstruct"}


def test_step_counts_match_the_scope_table():
    # flops and compulsory bytes of a whole sketch pass at 128^4 (BF16) against the
    # leading-order figures (the STTNN flop figures leave out the small contractions of
    # the contracted intermediates: R_B, R_3, R_4 and the chains after Z_A, under 1%)
    for variant, r, gflop, gbytes in (("ttnn", 32, 128.9, 1.079), ("sttnn", 16, 44.6, 0.619),
                                      ("sttnn", 32, 92.3, 0.726), ("sttnn", 64, 197.6, 1.018)):
        flops, drm, N = bench.work_counts((128,) * 4, r, r // 2, variant)
        assert gflop <= flops / 1e9 < gflop * 1.01, (variant, r, flops)
        assert abs((N + drm) * 2 / 1e9 - gbytes) < 0.01, (variant, r, (N + drm) * 2)
