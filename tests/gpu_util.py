"""Helpers shared by the GPU tests: move seeded inputs to the device, run the
oracle on exactly the values the GPU consumed, compare sketches."""
import numpy as np
import torch

import oracle as O
from workloads import synth as W

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-2}
# against an oracle fed the same rounded DRMs the GPU uses (arithmetic error only:
# FP32 accumulation of exact FP32 / BF16 products, FP64 across chunks)
TOL_ARITH = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-5}
# entry-wise bound, relative to the RMS entry of the reference: a factor over the
# Frobenius tolerance (the largest of 10^3..10^6 entries of a spread-out error sits a
# few times above its RMS), far below the O(1) that a wrong tile or tail row shows
MAX_FACTOR = 10.0


def to_device(T, dtype):
    """Logical numpy tensor -> flat column-major CUDA tensor of `dtype`, plus the
    float64 logical numpy tensor holding exactly the values stored on the device."""
    flat = np.ascontiguousarray(W.flat_colmajor(np.asarray(T, dtype=np.float64)))
    t64 = torch.from_numpy(flat)
    if dtype == "f64":
        dev = t64.cuda()
    elif dtype == "f32":
        dev = t64.to(torch.float32).cuda()
    else:
        dev = t64.to(torch.float32).to(torch.bfloat16).cuda()
    back = dev.double().cpu().numpy()
    consumed = back.reshape(tuple(reversed(T.shape))).T
    return dev, consumed


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def errs2(a, b):
    """(relative Frobenius error, largest entry error / RMS entry of b) of a against b."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    rms = nb / np.sqrt(max(b.size, 1))
    d = np.abs(a - b)
    return (float(np.linalg.norm(a - b) / max(nb, 1e-300)), float(d.max() / max(rms, 1e-300)) if d.size else 0.0)


def failures(errs, tol):
    """The entries of errs (key -> (frobenius, max/rms)) that break tol or MAX_FACTOR * tol."""
    return {k: v for k, v in errs.items() if not (v[0] <= tol and v[1] <= MAX_FACTOR * tol)}


def sketch_errors(plan, tree, sk):
    """Per GPU sketch (R_t, Omega_t, Psi_t, root Psi) against the oracle sketches `sk`,
    element by element: (relative Frobenius error, max |difference| / RMS entry)."""
    from paper_2412_06111_amd import KR, SK_R, SK_OMEGA, SK_PSI
    out = {}
    for n in tree.nodes:
        cid = plan.node(n.modes)
        if n.id == 0:
            out[("psi", n.modes)] = errs2(plan.read_sketch(cid, SK_PSI).cpu().numpy(), sk["Psi"][0])
            continue
        if plan.variant != KR or n.is_leaf:          # structured plans keep R_t of leaves only
            out[("R", n.modes)] = errs2(plan.read_sketch(cid, SK_R).cpu().numpy(), sk["R"][n.id])
        out[("omega", n.modes)] = errs2(plan.read_sketch(cid, SK_OMEGA).cpu().numpy(), sk["Omega"][n.id])
        out[("psi", n.modes)] = errs2(plan.read_sketch(cid, SK_PSI).cpu().numpy(), sk["Psi"][n.id])
    return out
