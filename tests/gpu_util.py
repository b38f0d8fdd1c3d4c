"""Helpers shared by the GPU tests: move seeded inputs to the device, run the
oracle on exactly the values the GPU consumed, compare sketches."""
import numpy as np
import torch

import oracle as O
from workloads import synth as W

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-2}


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


def sketch_errors(plan, tree, sk):
    """Relative errors of every GPU sketch against oracle sketches `sk` (by node modes)."""
    from paper_2412_06111_amd import SK_R, SK_OMEGA, SK_PSI
    out = {}
    for n in tree.nodes:
        cid = plan.node(n.modes)
        if n.id == 0:
            out[("psi", n.modes)] = rel(plan.read_sketch(cid, SK_PSI).cpu().numpy(), sk["Psi"][0])
            continue
        out[("R", n.modes)] = rel(plan.read_sketch(cid, SK_R).cpu().numpy(), sk["R"][n.id])
        out[("omega", n.modes)] = rel(plan.read_sketch(cid, SK_OMEGA).cpu().numpy(), sk["Omega"][n.id])
        out[("psi", n.modes)] = rel(plan.read_sketch(cid, SK_PSI).cpu().numpy(), sk["Psi"][n.id])
    return out
