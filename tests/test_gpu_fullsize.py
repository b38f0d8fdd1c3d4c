"""Parity at the full benchmark size (128^4 on ((1,2),(3,4)), r = 32, p = 16; STTNN BF16
also at r = 16 and 64 with p = r / 2), in the launch configuration the benchmark times
(one whole-tensor update: the fused sweep, its reduction, the streaming R_2 or the
TTNN leaf passes, the chains on Z_A).  Every sketch the plan holds (R_t, Omega_t,
Psi_t and the root Psi) is compared element by element with the full oracle sketch of
exactly the values the GPU consumed: with FP64 DRMs at the dtype tolerance, and, for
FP32 / BF16, with the same rounded DRMs at the arithmetic tolerance."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL, TOL_ARITH, failures, sketch_errors, to_device

pytestmark = pytest.mark.gpu

DIMS, SEED = (128, 128, 128, 128), 1


@pytest.fixture(scope="module")
def T():
    # logical T[i1, i2, i3, i4] stored column-major (mode 1 fastest)
    return np.random.default_rng(0).standard_normal(DIMS[::-1]).T


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    return P


_DEV = {}


def device_copy(T, dtype):
    """The tensor on the device in `dtype` and the values it holds (one dtype kept)."""
    if dtype not in _DEV:
        _DEV.clear()
        torch.cuda.empty_cache()
        _DEV[dtype] = to_device(T, dtype)
    return _DEV[dtype]


CASES = [(v, d, 32) for v in ("sttnn", "ttnn") for d in ("bf16", "f32", "f64")] + \
        [("sttnn", "bf16", 16), ("sttnn", "bf16", 64)]


@pytest.mark.parametrize("variant,dtype,r", CASES, ids=[f"{v}-{d}-r{r}" for v, d, r in CASES])
def test_fullsize_parity(P, T, variant, dtype, r):
    p = r // 2
    dev, consumed = device_copy(T, dtype)
    print(f"full-size parity {variant} {dtype} r={r}", flush=True)
    plan = P.Plan(O.T4, DIMS, r, p, variant=variant, dtype=dtype, seed=SEED)
    plan.update(dev)
    torch.cuda.synchronize()
    tree = O.Tree(O.T4, DIMS, r, p)
    sk = O.sketch(consumed, tree, O.DRMs(tree, SEED, variant), variant)
    errs = sketch_errors(plan, tree, sk)
    bad = failures(errs, TOL[dtype])
    assert not bad, bad
    if dtype != "f64":
        skr = O.sketch(consumed, tree, O.DRMs(tree, SEED, variant, dtype), variant)
        errs = sketch_errors(plan, tree, skr)
        bad = failures(errs, TOL_ARITH[dtype])
        assert not bad, bad
    plan.close()


@pytest.fixture(scope="module")
def T2():
    """The 128^4 benchmark tensor: a TTN with edge ranks 24 and 0.8^k spectra, unit RMS
    plus N(0, 1e-4^2) noise."""
    from workloads import synth as W
    return W.config2_tensor(n=128)


@pytest.mark.parametrize("variant", ["sttnn", "ttnn"])
@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_fullsize_error_matches_oracle_on_consumed_values(P, T2, variant, dtype):
    """Approximation error of the benchmark tensor: the GPU path against the oracle run
    on the same consumed (rounded) values with the same rounded DRMs, within 1%.  In
    BF16 both sit near 1.4e-2: the storage rounding (1.7e-3 relative) acts as input
    noise, which the method amplifies about ninefold on this tensor, as it does the
    1e-4 noise of the FP64 workload (error 1.0e-3)."""
    from workloads import synth as W
    dev, consumed = to_device(T2, dtype)
    plan = P.Plan(O.T4, DIMS, 32, 16, variant=variant, dtype=dtype, seed=SEED)
    plan.update(dev)
    cores = plan.assemble()
    ref = torch.from_numpy(np.ascontiguousarray(W.flat_colmajor(T2))).cuda()
    e2, n2 = P.diff_norms(plan.reconstruct(cores), ref)
    e_gpu = float(np.sqrt(e2 / n2))
    del ref, dev
    _DEV.clear()
    tree = O.Tree(O.T4, DIMS, 32, 16)
    oc, _ = O.assemble(O.sketch(consumed, tree, O.DRMs(tree, SEED, variant, dtype), variant), tree)
    e_or = float(np.linalg.norm(O.reconstruct(oc, tree) - T2) / np.linalg.norm(T2))
    plan.close()
    assert abs(e_gpu - e_or) <= 0.01 * e_or, (e_gpu, e_or)
