"""GPU parity of the MFMA forms of the whole-tensor contractions on shapes beyond the
order-4 sweep, through the C ABI.  Order-3 tensor 20 x 8 x 32768 (5.2M entries, large
enough for the MFMA forms) on ((1,2),3):

* row-contiguous right sketches (nodes that start at mode 1, where the contraction
  index is the slow one): node {1} (20 rows: one row block, three of its four waves
  past n), node {1,2} (160 rows: a second, ragged row block); FP64 / FP32;
* contiguous right sketches with short l-runs: node {2} (L = 20, 8 rows), and node
  {3} (L = 160, full row blocks);
* Y^T of a group at mode 1 applied to the raw tensor (the root sketch's first
  contraction, and STTNN's reuse prefixes), as the contiguous form with the
  contraction along the group's modes;

r = 6 (one column block) and 17 (two), against the FP64 oracle on the consumed
values, elementwise within the dtype tolerance (BF16 takes the forms its 16-byte
vectors allow)."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import TOL, failures, sketch_errors, to_device

pytestmark = pytest.mark.gpu

DIMS, SPEC = (20, 8, 32768), ((1, 2), 3)


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def tensor():
    return np.random.default_rng(19).standard_normal(DIMS)


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dtype,r", [("f64", 6), ("f64", 17), ("f32", 17), ("bf16", 17)])
def test_row_contiguous_right_sketch(P, tensor, variant, dtype, r):
    dev, consumed = to_device(tensor, dtype)
    plan = P.Plan(SPEC, DIMS, r, 3, variant=variant, dtype=dtype, seed=13)
    plan.update(dev)
    tree = O.Tree(SPEC, DIMS, r, 3)
    sk = O.sketch(consumed, tree, O.DRMs(tree, 13, variant), variant)
    errs = sketch_errors(plan, tree, sk)
    plan.close()
    bad = failures(errs, TOL[dtype])
    assert not bad, (bad, errs)


# Few rows (node {2} with n_t <= 32): the 32-row tile that takes four steps a stage and
# splits each over the waves.  (18, 8, 30030): L = 18, K = 540540, not a multiple of the
# four-step stage, so the last stage is masked vector by vector (FP64; FP32 / BF16 vectors
# do not fit an l-run of 18).  (16, 24, 11000): L = 16, 24 rows (the second row block
# ragged); whole stages in FP64 / FP32, a masked last stage in BF16.
# STTNN on (20, 16, 32770) and (20, 40, 16384): node {2} is sketched on T x_1 Y_1^T, an
# FP64 intermediate whose l-run is k_1 = 9 (odd), so FP64 vectors straddle runs and the
# tensor operand is loaded value by value (few rows with a masked last stage; 40 rows).
FEW = [((18, 8, 30030), "f64"), ((16, 24, 11000), "f64"), ((16, 24, 11000), "f32"), ((16, 24, 11000), "bf16"),
       ((20, 16, 32770), "f64"), ((20, 40, 16384), "f64")]


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dims,dtype", FEW, ids=[f"{d[0]}x{d[1]}x{d[2]}-{t}" for d, t in FEW])
def test_few_rows_right_sketch(P, variant, dims, dtype):
    T = np.random.default_rng(23).standard_normal(dims)
    dev, consumed = to_device(T, dtype)
    plan = P.Plan(SPEC, dims, 6, 3, variant=variant, dtype=dtype, seed=29)
    plan.update(dev)
    tree = O.Tree(SPEC, dims, 6, 3)
    sk = O.sketch(consumed, tree, O.DRMs(tree, 29, variant), variant)
    errs = sketch_errors(plan, tree, sk)
    plan.close()
    bad = failures(errs, TOL[dtype])
    assert not bad, (bad, errs)
