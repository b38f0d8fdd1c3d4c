"""C-ABI checks that need no GPU: every function declared in include/ttnn.h is
exported by libttnn.so, and host-side validation rejects bad problems with the
documented status before anything touches the device."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "ttnn.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ttnn_[a-z0-9_]+)\s*\(", src)))


def test_header_functions_exported():
    from paper_2412_06111_amd import _lib
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(_lib.lib, n), n


def _problem(spec, dims, r=2, p=1, variant=0, dtype=0):
    from paper_2412_06111_amd import _lib
    par, fst, lst, modes = _lib.tree_arrays(spec)
    nn = len(par)
    arrs = ((C.c_int64 * len(dims))(*dims), (C.c_int32 * nn)(*par), (C.c_int32 * nn)(*fst),
            (C.c_int32 * nn)(*lst), (C.c_int32 * nn)(*([r] * nn)), (C.c_int32 * nn)(*([p] * nn)))
    pr = _lib.Problem(len(dims), arrs[0], nn, arrs[1], arrs[2], arrs[3], arrs[4], arrs[5], variant, dtype, 1, 0.0)
    return pr, arrs


def _create(pr):
    from paper_2412_06111_amd import _lib
    h = C.c_void_p()
    st = _lib.lib.ttnn_plan_create(C.byref(pr), None, C.byref(h))
    return st, h


@pytest.mark.parametrize("spec,dims", [
    (((1, 3), (2, 4)), (2, 2, 2, 2)),        # non-contiguous node
    (((1, 2), (3,)), (2, 2, 2, 2)),          # root misses mode 4
    (((1, 2), (2, 3, 4)), (2, 2, 2, 2)),     # overlapping children
])
def test_bad_trees_rejected(spec, dims):
    pr, keep = _problem(spec, dims)
    st, h = _create(pr)
    assert st == -2 and not h.value


def test_bad_arguments_rejected():
    from paper_2412_06111_amd import _lib
    pr, keep = _problem(((1, 2), (3, 4)), (2, 2, 2, 2), variant=7)
    assert _create(pr)[0] == -1
    pr, keep = _problem(((1, 2), (3, 4)), (2, 2, 2, 2), r=0)
    assert _create(pr)[0] == -1
    pr, keep = _problem(((1, 2), (3, 4)), (2, 0, 2, 2))
    assert _create(pr)[0] == -1
    h = C.c_void_p()
    assert _lib.lib.ttnn_plan_create(None, None, C.byref(h)) == -1
    assert b"NULL" in _lib.lib.ttnn_last_error()
    # two roots
    arr = [(C.c_int64 * 2)(2, 2), (C.c_int32 * 3)(-1, -1, 0), (C.c_int32 * 3)(0, 0, 1),
           (C.c_int32 * 3)(1, 0, 1), (C.c_int32 * 3)(1, 1, 1), (C.c_int32 * 3)(0, 0, 0)]
    pr = _lib.Problem(2, arr[0], 3, arr[1], arr[2], arr[3], arr[4], arr[5], 0, 0, 1, 0.0)
    assert _create(pr)[0] == -2
    assert _lib.lib.ttnn_status_string(-7) == b"numerical failure"


def test_footprint_estimate_without_device():
    """Host-side sizing: no allocation or launch, so it runs without a GPU."""
    import paper_2412_06111_amd as P
    spec = ((1, 2), (3, 4))
    small = P.footprint_estimate(spec, (16, 16, 16, 16), 6, 3, "ttnn", "f64")
    big = P.footprint_estimate(spec, (64, 64, 64, 64), 6, 3, "ttnn", "f64")
    bf = P.footprint_estimate(spec, (64, 64, 64, 64), 6, 3, "ttnn", "bf16")
    assert 0 < small < big and 0 < small < bf
    # the TTNN leaf X maps alone: 4 leaves x 64^3 rows x 6 columns, FP64 masters + BF16 copies
    assert bf > 4 * 64 ** 3 * 6 * (8 + 2)
    assert big > 4 * 64 ** 3 * 6 * 8


def test_footprint_estimate_rejects_bad_tree():
    import paper_2412_06111_amd as P
    with pytest.raises(P.TTNNError) as e:
        P.footprint_estimate(((1, 3), (2, 4)), (4, 4, 4, 4), 2, 1)
    assert e.value.status == -2
