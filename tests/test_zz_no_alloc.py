"""The allocation-free entry point (ttnn_diff_norms_noalloc) against ttnn_diff_norms,
through the C ABI: the same kernels in the same order, so the two sums agree bit for
bit.  Two calls in a row, the second on a smaller input, each dtype: the static
scratch keeps the previous call's partials, and every partial is rewritten."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_noalloc_equals_diff_norms_twice(dtype):
    import paper_2412_06111_amd as P
    from paper_2412_06111_amd import _lib
    L = _lib.lib
    L.ttnn_diff_norms_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    L.ttnn_diff_norms_noalloc.restype = C.c_int
    code = {torch.float64: P.F64, torch.float32: P.F32, torch.bfloat16: P.BF16}[dtype]
    g = torch.Generator(device="cuda").manual_seed(7)
    stream = _lib.stream_ptr()
    for n in (3_000_001, 12_345):                       # the second call is smaller
        b = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
        a = (b + 1e-3 * torch.randn(n, generator=g, device="cuda", dtype=torch.float64)).to(dtype)
        want = P.diff_norms(a, b)                        # allocating, synchronous entry point
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        st = L.ttnn_diff_norms_noalloc(C.c_void_p(a.data_ptr()), code, C.c_void_p(b.data_ptr()), n,
                                       C.c_void_p(out.data_ptr()), stream)
        assert st == 0, L.ttnn_last_error()
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), np.array(want, dtype=np.float64).view(np.uint64)), (n, got, want)
        # and the sums themselves against a plain FP64 evaluation on the host
        a64, b64 = a.double().cpu().numpy(), b.cpu().numpy()
        assert abs(got[0] - np.sum((a64 - b64) ** 2)) <= 1e-10 * np.sum((a64 - b64) ** 2)
        assert abs(got[1] - np.sum(b64 ** 2)) <= 1e-10 * np.sum(b64 ** 2)


def test_noalloc_rejects_bad_arguments():
    from paper_2412_06111_amd import _lib
    L = _lib.lib
    L.ttnn_diff_norms_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert L.ttnn_diff_norms_noalloc(None, 0, C.c_void_p(x.data_ptr()), 4, C.c_void_p(x.data_ptr()), None) == -1
    assert L.ttnn_diff_norms_noalloc(C.c_void_p(x.data_ptr()), 9, C.c_void_p(x.data_ptr()), 4,
                                     C.c_void_p(x.data_ptr()), None) == -1
