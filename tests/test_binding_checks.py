"""Argument checks of the Python binding that run before any library call: a block
that is not contiguous, has the wrong size or dtype, or lives on the host is refused
with TypeError / ValueError (exceptions, not asserts, so python -O keeps them).  No GPU
needed: every refusal happens before the device is touched."""
import pytest
import torch

import paper_2412_06111_amd as P
from paper_2412_06111_amd._lib import check_block


def test_refuses_non_contiguous_block():
    blk = torch.zeros(6, 4, dtype=torch.float32).t()          # a transposed view, no strides given
    with pytest.raises(ValueError, match="contiguous"):
        check_block(blk, torch.float32, (6, 4), 2)


def test_views_of_the_box_shape_are_read_with_their_strides():
    from paper_2412_06111_amd._lib import view_strides
    base = torch.zeros(5, 7, 9, dtype=torch.float32)            # (n3, n2, n1): column-major 9 x 7 x 5
    view = base[1:4, 2:6, 3:8]                                  # box extents (5, 4, 3) at offset (3, 2, 1)
    assert view_strides(view, (5, 4, 3), 3) == (1, 9, 63)
    assert view_strides(base, (9, 7, 5), 3) is None             # contiguous: packed
    assert view_strides(view.reshape(-1) if view.is_contiguous() else torch.zeros(60), (5, 4, 3), 3) is None


def test_refuses_mis_sized_block():
    with pytest.raises(ValueError, match="entries"):
        check_block(torch.zeros(23, dtype=torch.float32), torch.float32, (6, 4), 2)


def test_refuses_wrong_order_and_dtype():
    with pytest.raises(ValueError, match="modes"):
        check_block(torch.zeros(24, dtype=torch.float32), torch.float32, (6, 4), 3)
    with pytest.raises(TypeError, match="dtype"):
        check_block(torch.zeros(24, dtype=torch.float64), torch.float32, (6, 4), 2)
    with pytest.raises(TypeError):
        check_block([0.0] * 24, torch.float32, (6, 4), 2)


def test_refuses_host_block():
    with pytest.raises(TypeError, match="CUDA"):
        check_block(torch.zeros(24, dtype=torch.float32), torch.float32, (6, 4), 2)


def test_strided_view_bounds():
    base = torch.zeros(10, 8, dtype=torch.float32)            # storage of 80 entries
    view = base[2:8, 1:5]                                      # rows of 8: strides (1, 8) over (4, 6)
    with pytest.raises(TypeError, match="CUDA"):               # in bounds: only the device is wrong
        check_block(view, torch.float32, (4, 6), 2, strides=(1, 8))
    with pytest.raises(ValueError, match="outside"):
        check_block(view, torch.float32, (4, 9), 2, strides=(1, 8))
    with pytest.raises(ValueError, match="outside"):
        check_block(view, torch.float32, (4, 6), 2, strides=(1, -8))


def test_update_batched_checks_before_marshalling():
    class FakePlan:                                            # only the fields the checks read
        torch_dtype, d, handle = torch.float32, 2, None
    with pytest.raises(ValueError, match="contiguous"):
        P.update_batched([(FakePlan(), torch.zeros(48)[::2], (6, 4), (0, 0), 1.0)])
    with pytest.raises(ValueError, match="entries"):
        P.update_batched([(FakePlan(), torch.zeros(5), (6, 4), (0, 0), 1.0)])
