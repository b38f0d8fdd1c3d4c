"""Large boxes read in place (strided views of a resident tensor, at least 2^22
entries) are packed before their update: through the C ABI, single and batched, the
sketches are bitwise those of the same box passed as a packed copy, for TTNN and STTNN
in FP32 and BF16, and a whole tensor given as a strided view takes the whole-tensor
path with the bits of the packed tensor."""
import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

T4 = ((1, 2), (3, 4))
DIMS = (70, 64, 60, 50)                  # 13.4M entries
BOX = ((3, 2, 5, 4), (60, 60, 50, 40))   # (offset, extent): 7.2M entries


@pytest.fixture(scope="module")
def P():
    import paper_2412_06111_amd as P
    assert torch.cuda.is_available()
    return P


def _sketches(P, plan):
    tree = O.Tree(T4, DIMS, 4, 2)
    out = []
    for n in tree.nodes:
        cid = plan.node(n.modes)
        kinds = (P.SK_PSI,) if n.id == 0 else (P.SK_R, P.SK_OMEGA, P.SK_PSI)
        out += [plan.read_sketch(cid, k).cpu().numpy() for k in kinds]
    return out


def _same(a, b):
    return all(np.array_equal(x.view(np.uint64), y.view(np.uint64)) for x, y in zip(a, b))


@pytest.mark.parametrize("variant", ["ttnn", "sttnn"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_large_strided_box_packed(P, variant, dtype):
    print(f"pack {variant} {dtype}", flush=True)
    td = torch.float32 if dtype == "f32" else torch.bfloat16
    X = torch.randn(int(np.prod(DIMS)), dtype=torch.float32, device="cuda").to(td)
    V = X.view(*DIMS[::-1])
    off, ext = BOX
    view = V[tuple(slice(o, o + e) for o, e in zip(off[::-1], ext[::-1]))]
    assert not view.is_contiguous()
    packed = view.contiguous()
    mk = lambda: P.Plan(T4, DIMS, 4, 2, variant=variant, dtype=dtype, seed=3)
    a, b, c = mk(), mk(), mk()
    a.update(view, extent=ext, offset=off, alpha=0.5)                 # strided, packed inside
    b.update(packed, extent=ext, offset=off, alpha=0.5)
    P.update_batched([(c, view, ext, off, 0.5)])
    torch.cuda.synchronize()
    sa, sb, sc = _sketches(P, a), _sketches(P, b), _sketches(P, c)
    assert _same(sa, sb) and _same(sc, sb)
    # the whole tensor as a strided view (every mode reversed in memory is not a view
    # torch can make; a transposed-then-transposed-back copy is): use a slice of a
    # larger array so that the strides are not the packed ones
    big = torch.zeros((DIMS[3], DIMS[2], DIMS[1], DIMS[0] + 8), dtype=td, device="cuda")
    big[..., :DIMS[0]] = V
    whole = big[..., :DIMS[0]]
    assert not whole.is_contiguous()
    d, e = mk(), mk()
    d.update(whole, extent=DIMS, offset=(0,) * 4)
    e.update(X)
    torch.cuda.synchronize()
    assert _same(_sketches(P, d), _sketches(P, e))
    for p in (a, b, c, d, e):
        p.close()
