"""Seeded streams of additive updates for the serving loop.

A stream is a random tree tensor network on ((1,2),(3,4)) (mode sizes, TTN edge
ranks and sketch ranks drawn per stream), delivered as the boxes of one random
axis-aligned tiling in random order, optionally plus cancelling pairs of rank-1
terms (+u and -u with the same factors), so that the updates sum to the tensor.
Arrivals are an aggregate Poisson process over the streams.  Nothing here computes
a sketch: these are inputs only.
"""

import numpy as np

from .synth import add_relative_noise, gaussian_ttn_cores, rng, ttn_dense

T4 = ((1, 2), (3, 4))


def tiling(n, g, lo=4, hi=48):
    """Segment lengths covering range(n): draw L ~ U{lo..min(hi, rem - lo)} while
    rem > hi; the last segment is the remainder."""
    segs, rem = [], n
    while rem > hi:
        L = int(g.integers(lo, min(hi, rem - lo) + 1))
        segs.append(L)
        rem -= L
    segs.append(rem)
    return segs


def boxes(dims, g, lo=4, hi=48):
    """All boxes (offset, extent) of one random tiling, in random order."""
    cuts = [tiling(n, g, lo, hi) for n in dims]
    starts = [np.concatenate([[0], np.cumsum(c)[:-1]]).astype(int) for c in cuts]
    out = []
    for idx in np.ndindex(*[len(c) for c in cuts]):
        off = tuple(int(starts[m][i]) for m, i in enumerate(idx))
        ext = tuple(int(cuts[m][i]) for m, i in enumerate(idx))
        out.append((off, ext))
    perm = g.permutation(len(out))
    return [out[i] for i in perm]


def stream_problem(s, base_seed=1000, nlo=32, nhi=160, rlo=8, rhi=32, ranks=(16, 32)):
    """Problem of stream s: dims, TTN edge ranks (clamped to the matricisation
    sizes), sketch rank r in `ranks`, oversampling r/2."""
    g = rng(base_seed + s)
    dims = tuple(int(x) for x in g.integers(nlo, nhi + 1, size=4))
    nA, nB = dims[0] * dims[1], dims[2] * dims[3]
    ttn = {}
    for m in ((1,), (2,), (3,), (4,)):
        ttn[m] = int(min(g.integers(rlo, rhi + 1), dims[m[0] - 1]))
    e = int(min(g.integers(rlo, rhi + 1), nA, nB))
    ttn[(1, 2)] = e
    ttn[(3, 4)] = e
    r = int(ranks[int(g.integers(0, len(ranks)))])
    return {"seed": base_seed + s, "dims": dims, "ttn_ranks": ttn, "r": r, "p": r // 2}


def stream_tensor(prob, noise=1e-5):
    """Dense FP64 tensor of a stream: random TTN (N(0,1) cores), unit RMS, plus
    N(0, noise^2) entries."""
    cores = gaussian_ttn_cores(T4, prob["dims"], prob["ttn_ranks"], prob["seed"])
    T = ttn_dense(T4, prob["dims"], cores)
    return add_relative_noise(T, noise, seed=prob["seed"] + 17, unit_rms=True)


def stream_tensor_device(prob, noise=1e-5, device="cuda"):
    """The same recipe as stream_tensor, contracted on the device (torch, FP64) for
    large streams: cores drawn on the host (seeded), noise from a seeded device
    generator.  Returns the flat column-major FP64 device tensor."""
    import torch
    dims = prob["dims"]
    c = gaussian_ttn_cores(T4, dims, prob["ttn_ranks"], prob["seed"])
    t = {m: torch.from_numpy(np.asarray(v, dtype=np.float64)).to(device) for m, v in c.items()}
    U1, U2, U3, U4 = t[(1,)], t[(2,)], t[(3,)], t[(4,)]            # (n, r) each
    A, B, root = t[(1, 2)], t[(3, 4)], t[(1, 2, 3, 4)]             # (r1, r2, rA), (r3, r4, rB), (rA, rB)
    # UA[(i1, i2), a] and UB[(i3, i4), b], first index fastest, then T = UA root UB^T
    UA = torch.einsum("ix,jy,xya->jia", U1, U2, A).reshape(dims[0] * dims[1], -1)
    UB = torch.einsum("kz,lw,zwb->lkb", U3, U4, B).reshape(dims[2] * dims[3], -1)
    Tm = UA @ root @ UB.T                       # (nA, nB): column-major flat = Tm.T row-major
    flat = Tm.T.contiguous().reshape(-1)
    flat *= (flat.numel() ** 0.5) / torch.linalg.vector_norm(flat)
    g = torch.Generator(device=device)
    g.manual_seed(int(prob["seed"]) + 17)
    flat += noise * torch.randn(flat.numel(), generator=g, device=device, dtype=torch.float64)
    return flat


T5 = (((1, 2), 3), (4, 5))


def order5_tensor_device(n=64, rank=16, seed=2024, noise=1e-5, device="cuda"):
    """Single-stream serving tensor: a random TTN on (((1,2),3),(4,5)) with every edge
    rank `rank` (N(0,1) cores drawn on the host, seeded), contracted on the device in
    FP64, scaled to unit RMS, plus seeded N(0, noise^2) entries.  Returns the flat
    column-major FP64 device tensor of n^5 entries."""
    import torch
    dims = (n,) * 5
    c = gaussian_ttn_cores(T5, dims, rank, seed)
    t = {m: torch.from_numpy(np.asarray(v, dtype=np.float64)).to(device) for m, v in c.items()}
    U1, U2, U3, U4, U5 = (t[(m,)] for m in range(1, 6))               # (n, r) each
    A, Cc, E, root = t[(1, 2)], t[(1, 2, 3)], t[(4, 5)], t[(1, 2, 3, 4, 5)]
    # UA[(i1, i2), a], UC[(i1, i2, i3), c], UE[(i4, i5), e], first index fastest
    UA = torch.einsum("ix,jy,xya->jia", U1, U2, A).reshape(n * n, -1)
    UC = torch.einsum("pa,kz,azc->kpc", UA, U3, Cc).reshape(n ** 3, -1)
    UE = torch.einsum("ix,jy,xye->jie", U4, U5, E).reshape(n * n, -1)
    Tm = UC @ root @ UE.T                       # (n^3, n^2): column-major flat = Tm.T row-major
    flat = Tm.T.contiguous().reshape(-1)
    del Tm
    flat *= (flat.numel() ** 0.5) / torch.linalg.vector_norm(flat)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) + 17)
    flat += noise * torch.randn(flat.numel(), generator=g, device=device, dtype=torch.float64)
    return flat


def box_updates(T, prob, lo=4, hi=48):
    """(offset, extent, block) for the boxes of one tiling of T; block is the
    column-major flat FP64 copy of T over the box."""
    g = rng(prob["seed"] + 31)
    out = []
    for off, ext in boxes(T.shape, g, lo, hi):
        sl = tuple(slice(o, o + e) for o, e in zip(off, ext))
        blk = np.ascontiguousarray(T[sl].T).reshape(-1)
        out.append((off, ext, blk))
    return out


def cut_tilings(dims, ntilings, seed, lo=8, hi=56):
    """The boxes of `ntilings` independent two-piece tilings: in each tiling every mode
    is cut once at c ~ U{lo..hi} (pieces [0, c) and [c, n)), which gives 2^d boxes with
    extents in [lo, hi] when n - hi >= lo.  Returns (offset, extent) per box."""
    g = rng(seed)
    out = []
    for _ in range(ntilings):
        cuts = [int(g.integers(lo, hi + 1)) for _ in dims]
        segs = [((0, c), (c, n - c)) for c, n in zip(cuts, dims)]
        for idx in np.ndindex(*([2] * len(dims))):
            out.append((tuple(segs[m][i][0] for m, i in enumerate(idx)),
                        tuple(segs[m][i][1] for m, i in enumerate(idx))))
    return out


def rank1_pairs(dims, npairs, seed):
    """npairs cancelling pairs (factors, +1) and (factors, -1), factors N(0,1)."""
    g = rng(seed)
    out = []
    for _ in range(npairs):
        f = [g.standard_normal(n) for n in dims]
        out.append((f, 1.0))
        out.append((f, -1.0))
    return out


def poisson_arrivals(n, rate, seed):
    """n arrival times (seconds) of a Poisson process of the given rate."""
    g = rng(seed)
    return np.cumsum(g.exponential(1.0 / rate, size=n))
