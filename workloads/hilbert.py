"""The 6-D Hilbert tensor of the paper's first accuracy experiment (Sec. 8):
H(i_1, .., i_d) = 1 / (1 + i_1 + .. + i_d) with 1-based indices (so the largest
entry is 1 / (1 + d)), mode size n (20 in the paper), approximated on the index
tree of Fig. 1 with equal ranks r and oversampling p = 3.

H is symmetric under any permutation of its modes, so its column-major and
row-major flat orders coincide: the device copy is the plain row-major flattening.
"""

import numpy as np

TOY = (((1, 2), 3), 4, (5, 6))          # index tree of Fig. 1
N_PAPER, D_PAPER, P_PAPER = 20, 6, 3
RANKS_PAPER = tuple(range(2, 14))       # the ranks of the error curve


def hilbert_host(n, d=D_PAPER):
    """FP64 array with logical indexing H[i1, .., id] (0-based here: H = 1 / (d + 1 + sum))."""
    s = np.zeros((n,) * d, dtype=np.int64)
    ar = np.arange(n, dtype=np.int64)
    for k in range(d):
        shape = [1] * d
        shape[k] = n
        s = s + ar.reshape(shape)
    return 1.0 / (1.0 + d + s).astype(np.float64)


def hilbert_device(n, d=D_PAPER, device="cuda"):
    """The same values as a flat FP64 torch tensor on `device` (column-major order)."""
    import torch
    ar = torch.arange(n, dtype=torch.int64, device=device)
    s = torch.zeros((n,) * d, dtype=torch.int64, device=device)
    for k in range(d):
        shape = [1] * d
        shape[k] = n
        s += ar.view(shape)
    out = 1.0 / (s + (1 + d)).to(torch.float64)
    return out.reshape(-1)
