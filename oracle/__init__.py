"""FP64 CPU oracle of the tree tensor network Nystrom method (TTNN) and its
sequential variant (STTNN).

TEST INFRASTRUCTURE ONLY.  Plain, slow, NumPy float64 code written from the paper
("Randomized algorithms for streaming low-rank approximation in tree tensor
network format", Bucci and Verzella): Sec. 3 (definitions), Sec. 4 (TTNN sketch and
recovery phases, Alg. 2), Sec. 5 (STTNN), Sec. 6 (error bounds).  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it; the product
library never does, and this package imports nothing from the product.

Pins (tests/test_oracle_*.py): Philox known-answer vectors, closed-form ln/cos
accuracy and Gaussian moments, Def. 2 unfolding by its index formula, projector
form of the approximant by explicit Kronecker products, exact recovery of tensors
of TTN rank <= r, linearity, reduction to stabilised generalised Nystrom for an
order-2 tree and to MLN for a Tucker tree, Lemma 2 / Lemma 3 inequalities and the
expected bound of Theorem 2.  Parity unpinned: none of the functions exported
here; the STTNN set S_t reading is pinned by the nine panels of Fig. 5, and the sets
of other visiting orders by the relabelling to the lexicographic order of a tree with
its modes renumbered.
"""

from .tree import Tree, TreeError, TOY, T4, T5
from .drm import gaussian, philox4x32_10, rounded, bf16_bits, bf16_to_f64
from .drm import drm as drm_matrix
from .sketch import DRMs, sketch, sketch_update, unfold, fold, group_product
from .recover import assemble, reconstruct, core_shape, qr_signed, eps_pinv, DEFAULT_EPS_FACTOR

__all__ = [
    "Tree", "TreeError", "TOY", "T4", "T5",
    "gaussian", "drm_matrix", "philox4x32_10", "rounded", "bf16_bits", "bf16_to_f64",
    "DRMs", "sketch", "sketch_update", "unfold", "fold", "group_product",
    "assemble", "reconstruct", "core_shape", "qr_signed", "eps_pinv", "DEFAULT_EPS_FACTOR",
]
