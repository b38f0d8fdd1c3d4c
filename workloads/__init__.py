"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only draws random numbers and builds input tensors; it contains none
of the sketching or recovery arithmetic and imports neither the oracle nor the
product library.
"""

from .synth import (
    tree_spec_nodes, gaussian_ttn_cores, decaying_ttn_cores, ttn_dense,
    add_relative_noise, config1_tensor, config2_tensor, small_random_ttn,
    flat_colmajor, rng,
)
