"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only generates *inputs*: cell geometry, atom positions, the
species parameter table and seeded random start blocks.  It holds none of the
method's arithmetic (no stencil weights, no potentials on the grid, no atomic
functions, no solver steps); each consumer computes those itself.
"""
from .tio2 import (  # noqa: F401
    CONFIG_NAMES,
    make_config,
    random_block,
    random_vector,
    start_seed,
    lanczos_seed,
    initial_occupation_diag,
    with_kpoints,
    batch_cells,
    species_table,
    mlp_init_params,
)
