"""Seeded synthetic tensor networks shared by the oracle, the tests and the benchmark.

This package only *builds inputs*: lattice geometry, site tensors drawn from
seeded generators, and the physical constructions the paper benchmarks on
(Appendix A: Ising, AKLT and random tensors).  It contains none of the
expansion's arithmetic (no message passing, projectors, clusters or sums), so
the oracle and the GPU path can both consume it without sharing method code.
"""

from .networks import (  # noqa: F401
    Network,
    lattice_2d,
    lattice_3d,
    ising_2d,
    ising_3d,
    random_2d,
    random_3d,
    aklt_2d,
    ring_network,
    chain_network,
    grid_from_tensors,
    apply_random_gauge,
    config1_network,
    config1_betas,
    config2_network,
    config3_ising_network,
    config3_aklt_network,
    config4_request,
    config4_arrivals,
    config5_network,
    ISING_BETA_C,
    bond_index,
    small_network,
    double_loop_partitions,
    grid3_single_partitions,
    grid3_multi_partitions,
    grid3x4_recursive_partitions,
    ising_uniform_tensor,
    ising_blocked_tensor,
    random_uniform_tensor,
    block_lattice,
    ising_blocked_lattice,
)
