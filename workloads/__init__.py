"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module builds atomic structures, run parameters and one input field: the
frozen density that the fixed-density mode reads in (atom-centred Gaussians, a
stand-in for a density file).  It holds none of the method's arithmetic (no
potentials, no Hamiltonian, no density the method computes), so that the oracle
and the HIP path can both consume its arrays without sharing any of the
computation they are compared on.
"""
from .systems import (  # noqa: F401
    Species, System, RunConfig, diamond_si, water_box, config, CONFIG_NAMES,
    fragment_valence_counts, superposed_density, si_cells_config,
)
