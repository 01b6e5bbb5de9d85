"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module builds atomic structures and run parameters only.  It holds none
of the method's arithmetic (no potentials, no Hamiltonian, no densities), so
that the oracle and the HIP path can both consume its arrays without sharing
any of the computation they are compared on.
"""
from .systems import (  # noqa: F401
    Species, System, RunConfig, diamond_si, water_box, config, CONFIG_NAMES,
    fragment_valence_counts,
)
