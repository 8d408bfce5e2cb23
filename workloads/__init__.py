"""Seeded synthetic particle systems shared by tests, smoke check and benchmark.

This package holds input generators only: positions and charges.  It contains
none of the Ewald method's arithmetic, so it can serve both the GPU path and
the CPU oracle without coupling them.
"""
from .systems import (  # noqa: F401
    CONFIGS,
    SystemSpec,
    ions,
    make_system,
    nacl_lattice,
    water,
)
