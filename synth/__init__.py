"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This package only draws random numbers and lays them out; it holds none of the
method's arithmetic (no overlaps, Green's functions, energies or propagators).
"""
from .gen import (  # noqa: F401
    CONFIGS,
    Workload,
    make_workload,
    make_config,
    fields_for_step,
    make_uneven,
)
