"""Seeded synthetic inputs shared by the oracle, the tests, the smoke check and the bench.

This package draws random numbers and lays them out; it holds none of the
eigensolver's arithmetic (no sphere, no projector, no Hamiltonian, no filter).
"""
from .systems import (  # noqa: F401
    BATCH,
    CONFIGS,
    PAW_Q_SCALE,
    System,
    make_batch,
    make_system,
    random_block,
    random_vector,
    smooth_235,
    streams,
)
