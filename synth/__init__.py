"""Seeded synthetic inputs for the zSort workloads.

This package draws keys and payloads only.  It holds none of the sorting
method's arithmetic, so the CPU oracle and the GPU path can both be fed from
it without sharing any of the method's code.
"""
from .gen import (  # noqa: F401
    SEED_BASE,
    seed_for,
    uniform,
    normal,
    dup_heavy,
    partial,
    descending,
    lognormal,
    zipf,
    gmm,
    segments,
    wide_range_arrays,
    make,
    WORKLOADS,
    small_range,
    clustered_ranges,
    make128,
    WORKLOADS128,
)
