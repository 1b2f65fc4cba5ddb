"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds only parameter sets and random placement of bubble nuclei. It contains
none of the method's arithmetic, so both the oracle and the GPU library can consume its
output without sharing code.
"""
from .workloads import (  # noqa: F401
    SplitMix64,
    WORKLOADS,
    batch_workloads,
    place_nuclei,
    workload,
    small_case,
)
