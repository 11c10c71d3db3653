"""Seeded synthetic particle sets that stand in for the paper's simulation snapshots.

This package holds input generation only: it draws positions and states the
per-workload parameters (box side, cells per side, softening length, G*m).  It
contains none of the near-field method's arithmetic, so both the HIP path and
the FP64 oracle can consume its output without sharing any force code.
"""
from .gen import (Box, Workload, uniform_positions, plummer_halo_positions,
                  power_law_masses, largest_remainder, workload, WORKLOADS)

__all__ = ["Box", "Workload", "uniform_positions", "plummer_halo_positions",
           "power_law_masses", "largest_remainder", "workload", "WORKLOADS"]
