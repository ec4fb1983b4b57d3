"""Seeded, synthetic inputs shared by the CPU oracle and the HIP path.

This package only *describes* workloads: discharge parameters, the lateral
area and macro-particle weight that normalise them, and the tabulated cross
sections.  It contains none of the PIC-MCC arithmetic (no push, no field solve,
no collision sampling); both implementations receive these numbers as inputs.
"""
from .configs import WORKLOADS, Workload, served_stream, sweep, workload
from .xsec import CHANNELS, N_CHANNELS, N_POINTS, energy_grid, build_tables

__all__ = ["WORKLOADS", "Workload", "served_stream", "sweep", "workload", "CHANNELS", "N_CHANNELS",
           "N_POINTS", "energy_grid", "build_tables"]
