"""Seeded synthetic inputs for the recursive Green's function (RGF) hot path.

This package draws Hamiltonian blocks, lead blocks, energy and k grids and the
scattering / bias parameters of the workloads.  It holds none of the method's
arithmetic (no inverse, no self-energy, no Green's function): both the CPU
oracle and the GPU path read what it produces.
"""
from .workloads import (  # noqa: F401
    Workload,
    KT_300K,
    make_workload,
    strip_workload,
    cross_section_workload,
    random_tiny,
    WORKLOAD_NAMES,
)
