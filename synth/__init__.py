"""Seeded synthetic workloads for the MAS-preconditioned PCG solve.

This package builds the *inputs* of the linear solve only: meshes, element
Hessians projected to PSD, contact-like couplings, the assembled 3x3-block
BCSR matrix ``H = M + h^2 * sum(K_e)`` and right-hand sides.  It holds none
of the solver's arithmetic (no ordering, no hierarchy, no preconditioner, no
CG), so both the CPU oracle and the HIP library can consume what it writes
without sharing any code with each other.

Every random draw comes from ``numpy.random.SeedSequence(seed).spawn(k)``
sub-streams, so a workload is a pure function of its configuration and seed.
"""

from .mesh import tet_cube, cube_surface_nodes, mesh_edges
from .bcsr import BlockSystem, assemble_bcsr, graph_from_edges, random_spd_system, spd_system_from_edges
from .workloads import (
    cube_system,
    config_tiny,
    config_small,
    config_large,
    config_membrane,
    WORKLOADS,
)
from .membrane import membrane_system

__all__ = [
    "tet_cube",
    "cube_surface_nodes",
    "mesh_edges",
    "BlockSystem",
    "assemble_bcsr",
    "graph_from_edges",
    "random_spd_system",
    "spd_system_from_edges",
    "cube_system",
    "config_tiny",
    "config_small",
    "config_large",
    "config_membrane",
    "membrane_system",
    "WORKLOADS",
]
