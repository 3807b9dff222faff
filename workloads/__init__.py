"""Seeded synthetic inputs shared by the oracle-based tests and the GPU path.

Nothing here evaluates the discretization: these modules only produce mesh
arrays (vertex coordinates, topological vertex ids, boundary tags) and
primitive initial fields at given points.  Both the FP64 CPU oracle and the
HIP library consume the same arrays; each side derives its own nodes,
operators, geometry and state from them.
"""
from .meshes import (BC_INTERIOR, BC_OUTFLOW_CHAR, BC_PASSTHRU, BC_WALL,
                     BC_INFLOW, BC_LEARNED, box_kuhn, trumpet_domain)
from .fields import gaussian_pulse, plane_wave, isentropic_vortex
from .order import locality_order, reorder

__all__ = ["BC_INTERIOR", "BC_OUTFLOW_CHAR", "BC_PASSTHRU", "BC_WALL",
           "BC_INFLOW", "BC_LEARNED", "box_kuhn", "trumpet_domain",
           "gaussian_pulse", "plane_wave", "isentropic_vortex", "locality_order", "reorder"]
