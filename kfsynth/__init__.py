"""Seeded synthetic detector events (input generator shared by the oracle
and the GPU path; holds no reconstruction arithmetic)."""
from .events import (BARREL, C_LIGHT, DISK, Events, Geometry, Workload,
                     generate, make_geometry, workload)

__all__ = ["BARREL", "DISK", "C_LIGHT", "Events", "Geometry", "Workload",
           "generate", "make_geometry", "workload"]
