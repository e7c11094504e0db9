"""Seeded synthetic detector events (input generator shared by the oracle
and the GPU path; holds no reconstruction arithmetic)."""
from .events import (BARREL, C_LIGHT, DISK, Events, Geometry, Workload,
                     duplicate_seeds, generate, make_geometry, track_lists,
                     workload)
from .strips import strip_detector, strip_events

__all__ = ["BARREL", "DISK", "C_LIGHT", "Events", "Geometry", "Workload",
           "duplicate_seeds", "generate", "make_geometry", "track_lists",
           "workload", "strip_detector", "strip_events"]
