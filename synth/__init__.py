"""Seeded synthetic contact workloads for thickened rods and shells.

This package builds geometry only: positions, topology and the reference
(rest-space) parameters of each mesh.  It holds none of the contact method's
arithmetic (no distances, no filter, no barrier), so the CPU oracle and the
GPU path can both consume its output without sharing any of that code.

All lengths are in micrometres.  Every constant that the method compares
against (thickness h, offset eta, rest edge lengths, rest coordinates) is an
exact integer in these units, so generator-level ties are exact in IEEE
double precision.

The paper's own scenes (knitted yarn patterns, a dragon mesh, knot polylines,
photographs) are not available here; these generators are stand-ins with the
shapes and sizes of the paper's workloads (its yarn table: 18 to 80k
segments, 0.18-0.5 mm thick; its cloth table: 10k-100k triangles,
0.1-5 mm thick).
"""
from .scenes import (Scene, helix_loop_rod, woven_patch, folded_cloth,
                     batch_scenes, serving_scenes, crossing_rods, straight_rod, flat_sheet, search_direction,
                     workload, WORKLOADS)

__all__ = ["Scene", "helix_loop_rod", "woven_patch", "folded_cloth",
           "batch_scenes", "serving_scenes", "crossing_rods", "straight_rod", "flat_sheet", "search_direction",
           "workload", "WORKLOADS"]
