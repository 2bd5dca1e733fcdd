"""Seeded synthetic inputs shared by the GPU library's tests/benchmarks and the oracle.

Holds no arithmetic of the numerical method: it builds quadtree leaf lists
(level, ix, iy) and evaluates initial conditions at node coordinates that the
caller supplies.  Random numbers come from a counter-based SplitMix64.
"""
from .rng import uniform  # noqa: F401
from .meshes import MeshSpec, uniform_mesh, refined_box_mesh, workload_mesh  # noqa: F401
from . import states  # noqa: F401
