"""Seeded synthetic inputs (rest meshes, batches of cells, external forces).

Shared by the oracle's tests, the GPU tests and the benchmark.  Holds geometry and
forcing only; none of the solver's arithmetic lives here.
"""
from . import meshes, workloads  # noqa: F401
