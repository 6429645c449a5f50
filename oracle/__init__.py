"""ORACLE — test infrastructure, not part of the product.

A plain, slow, FP64 CPU implementation of the embedded-boundary
finite-volume elliptic problem that the GPU library solves. Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it. It shares no code with the library: it reads the seeded problem
descriptions from ``workloads`` and nothing else.

Modules
  geometry  cut-cell moments from node-sampled level sets
  operator  the linear system A phi = b (rows in the volume-weighted integral form)
  solvers   dense LU, SuperLU with refinement, and a multigrid-preconditioned GMRES
  efield    flux-based electric field
  exact     closed forms used as pins

Parity status per function is stated in each module header.
"""
from .geometry import Geometry, GeometryError  # noqa: F401

