"""MI355X-native hot path of the cell-task short-range MD method (arXiv:1305.4196).

Linked cells, Verlet neighbor lists, Lennard-Jones and Finnis-Sinclair EAM
forces, velocity Verlet and hand-written adjoints, as HIP kernels for gfx950
behind the C ABI in ``include/md.h``.

Submodules:
  binding    ctypes marshalling of every entry point (same names as the C ABI)
  system     MDSystem convenience class and the MDForces autograd function
  workloads  seeded synthetic inputs (no method arithmetic)
  build      hipcc build of libmd.so
  tune       autotuner for the per-shape launch parameters

Importing the package loads nothing; the library is loaded on first use and a
missing library raises instead of falling back to anything else.
"""

__all__ = ["binding", "system", "workloads", "build", "tune"]
