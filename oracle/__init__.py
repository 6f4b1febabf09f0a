"""Plain FP64 CPU oracle for the adaptive BDDC method of Peng, Shu, Wang and
Zhong, "A BDDC method with an adaptive coarse space for three-dimensional
advection-diffusion problems" (arXiv 2501.01676).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package; only the test suite, the smoke check and the CPU baseline
leg of the benchmark do.  It shares no code with the GPU library: it has its
own topology, assembly and algebra, written from the paper in its order and
notation, with numpy/scipy library routines (dense solves, Cholesky,
symmetric eigensolver, SVD, QR, sparse direct solve) as the only building
blocks.  There is no blocking, fusion or reordering beyond what the paper's
definitions state.

Modules
  topology  box partition, face/edge/vertex classes, orderings (Section 3)
  fem       GLS-stabilised Q1 element matrices and assembly (Section 2)
  bddc      Schur complements, deluxe scaling, face and edge eigenproblems,
            change of basis, coarse problem, preconditioner, GMRES (Section 3)

Parity status of each function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
from .topology import PartitionTopology, Topology, make_topology  # noqa: F401
from . import fem, bddc  # noqa: F401
