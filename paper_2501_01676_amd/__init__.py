"""MI355X (gfx950) adaptive BDDC for 3D advection-diffusion (arXiv 2501.01676).

The compute path is the HIP library libabddc_hip.so behind the C ABI of
include/abddc.h; this package holds its ctypes binding (``api``), the
in-tree build script (``build``) and the seeded synthetic workloads
(``workloads``).  Importing the package does not load the library.
"""

__all__ = ["api", "build", "workloads"]
