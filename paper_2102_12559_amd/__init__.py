"""MI355X multi-scale semi-Lagrangian lattice Boltzmann step (arXiv 2102.12559).

The compute path is libmsl.so (hand-written HIP for gfx950 behind the C-ABI in
include/msl.h); `msl` is its Python binding and `inputs` the seeded synthetic
workloads.
"""
from . import inputs  # noqa: F401
