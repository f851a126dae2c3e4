"""MI355X-native sliding-mesh spectral difference (SSD) solver.

The compute path is the HIP library libssd.so (C ABI in include/ssd.h);
`paper_1503_02198_amd.ssd` is its ctypes binding.
"""
from .ssd import (MLP, Batch, Mesh, SSDError, lib, pack_state, restrict,  # noqa: F401
                  subgrid_nudge, subgrid_targets, unpack_state)
