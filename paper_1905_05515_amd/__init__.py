"""MI355X-native TPC track-finding hot path (arXiv:1905.05515, section 3):
pad-row grid, cellular-automaton neighbour finding, Kalman tracklet
construction and selection, calibrated refit with its adjoint.  All steps
run in the HIP kernels of libtpc.so (C ABI in include/tpc.h); this package
binds them to torch tensors and streams."""
from .layout import SECTOR_DTYPE, grid_layout  # noqa: F401

__all__ = ["SECTOR_DTYPE", "grid_layout"]
