"""Occupancy-Based Dual Contouring on AMD MI355X: HIP kernels behind a C ABI
(include/odc.h) and a thin ctypes binding (odc.py)."""
from . import odc  # noqa: F401
