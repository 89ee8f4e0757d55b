"""MI355X-native (gfx950, HIP, FP64) implementation of the data-parallel hot path
of the structure-preserving ALE-WENO finite-volume scheme for the shallow water
equations (Zhang, Xia & Xu, arXiv 2208.06588): one modified SSP-RK3 step per cell
on a moving 1D mesh, behind the C ABI of include/alew.h.

``paper_2208_06588_amd.alew`` is the ctypes binding; ``workloads`` builds the
seeded synthetic inputs.
"""
__all__ = ["alew", "workloads"]
