"""LB-IMB-DEM on AMD MI355X: fused lattice-Boltzmann / immersed-moving-boundary /
DEM step in hand-written HIP for gfx950 behind a C ABI (``include/lbimb.h``).

Importing the package loads nothing; ``paper_1011_2613_amd.binding`` loads the
native library on first use and fails loudly if it has not been built.
"""
__all__ = ["inputs", "binding"]
