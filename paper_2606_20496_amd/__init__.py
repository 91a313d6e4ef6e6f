"""MI355X-native two-level Schwarz coarse solver (PCG on the Q1 element-vertex
Poisson system) with a C-ABI library of hand-written gfx950 HIP kernels.

Importing the package is cheap: the shared library is loaded on first use by
:mod:`paper_2606_20496_amd.coarse`.
"""
__all__ = ["meshgen", "coarse"]
