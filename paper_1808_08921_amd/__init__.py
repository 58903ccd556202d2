"""MI355X (gfx950) coupled lattice-Boltzmann / DEM library for the hydro-micromechanical
model of Cheng et al., arXiv 1808.08921.

The compute path is the HIP library ``liblbdem.so`` behind the C interface of
``include/lbdem.h``; :mod:`paper_1808_08921_amd.lbdem` is a thin ctypes binding (argument
marshalling only) with PyTorch providing device memory and streams.
"""
