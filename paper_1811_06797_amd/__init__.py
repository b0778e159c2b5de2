"""MI355X (gfx950) library for the low-rank TT method for IgA PDE-constrained optimisation.

The HIP/C++ library ``libiga.so`` (C ABI in include/iga.h) holds the whole
hot path; ``paper_1811_06797_amd.iga`` is its ctypes binding. Build with
``python paper_1811_06797_amd/build.py``.
"""
