"""Seeded synthetic inputs shared by the CPU oracle tests, the GPU tests and bench.py.

This package holds none of the method's arithmetic: it evaluates no B-spline
basis function, assembles no matrix and solves nothing. It only writes knot
vectors, control-point tensors and TT cores of desired states from closed-form
formulas and a seeded random generator.
"""
from .generators import *  # noqa: F401,F403
