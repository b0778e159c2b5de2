"""Writes the expected state of the twisted-annulus workload at n = 32 (tests/golden/annulus_n32_state.npz).

Calls only the oracle (and the seeded input generators): full 3-D Galerkin assembly of M and K
with the weights interpolated in the degree-(2p+1) space (the integrand of the Kronecker form),
then the reduced state equation (M + beta K M^-1 K) y = M yhat by preconditioned CG
(oracle.kkt.solve_reduced). Workload: twisted quarter annulus (seed 1), degree 3, n = 32 free
functions per direction, beta = 1e-6, Fourier desired state (seed 2, 8 modes per axis) -- the
n = 64 workload's geometry, desired state and beta at half the resolution.

Stored: y (n^3, C order), the KKT relative residual of (y, u, lambda) in the oracle's own
operators, the CG iteration count and the parameters. Takes about 20 minutes on 8 cores
(two sparse LU factorisations of 32768 x 32768 matrices).

Usage: python tests/golden/make_reduced_state.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import assembly, kkt, tt  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "annulus_n32_state.npz")


def main():
    n, p, beta, seed_geo, seed_y = 32, 3, 1e-6, 1, 2
    geo = synth.twisted_annulus(seed=seed_geo)
    yh = tt.tt_full(synth.yhat_fourier(n, p, seed=seed_y)).ravel()
    t0 = time.perf_counter()
    M, K = assembly.assemble(geo, n, p, mode="interp")
    t1 = time.perf_counter()
    print("assembly %.1f s" % (t1 - t0), flush=True)
    y, u, lam, its = kkt.solve_reduced(M, K, beta, yh)
    t2 = time.perf_counter()
    res = kkt.residual(M, K, beta, yh, np.concatenate([y, u, lam]))
    print("reduced solve %.1f s, %d CG steps, KKT residual %.3e" % (t2 - t1, its, res), flush=True)
    np.savez(OUT, y=y, kkt_residual=np.float64(res), cg_iterations=np.int64(its), n=np.int64(n),
             degree=np.int64(p), beta=np.float64(beta), seed_geometry=np.int64(seed_geo),
             seed_yhat=np.int64(seed_y))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
