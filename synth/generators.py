"""Seeded synthetic workloads: geometries, desired states and random TT data.

Conventions shared with the library's C-ABI:

* A geometry is a trivariate B-spline volume: ``degree``, one open knot vector
  per direction and a control-point tensor ``ctrl`` of shape
  ``(3, ncp1, ncp2, ncp3)`` (C order, last index fastest), i.e. the tensor C
  of the geometry-mapping equation in Section 2 of the paper.
* Desired states and solution vectors are coefficient tensors of shape
  ``(n, n, n)`` over the free (interior) B-splines, flattened in C order.
  TT cores have shape ``(r_{d-1}, n_d, r_d)``.

Control points of curved geometries are the analytic map sampled at the
Greville abscissae of the geometry's own knot vector (Schoenberg's
variation-diminishing spline approximation); desired states use the same
recipe on the solution space. No basis function is evaluated here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Geometry", "open_uniform_knots", "greville_abscissae", "interior_greville",
    "identity_geometry", "box_geometry", "affine_geometry", "twisted_annulus",
    "perturbed_cube", "yhat_sine", "yhat_fourier", "random_tt", "random_btt",
    "random_local_problem", "tt_ranks_of", "CONFIGS", "config", "batch_problems",
]


@dataclass
class Geometry:
    degree: int
    knots: list  # three 1-D float64 arrays
    ctrl: np.ndarray  # (3, n1, n2, n3) float64
    name: str = "geometry"
    meta: dict = field(default_factory=dict)

    @property
    def ncp(self):
        return tuple(int(s) for s in self.ctrl.shape[1:])


def open_uniform_knots(nbasis: int, degree: int) -> np.ndarray:
    """Open knot vector on [0,1] with ``nbasis`` functions and uniform interior knots."""
    nel = nbasis - degree
    if nel < 1:
        raise ValueError("need nbasis > degree")
    inner = np.arange(1, nel, dtype=np.float64) / nel
    return np.concatenate([np.zeros(degree + 1), inner, np.ones(degree + 1)])


def greville_abscissae(knots: np.ndarray, degree: int) -> np.ndarray:
    nb = len(knots) - degree - 1
    if degree == 0:
        return 0.5 * (knots[:-1] + knots[1:])
    return np.array([knots[i + 1:i + degree + 1].mean() for i in range(nb)])


def interior_greville(n: int, degree: int) -> np.ndarray:
    """Greville abscissae of the n free functions of the degree-p space with n+2 functions."""
    g = greville_abscissae(open_uniform_knots(n + 2, degree), degree)
    return g[1:-1]


def _grid_ctrl(fn, knots, degree):
    g = [greville_abscissae(k, degree) for k in knots]
    X1, X2, X3 = np.meshgrid(g[0], g[1], g[2], indexing="ij")
    return np.stack(fn(X1, X2, X3), axis=0).astype(np.float64)


def identity_geometry() -> Geometry:
    """Unit cube, trilinear map with the eight corners as control points."""
    knots = [np.array([0.0, 0.0, 1.0, 1.0]) for _ in range(3)]
    ctrl = _grid_ctrl(lambda a, b, c: (a, b, c), knots, 1)
    return Geometry(1, knots, ctrl, "identity")


def box_geometry(a: float, b: float, c: float) -> Geometry:
    knots = [np.array([0.0, 0.0, 1.0, 1.0]) for _ in range(3)]
    ctrl = _grid_ctrl(lambda x, y, z: (a * x, b * y, c * z), knots, 1)
    return Geometry(1, knots, ctrl, "box", {"scale": (a, b, c)})


def affine_geometry(A, shift=(0.0, 0.0, 0.0)) -> Geometry:
    A = np.asarray(A, dtype=np.float64)
    s = np.asarray(shift, dtype=np.float64)
    knots = [np.array([0.0, 0.0, 1.0, 1.0]) for _ in range(3)]
    ctrl = _grid_ctrl(lambda x, y, z: tuple(A[i, 0] * x + A[i, 1] * y + A[i, 2] * z + s[i]
                                            for i in range(3)), knots, 1)
    return Geometry(1, knots, ctrl, "affine", {"A": A, "shift": s})


def twisted_annulus(seed: int = 1, ncp: int = 8, degree: int = 3, r_in: float = 1.0,
                    r_out: float = 2.0, height: float = 1.0, twist_deg: float | None = None) -> Geometry:
    """Quarter annulus (radii r_in, r_out) extruded along z with a twist growing linearly in z.

    The twist angle is ``twist_deg`` if given, else 30 degrees times U(0.5, 1)
    drawn from ``seed``. ``twist_deg=0`` gives the untwisted quarter annulus,
    whose control net is of product form.
    """
    if twist_deg is None:
        rng = np.random.default_rng(seed)
        twist_deg = 30.0 * rng.uniform(0.5, 1.0)
    phi_max = math.radians(twist_deg)
    knots = [open_uniform_knots(ncp, degree) for _ in range(3)]

    def fn(x1, x2, x3):
        rho = r_in + (r_out - r_in) * x1
        ang = 0.5 * math.pi * x2 + phi_max * x3
        return rho * np.cos(ang), rho * np.sin(ang), height * x3

    if twist_deg == 0.0:
        # exact product form: (rho_i cos th_j, rho_i sin th_j, z_k)
        g = [greville_abscissae(k, degree) for k in knots]
        rho = r_in + (r_out - r_in) * g[0]
        th = 0.5 * math.pi * g[1]
        z = height * g[2]
        ctrl = np.stack([
            np.einsum("i,j,k->ijk", rho, np.cos(th), np.ones_like(z)),
            np.einsum("i,j,k->ijk", rho, np.sin(th), np.ones_like(z)),
            np.einsum("i,j,k->ijk", np.ones_like(rho), np.ones_like(th), z)], axis=0)
    else:
        ctrl = _grid_ctrl(fn, knots, degree)
    return Geometry(degree, knots, ctrl, "twisted_annulus",
                    {"seed": seed, "twist_deg": twist_deg, "r_in": r_in, "r_out": r_out})


def perturbed_cube(seed: int = 3, ncp: int = 8, degree: int = 3, amplitude: float = 0.1,
                   passes: int = 3) -> Geometry:
    """Unit cube whose control points get a seeded smooth perturbation of max size ``amplitude``.

    xi ~ N(0,1) per control-point coordinate, smoothed by ``passes`` passes of
    the [1,2,1]/4 filter along each axis (edges replicated), then scaled so
    that max |xi| = amplitude. With one pass, amplitude 0.1 folds the map
    for most seeds (det grad G < 0 near the faces); three passes keep it
    one-to-one for the seeds used here.
    """
    rng = np.random.default_rng(seed)
    knots = [open_uniform_knots(ncp, degree) for _ in range(3)]
    base = _grid_ctrl(lambda a, b, c: (a, b, c), knots, degree)
    xi = rng.standard_normal(base.shape)
    for _ in range(passes):
        for ax in (1, 2, 3):
            pad = [(0, 0)] * 4
            pad[ax] = (1, 1)
            xp = np.pad(xi, pad, mode="edge")
            L = xi.shape[ax]

            def sl(s, e):
                return tuple(slice(None) if k != ax else slice(s, e) for k in range(4))
            xi = 0.25 * xp[sl(0, L)] + 0.5 * xp[sl(1, L + 1)] + 0.25 * xp[sl(2, L + 2)]
    xi *= amplitude / np.abs(xi).max()
    return Geometry(degree, knots, base + xi, "perturbed_cube", {"seed": seed, "amplitude": amplitude})


def yhat_sine(n: int, degree: int):
    """TT (rank 1) coefficients of sin(pi x1) sin(pi x2) sin(pi x3) sampled at interior Greville points."""
    g = interior_greville(n, degree)
    v = np.sin(math.pi * g)
    return [v.reshape(1, n, 1).copy() for _ in range(3)]


def yhat_fourier(n: int, degree: int, seed: int = 2, modes: int = 8):
    """TT coefficients of sum_k g_k |k|^-2 prod_d sin(pi k_d x_d), k in {1..modes}^3, g_k ~ N(0,1).

    Written directly as a TT with ranks (modes, modes): core 1 carries k1,
    core 2 sums over k2 and carries k3, core 3 evaluates mode k3.
    """
    rng = np.random.default_rng(seed)
    k = np.arange(1, modes + 1)
    K1, K2, K3 = np.meshgrid(k, k, k, indexing="ij")
    G = rng.standard_normal((modes, modes, modes)) / (K1 ** 2 + K2 ** 2 + K3 ** 2)
    g = interior_greville(n, degree)
    S = np.sin(math.pi * np.outer(g, k))  # (n, modes)
    c1 = S.reshape(1, n, modes)
    c2 = np.einsum("abc,jb->ajc", G, S)  # (k1, n, k3)
    c3 = S.T.reshape(modes, n, 1)
    return [np.ascontiguousarray(c1), np.ascontiguousarray(c2), np.ascontiguousarray(c3)]


def random_tt(ns, ranks, seed: int = 0):
    rng = np.random.default_rng(seed)
    r = [1] + list(ranks) + [1]
    return [rng.standard_normal((r[d], ns[d], r[d + 1])) / math.sqrt(r[d] * r[d + 1])
            for d in range(len(ns))]


def random_btt(ns, ranks, ell_core: int, seed: int = 0):
    """Block-TT with 3 components: the core ``ell_core`` has shape (3, r_{d-1}, n_d, r_d)."""
    rng = np.random.default_rng(seed)
    r = [1] + list(ranks) + [1]
    cores = []
    for d in range(len(ns)):
        shape = (r[d], ns[d], r[d + 1]) if d != ell_core else (3, r[d], ns[d], r[d + 1])
        cores.append(rng.standard_normal(shape) / math.sqrt(r[d] * r[d + 1]))
    return cores


def random_local_problem(r: int, RM: int, RK: int, n: int, degree: int, seed: int = 0,
                         r_right: int | None = None):
    """Random inputs of the projected local matvec at one core.

    Returns dict with left/right interfaces for M and K (shapes (R, r, r)),
    banded operator cores (R_{d-1}, n, 2p+1, R_d) with entries outside the
    matrix set to zero, and a 3-component local vector (3, r, n, r_right).
    """
    rng = np.random.default_rng(seed)
    rr = r if r_right is None else r_right
    b = 2 * degree + 1

    def band_core(R0, R1):
        A = rng.standard_normal((R0, n, b, R1)) / math.sqrt(R0 * b)
        for i in range(n):
            for o in range(b):
                j = i + o - degree
                if j < 0 or j >= n:
                    A[:, i, o, :] = 0.0
        return A

    out = {
        "PhiL_M": rng.standard_normal((RM, r, r)) / math.sqrt(r),
        "PhiR_M": rng.standard_normal((RM, rr, rr)) / math.sqrt(rr),
        "PhiL_K": rng.standard_normal((RK, r, r)) / math.sqrt(r),
        "PhiR_K": rng.standard_normal((RK, rr, rr)) / math.sqrt(rr),
        "M": band_core(RM, RM),
        "K": band_core(RK, RK),
        "x": rng.standard_normal((3, r, n, rr)),
    }
    return out


def tt_ranks_of(cores):
    return [c.shape[-1] for c in cores[:-1]]


# The five workloads the method is exercised on (sizes, degrees, regularisation).
CONFIGS = {
    "cube_n16": dict(name="identity cube p=2 n=16", geometry="identity", degree=2, n=16, beta=1e-4,
               yhat="sine", tol=1e-8, weight_tol=1e-10, seed_geo=0, seed_y=0),
    "annulus_n64": dict(name="twisted annulus p=3 n=64", geometry="twisted_annulus", degree=3, n=64, beta=1e-6,
               yhat="fourier", tol=1e-7, weight_tol=1e-10, seed_geo=1, seed_y=2),
    "perturbed_cube_n128": dict(name="perturbed cube p=3 n=128", geometry="perturbed_cube", degree=3, n=128, beta=1e-6,
               yhat="fourier", tol=1e-6, weight_tol=1e-6, seed_geo=3, seed_y=4),
    "annulus_n256": dict(name="twisted annulus p=3 n=256", geometry="twisted_annulus", degree=3, n=256, beta=1e-6,
               yhat="fourier", tol=1e-6, weight_tol=1e-10, seed_geo=5, seed_y=6, r_max=40),
}


def batch_problems(count: int = 64, seed0: int = 100, n_choices=(32, 48, 64, 96, 128)):
    """Independent problems of the batching workload, problem i from seed seed0 + i: n drawn
    uniformly from n_choices, degree from {2, 3}, log10 beta uniform in [-8, -2], the geometry a
    perturbed cube (amplitude 0.07: at 0.1 one of the 64 draws folds near a face) or a twisted
    annulus (coin flip, own seed), a Fourier desired state.
    Returns a list of (geometry, yhat cores, params)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.choice(n_choices))
        degree = int(rng.integers(2, 4))
        beta = float(10.0 ** rng.uniform(-8.0, -2.0))
        gseed = int(rng.integers(0, 1 << 30))
        if rng.random() < 0.5:
            geo, gname = perturbed_cube(seed=gseed, amplitude=0.07), "perturbed_cube"
        else:
            geo, gname = twisted_annulus(seed=gseed), "twisted_annulus"
        y = yhat_fourier(n, degree, seed=gseed + 1)
        out.append((geo, y, dict(name="batch %d" % i, geometry=gname, degree=degree, n=n, beta=beta,
                                 seed=seed0 + i)))
    return out


def config(key: str, n: int | None = None):
    """Build (geometry, yhat_cores, params) for a named workload, optionally at another n."""
    c = dict(CONFIGS[key])
    if n is not None:
        c["n"] = n
    if c["geometry"] == "identity":
        geo = identity_geometry()
    elif c["geometry"] == "twisted_annulus":
        geo = twisted_annulus(seed=c["seed_geo"])
    elif c["geometry"] == "perturbed_cube":
        geo = perturbed_cube(seed=c["seed_geo"])
    else:
        raise KeyError(c["geometry"])
    if c["yhat"] == "sine":
        y = yhat_sine(c["n"], c["degree"])
    else:
        y = yhat_fourier(c["n"], c["degree"], seed=c["seed_y"])
    return geo, y, c
