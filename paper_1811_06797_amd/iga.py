"""ctypes binding of libiga.so (include/iga.h): argument marshalling only.

Every function here has the name of the C entry point without the ``iga_``
prefix and does nothing but convert arguments and check the status code.
All computation happens in the HIP library; if it is not built, importing
this module raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiga.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libiga.so is not built; run python paper_1811_06797_amd/build.py "
                      "(or __graft_entry__.build())")
lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EHIP, EGEOM, ENOCONV, ERANK, ENUM = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32, BF16 = 0, 1, 2
MAX_HISTORY = 64  # IGA_MAX_HISTORY
_NAMES = {EINVAL: "IGA_EINVAL", ENOMEM: "IGA_ENOMEM", EHIP: "IGA_EHIP", EGEOM: "IGA_EGEOM",
          ENOCONV: "IGA_ENOCONV", ERANK: "IGA_ERANK", ENUM: "IGA_ENUM"}

EXPORTED = [
    "iga_ctx_create", "iga_ctx_destroy", "iga_assemble_factors", "iga_ttop_create", "iga_ttop_info",
    "iga_ttop_get_core", "iga_ttop_destroy", "iga_tt_create", "iga_tt_wrap", "iga_tt_from_full", "iga_tt_round", "iga_tt_destroy",
    "iga_tt_info", "iga_tt_get_core",
    "iga_btt_create", "iga_btt_info", "iga_btt_blocks", "iga_btt_get_core", "iga_btt_to_full", "iga_btt_destroy",
    "iga_kkt_create", "iga_kkt_create_parabolic", "iga_kkt_blocks", "iga_kkt_destroy", "iga_kkt_apply", "iga_kkt_residual", "iga_amen_solve",
    "iga_amen_solve_many",
    "iga_local_matvec", "iga_local_matvec_noalloc", "iga_local_matvec_batched", "iga_local_matvec_flops", "iga_profile_start", "iga_profile_stop",
    "iga_measure_peaks", "iga_objective",
    "iga_grad_yhat", "iga_grad_geometry", "iga_last_error",
]


class IgaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("degree", C.c_int), ("ncp", C.c_int * 3), ("knots", C.POINTER(C.c_double) * 3),
                ("ctrl", C.POINTER(C.c_double))]


class AssemblyOpts(C.Structure):
    _fields_ = [("p_interp", C.c_int), ("nquad", C.c_int), ("weight_tol", C.c_double),
                ("weight_rmax", C.c_int)]


class AmenOpts(C.Structure):
    _fields_ = [("nswp", C.c_int), ("r_max", C.c_int), ("kick_rank", C.c_int), ("local_tol", C.c_double),
                ("local_maxit", C.c_int), ("local_restart", C.c_int), ("precision", C.c_int),
                ("init_rank", C.c_int), ("seed", C.c_ulonglong), ("verbose", C.c_int)]


class AmenStats(C.Structure):
    _fields_ = [("half_sweeps", C.c_int), ("converged", C.c_int), ("max_local_residual", C.c_double),
                ("residual", C.c_double), ("ranks", C.c_int * 2), ("local_solves", C.c_longlong),
                ("local_iterations", C.c_longlong), ("local_matvecs", C.c_longlong),
                ("local_matvec_flops", C.c_double), ("t_total", C.c_double), ("t_local_matvec", C.c_double),
                ("t_precond", C.c_double), ("t_krylov_other", C.c_double), ("t_interfaces", C.c_double),
                ("t_svd", C.c_double), ("t_residual", C.c_double), ("local_matvecs_fp32", C.c_longlong),
                ("local_matvec_flops_fp32", C.c_double), ("t_local_matvec_fp32", C.c_double),
                ("refinements", C.c_longlong),
                ("history_max_local_residual", C.c_double * MAX_HISTORY),
                ("history_ranks", (C.c_int * 2) * MAX_HISTORY),
                ("history_storage", C.c_longlong * MAX_HISTORY)]

    def as_dict(self):
        out = {}
        h = min(self.half_sweeps, MAX_HISTORY)
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name == "ranks":
                v = list(v)
            elif name == "history_ranks":
                v = [list(v[i]) for i in range(h)]
            elif name.startswith("history_"):
                v = list(v)[:h]
            out[name] = v
        return out


class LocalProblem(C.Structure):
    _fields_ = [("r0", C.c_int), ("n", C.c_int), ("r1", C.c_int), ("degree", C.c_int), ("RM0", C.c_int),
                ("RM1", C.c_int), ("RK0", C.c_int), ("RK1", C.c_int), ("PhiL_M", C.c_void_p), ("PhiR_M", C.c_void_p),
                ("PhiL_K", C.c_void_p), ("PhiR_K", C.c_void_p), ("Mcore", C.c_void_p), ("Kcore", C.c_void_p),
                ("beta", C.c_double), ("x", C.c_void_p), ("y", C.c_void_p)]


class Profile(C.Structure):
    _fields_ = [("stages", C.c_long * 6), ("launches", C.c_long * 6), ("ms", C.c_double * 6),
                ("flops", C.c_double * 6), ("s1_ms", C.c_double * 6), ("s1_flops", C.c_double * 6),
                ("s3_ms", C.c_double * 6), ("s3_flops", C.c_double * 6)]

    def as_dict(self):
        return {name: list(getattr(self, name)) for name, _ in self._fields_}


P = C.c_void_p
PD = C.POINTER(C.c_double)
I3 = C.c_int * 3
I4 = C.c_int * 4

lib.iga_last_error.restype = C.c_char_p
lib.iga_ctx_create.argtypes = [C.c_int, P, C.POINTER(P)]
lib.iga_ctx_destroy.argtypes = [P]
lib.iga_ctx_destroy.restype = None
lib.iga_assemble_factors.argtypes = [P, C.POINTER(Geometry), C.c_int, I3, C.POINTER(AssemblyOpts),
                                     C.POINTER(P), C.POINTER(P), C.POINTER(C.c_int)]
lib.iga_ttop_create.argtypes = [P, C.c_int, I3, I4, PD * 3, C.POINTER(P)]
lib.iga_ttop_info.argtypes = [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
lib.iga_ttop_get_core.argtypes = [P, P, C.c_int, PD]
lib.iga_ttop_destroy.argtypes = [P]
lib.iga_ttop_destroy.restype = None
lib.iga_tt_create.argtypes = [P, I3, I4, PD * 3, C.POINTER(P)]
lib.iga_tt_wrap.argtypes = [P, I3, I4, PD * 3, C.POINTER(P)]
lib.iga_tt_from_full.argtypes = [P, I3, P, C.c_double, C.POINTER(P)]
lib.iga_tt_round.argtypes = [P, P, C.c_double, C.POINTER(P)]
lib.iga_tt_destroy.argtypes = [P]
lib.iga_tt_destroy.restype = None
lib.iga_tt_info.argtypes = [P, I3, I4]
lib.iga_tt_get_core.argtypes = [P, P, C.c_int, PD]
lib.iga_btt_create.argtypes = [P, I3, I4, C.c_int, PD * 3, C.POINTER(P)]
lib.iga_btt_info.argtypes = [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
lib.iga_btt_get_core.argtypes = [P, P, C.c_int, PD]
lib.iga_btt_to_full.argtypes = [P, P, PD]
lib.iga_btt_destroy.argtypes = [P]
lib.iga_btt_destroy.restype = None
lib.iga_kkt_create.argtypes = [P, P, P, C.c_double, C.POINTER(P)]
lib.iga_kkt_create_parabolic.argtypes = [P, P, P, C.c_double, C.c_int, C.c_double, C.POINTER(P)]
lib.iga_kkt_blocks.argtypes = [P]
lib.iga_amen_solve_many.argtypes = [P, C.c_int, C.POINTER(P), C.POINTER(P), C.POINTER(C.c_double), C.POINTER(AmenOpts),
                                    C.c_int, C.POINTER(P), C.c_void_p, C.POINTER(C.c_int)]
lib.iga_btt_blocks.argtypes = [P]
lib.iga_kkt_destroy.argtypes = [P]
lib.iga_kkt_destroy.restype = None
lib.iga_kkt_apply.argtypes = [P, P, P, C.POINTER(P)]
lib.iga_kkt_residual.argtypes = [P, P, P, P, PD]
lib.iga_amen_solve.argtypes = [P, P, P, C.c_double, C.POINTER(AmenOpts), P, C.POINTER(P),
                               C.POINTER(AmenStats)]
lib.iga_local_matvec.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                 C.c_int, P, P, P, P, P, P, C.c_double, P, P, C.c_int]
lib.iga_local_matvec_noalloc.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_int, P, P, P, P, P, P, C.c_double, P, P]
lib.iga_local_matvec_batched.argtypes = [P, C.c_int, C.POINTER(LocalProblem), C.c_int, C.c_int]
lib.iga_local_matvec_flops.argtypes = [C.c_int] * 8
lib.iga_local_matvec_flops.restype = C.c_double
lib.iga_objective.argtypes = [P, P, P, P, PD]
lib.iga_grad_yhat.argtypes = [P, P, P, P, P]
lib.iga_grad_geometry.argtypes = [P, C.POINTER(Geometry), C.c_int, I3, C.POINTER(AssemblyOpts), C.c_double, P, P,
                                  PD]
lib.iga_profile_start.argtypes = [P]
lib.iga_profile_stop.argtypes = [P, C.POINTER(Profile)]
lib.iga_measure_peaks.argtypes = [P, PD]


def last_error() -> str:
    return lib.iga_last_error().decode()


def _check(rc):
    if rc != OK:
        raise IgaError(rc, last_error())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(PD)


def _host(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def ctx_create(device: int = 0, stream: int | None = None):
    out = P()
    _check(lib.iga_ctx_create(device, P(stream) if stream else None, C.byref(out)))
    return out


def ctx_destroy(ctx):
    lib.iga_ctx_destroy(ctx)


def assemble_factors(ctx, geo, degree: int, n, p_interp: int = 0, nquad: int = 0,
                     weight_tol: float = 0.0, weight_rmax: int = 0):
    """geo: any object with .degree, .knots (3 arrays) and .ctrl (3, n1, n2, n3). Returns (M, K, ranks[7][2])."""
    knots = [_host(k) for k in geo.knots]
    ctrl = _host(geo.ctrl)
    g = Geometry()
    g.degree = int(geo.degree)
    for d in range(3):
        g.ncp[d] = int(ctrl.shape[1 + d])
        g.knots[d] = _dptr(knots[d])
    g.ctrl = _dptr(ctrl)
    o = AssemblyOpts(int(p_interp), int(nquad), float(weight_tol), int(weight_rmax))
    M, K = P(), P()
    ranks = (C.c_int * 14)()
    nn = I3(*[int(v) for v in (n if hasattr(n, "__len__") else (n, n, n))])
    _check(lib.iga_assemble_factors(ctx, C.byref(g), int(degree), nn, C.byref(o), C.byref(M), C.byref(K),
                                    ranks))
    return M, K, np.array(list(ranks)).reshape(7, 2)


def ttop_create(ctx, degree, n, R, cores):
    cs = [_host(c) for c in cores]
    arr = (PD * 3)(*[_dptr(c) for c in cs])
    out = P()
    _check(lib.iga_ttop_create(ctx, int(degree), I3(*n), I4(*R), arr, C.byref(out)))
    return out


def ttop_info(op):
    n, R, deg = I3(), I4(), C.c_int()
    _check(lib.iga_ttop_info(op, n, R, C.byref(deg)))
    return list(n), list(R), deg.value


def ttop_get_core(ctx, op, d):
    n, R, p = ttop_info(op)
    out = np.empty((R[d], n[d], 2 * p + 1, R[d + 1]))
    _check(lib.iga_ttop_get_core(ctx, op, d, _dptr(out)))
    return out


def ttop_destroy(op):
    lib.iga_ttop_destroy(op)


def tt_create(ctx, cores):
    cs = [_host(c) for c in cores]
    n = [c.shape[1] for c in cs]
    r = [1, cs[0].shape[2], cs[1].shape[2], 1]
    out = P()
    _check(lib.iga_tt_create(ctx, I3(*n), I4(*r), (PD * 3)(*[_dptr(c) for c in cs]), C.byref(out)))
    return out


def tt_wrap(ctx, n, r, dev_ptrs):
    out = P()
    arr = (PD * 3)(*[C.cast(P(int(p)), PD) for p in dev_ptrs])
    _check(lib.iga_tt_wrap(ctx, I3(*n), I4(*r), arr, C.byref(out)))
    return out


def tt_destroy(t):
    lib.iga_tt_destroy(t)


def btt_create(ctx, cores, ell_core: int):
    cs = [_host(c) for c in cores]
    n, r = [], [1]
    for d, c in enumerate(cs):
        sh = c.shape[1:] if d == ell_core else c.shape
        n.append(sh[1])
        if d < 2:
            r.append(sh[2])
    r.append(1)
    out = P()
    _check(lib.iga_btt_create(ctx, I3(*n), I4(*r), int(ell_core), (PD * 3)(*[_dptr(c) for c in cs]),
                              C.byref(out)))
    return out


def btt_info(x):
    n, r, e = I3(), I4(), C.c_int()
    _check(lib.iga_btt_info(x, n, r, C.byref(e)))
    return list(n), list(r), e.value


def btt_blocks(x) -> int:
    """Number of solution blocks: 3 (stationary) or 3 nt (time-dependent)."""
    nb = lib.iga_btt_blocks(x)
    if nb < 0:
        raise IgaError(nb, last_error())
    return nb


def btt_get_core(ctx, x, d):
    n, r, e = btt_info(x)
    shape = (r[d], n[d], r[d + 1]) if d != e else (btt_blocks(x), r[d], n[d], r[d + 1])
    out = np.empty(shape)
    _check(lib.iga_btt_get_core(ctx, x, d, _dptr(out)))
    return out


def btt_get_cores(ctx, x):
    return [btt_get_core(ctx, x, d) for d in range(3)]


def btt_to_full(ctx, x, out=None):
    """Expand into a device tensor [nblk][n1][n2][n3] (torch, on the context's device)."""
    import torch
    n, _, _ = btt_info(x)
    nb = btt_blocks(x)
    if out is None:
        out = torch.empty((nb, n[0], n[1], n[2]), dtype=torch.float64, device="cuda")
    assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() == nb * np.prod(n)
    _check(lib.iga_btt_to_full(ctx, x, C.cast(P(out.data_ptr()), PD)))
    return out


def btt_destroy(x):
    lib.iga_btt_destroy(x)


def kkt_create(ctx, M, K, beta: float):
    out = P()
    _check(lib.iga_kkt_create(ctx, M, K, float(beta), C.byref(out)))
    return out


def kkt_create_parabolic(ctx, M, K, beta: float, nt: int, tau: float):
    """Time-dependent KKT system (implicit Euler, nt steps of length tau); solutions have
    3 nt blocks y_1..y_nt, u_1..u_nt, lambda_1..lambda_nt."""
    out = P()
    _check(lib.iga_kkt_create_parabolic(ctx, M, K, float(beta), int(nt), float(tau), C.byref(out)))
    return out


def kkt_blocks(k) -> int:
    nb = lib.iga_kkt_blocks(k)
    if nb < 0:
        raise IgaError(nb, last_error())
    return nb


def kkt_destroy(k):
    lib.iga_kkt_destroy(k)


def kkt_apply(ctx, kkt, x):
    out = P()
    _check(lib.iga_kkt_apply(ctx, kkt, x, C.byref(out)))
    return out


def kkt_residual(ctx, kkt, yhat, f) -> float:
    r = C.c_double()
    _check(lib.iga_kkt_residual(ctx, kkt, yhat, f, C.byref(r)))
    return r.value


def amen_solve(ctx, kkt, yhat, tol: float, x0=None, raise_on_noconv: bool = False, **opts):
    """Returns (solution handle, stats dict, status code). opts: fields of iga_amen_opts."""
    o = AmenOpts()
    for k, v in opts.items():
        setattr(o, k, v)
    st = AmenStats()
    sol = P()
    rc = lib.iga_amen_solve(ctx, kkt, yhat, float(tol), C.byref(o), x0, C.byref(sol), C.byref(st))
    if rc != OK and not (rc in (ENOCONV, ERANK) and not raise_on_noconv and sol):
        raise IgaError(rc, last_error())
    return sol, st.as_dict(), rc


def amen_solve_many(ctx, kkts, yhats, tols, workers: int = 8, **opts):
    """Independent solves run concurrently (iga_amen_solve_many). Returns (solution handles,
    stats dicts, status codes); a handle is None where a solve produced no solution."""
    n = len(kkts)
    o = AmenOpts()
    for k, v in opts.items():
        setattr(o, k, v)
    if not isinstance(tols, (list, tuple)):
        tols = [tols] * n
    K = (P * n)(*kkts)
    Y = (P * n)(*yhats)
    T = (C.c_double * n)(*[float(t) for t in tols])
    S = (P * n)()
    st = (AmenStats * n)()
    rc = (C.c_int * n)()
    code = lib.iga_amen_solve_many(ctx, n, K, Y, T, C.byref(o), int(workers), S, C.cast(st, C.c_void_p), rc)
    sols = [P(S[i]) if S[i] else None for i in range(n)]
    if code != OK:
        for s_ in sols:
            if s_ is not None:
                btt_destroy(s_)
        raise IgaError(code, last_error())
    return sols, [st[i].as_dict() for i in range(n)], list(rc)


def local_matvec(ctx, r0, n, r1, degree, RM0, RM1, RK0, RK1, PhiL_M, PhiR_M, PhiL_K, PhiR_K, Mcore, Kcore,
                 beta, x, y, precision=FP64):
    """All array arguments are device pointers (ints) or torch CUDA tensors."""
    def ptr(t):
        return P(t.data_ptr() if hasattr(t, "data_ptr") else int(t))
    _check(lib.iga_local_matvec(ctx, r0, n, r1, degree, RM0, RM1, RK0, RK1, ptr(PhiL_M), ptr(PhiR_M),
                                ptr(PhiL_K), ptr(PhiR_K), ptr(Mcore), ptr(Kcore), float(beta), ptr(x), ptr(y),
                                int(precision)))


def local_matvec_noalloc(ctx, r0, n, r1, degree, RM0, RM1, RK0, RK1, PhiL_M, PhiR_M, PhiL_K, PhiR_K, Mcore, Kcore,
                         beta, x, y):
    """iga_local_matvec_noalloc: the FP64 local matvec with its intermediates in the library's
    fixed per-GPU scratch array. Array arguments are device pointers (ints) or CUDA tensors."""
    def ptr(t):
        return P(t.data_ptr() if hasattr(t, "data_ptr") else int(t))
    _check(lib.iga_local_matvec_noalloc(ctx, r0, n, r1, degree, RM0, RM1, RK0, RK1, ptr(PhiL_M), ptr(PhiR_M),
                                        ptr(PhiL_K), ptr(PhiR_K), ptr(Mcore), ptr(Kcore), float(beta), ptr(x),
                                        ptr(y)))


NOALLOC_SCRATCH_BYTES = 64 << 20  # IGA_NOALLOC_SCRATCH_BYTES


def local_matvec_flops(r0, n, r1, degree, RM0, RM1, RK0, RK1) -> float:
    return lib.iga_local_matvec_flops(r0, n, r1, degree, RM0, RM1, RK0, RK1)


def profile_start(ctx):
    _check(lib.iga_profile_start(ctx))


def profile_stop(ctx) -> dict:
    """Per operator and precision (0: M FP64, 1: K FP64, 2: M FP32, 3: K FP32, 4: M BF16,
    5: K BF16): banded stages timed, kernel launches, summed ms, flops."""
    out = Profile()
    _check(lib.iga_profile_stop(ctx, C.byref(out)))
    return out.as_dict()


PEAK_KEYS = ("mfma_f64_4x4x4_tflops", "mfma_f64_16x16x4_tflops", "mfma_f32_16x16x4_tflops",
             "mfma_bf16_16x16x32_tflops", "hbm_copy_gbps", "hbm_read_gbps")


def measure_peaks(ctx) -> dict:
    """Measured device ceilings from the library's probe kernels (iga_measure_peaks)."""
    out = (C.c_double * 6)()
    _check(lib.iga_measure_peaks(ctx, out))
    return dict(zip(PEAK_KEYS, list(out)))


def objective(ctx, kkt, yhat, f) -> float:
    """J = 1/2 (y - yhat)^T M (y - yhat) + beta/2 u^T M u at the solution handle f."""
    out = C.c_double()
    _check(lib.iga_objective(ctx, kkt, yhat, f, C.byref(out)))
    return out.value


def grad_yhat(ctx, kkt, yhat, f, n):
    """dJ/dyhat = -M (y - yhat) as a CUDA tensor of shape n (FP64)."""
    import torch
    out = torch.empty(tuple(n), dtype=torch.float64, device="cuda")
    _check(lib.iga_grad_yhat(ctx, kkt, yhat, f, C.c_void_p(out.data_ptr())))
    return out


def grad_geometry(ctx, geo, degree: int, n, beta: float, yhat, f, p_interp: int = 0, nquad: int = 0):
    """dJ/d(control points), numpy array shaped like geo.ctrl."""
    knots = [_host(k) for k in geo.knots]
    ctrl = _host(geo.ctrl)
    g = Geometry()
    g.degree = int(geo.degree)
    for d in range(3):
        g.ncp[d] = int(ctrl.shape[1 + d])
        g.knots[d] = _dptr(knots[d])
    g.ctrl = _dptr(ctrl)
    o = AssemblyOpts(int(p_interp), int(nquad), 0.0, 0)
    nn = I3(*[int(v) for v in (n if hasattr(n, "__len__") else (n, n, n))])
    out = np.zeros(ctrl.shape, dtype=np.float64)
    _check(lib.iga_grad_geometry(ctx, C.byref(g), int(degree), nn, C.byref(o), float(beta), yhat, f, _dptr(out)))
    return out


def tt_info(t):
    """(n, r) of a TT handle."""
    n, r = I3(), I4()
    _check(lib.iga_tt_info(t, n, r))
    return list(n), list(r)


def tt_get_cores(ctx, t):
    """The three cores of a TT handle as host arrays [r_d][n_d][r_{d+1}]."""
    n, r = tt_info(t)
    out = []
    for d in range(3):
        c = np.empty((r[d], n[d], r[d + 1]), dtype=np.float64)
        _check(lib.iga_tt_get_core(ctx, t, d, _dptr(c)))
        out.append(c)
    return out


def tt_from_full(ctx, full, rel_tol: float = 0.0):
    """TT (library handle) of a contiguous FP64 CUDA tensor of shape (n0, n1, n2)."""
    assert full.is_cuda and full.dtype.is_floating_point and full.dim() == 3 and full.is_contiguous()
    out = P()
    _check(lib.iga_tt_from_full(ctx, I3(*full.shape), C.c_void_p(full.data_ptr()), float(rel_tol), C.byref(out)))
    return out


def tt_round(ctx, t, rel_tol: float = 0.0):
    """New TT handle: the rounding of t to the relative Frobenius tolerance rel_tol."""
    out = P()
    _check(lib.iga_tt_round(ctx, t, float(rel_tol), C.byref(out)))
    return out



def local_matvec_batched(ctx, problems, precision=FP64, autotune=True):
    """problems: list of dicts with keys r0, n, r1, degree, RM0, RM1, RK0, RK1, beta and CUDA FP64
    tensors PhiL_M, PhiR_M, PhiL_K, PhiR_K, Mcore, Kcore, x, y (y is written)."""
    arr = (LocalProblem * max(len(problems), 1))()
    for i, q in enumerate(problems):
        e = arr[i]
        for k in ("r0", "n", "r1", "degree", "RM0", "RM1", "RK0", "RK1"):
            setattr(e, k, int(q[k]))
        e.beta = float(q["beta"])
        for k in ("PhiL_M", "PhiR_M", "PhiL_K", "PhiR_K", "Mcore", "Kcore", "x", "y"):
            t = q[k]
            assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous()
            setattr(e, k, t.data_ptr())
    _check(lib.iga_local_matvec_batched(ctx, len(problems), arr, int(precision), int(bool(autotune))))
