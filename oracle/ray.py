"""ctypes binding of the per-ray C oracle (``ray_oracle.c``).

Test infrastructure only.  Each screen point is one backward ray (the paper
treats ray tracing as sampling an intensity function I(x) on the screen,
Sec. 3 opening paragraph); everything per ray is this project's written method.
"""
import ctypes
import os

import numpy as np

from . import build as _build

G_CGS = 6.67430e-8
C_CGS = 2.99792458e10
MSUN_CGS = 1.98847e33

MODEL_IDS = {"toy_disk": 1, "thermal": 2, "grid": 3, "screen_ring": 10, "screen_poly": 11}
STATUS = {0: "ok", 1: "captured", 2: "escaped", 3: "step_cap", 4: "thick", 5: "nan"}


class OrParams(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_double), ("r_cam", ctypes.c_double), ("inc", ctypes.c_double),
        ("r_out", ctypes.c_double), ("eps", ctypes.c_double),
        ("max_steps", ctypes.c_int32), ("nstokes", ctypes.c_int32),
        ("model", ctypes.c_int32), ("nsub", ctypes.c_int32),
        ("freq", ctypes.c_double), ("L_cm", ctypes.c_double),
        ("mp", ctypes.c_double * 16),
        ("grid", ctypes.POINTER(ctypes.c_float)),
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
        ("pad2", ctypes.c_int32),
        ("gp", ctypes.c_double * 8),
        ("phi_cam", ctypes.c_double),
    ]


MAX_SUB = 8          # subring planes the C oracle can accumulate

FEAT_DTYPE = np.dtype([("rmin", np.float32), ("ncross", np.int32),
                       ("steps", np.int32), ("status", np.int32)])

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_trace.argtypes = [ctypes.POINTER(OrParams), ctypes.c_int, dp, dp, dp,
                               ctypes.c_void_p, ctypes.c_int]
        L.or_trace.restype = ctypes.c_int
        L.or_null_norm.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.or_null_norm.restype = ctypes.c_double
        L.or_geo_rhs.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_camera.argtypes = [ctypes.POINTER(OrParams), ctypes.c_double, ctypes.c_double,
                                dp, dp, dp, dp, dp]
        L.or_walker_penrose.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        dp, dp, dp]
        L.or_r_isco.argtypes = [ctypes.c_double]
        L.or_r_isco.restype = ctypes.c_double
        L.or_circ_EL.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_flow_u.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.or_thermal_coefs.argtypes = [ctypes.c_double] * 5 + [dp]
        L.or_lorentz_exp.argtypes = [ctypes.c_double, dp, dp, ctypes.c_double, dp]
        L.or_transfer_step4.argtypes = [dp, dp, ctypes.c_double, dp, dp, dp, ctypes.c_double]
        L.or_trace_path.argtypes = [ctypes.POINTER(OrParams), ctypes.c_double, ctypes.c_double,
                                    dp, ctypes.c_void_p, dp, ctypes.c_int, dp]
        L.or_trace_path.restype = ctypes.c_int
        L.or_plasma_point.argtypes = [ctypes.POINTER(OrParams), ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_plasma_point.restype = ctypes.c_int
        _lib = L
    return _lib


def default_threads():
    """Threads of a trace call: the process's CPUs, at most 16 (the CPU share
    of one GPU on the machines this runs on beside a GPU job)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _dp(x):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def length_unit_cm(mass_msun):
    """Gravitational radius GM/c^2 in cm."""
    return G_CGS * mass_msun * MSUN_CGS / C_CGS ** 2


def make_params(cfg, grid=None):
    """Build the C parameter block from a workload dictionary."""
    p = OrParams()
    p.a = float(cfg["a"])
    p.r_cam = float(cfg["r_cam"])
    p.inc = np.deg2rad(float(cfg["inc_deg"]))
    p.phi_cam = np.deg2rad(float(cfg.get("phi_deg", 0.0)))
    p.r_out = float(cfg.get("r_out", cfg["r_cam"]))
    p.eps = float(cfg.get("eps", 0.03))
    p.max_steps = int(cfg.get("max_steps", 100000))
    p.nstokes = int(cfg.get("nstokes", 1))
    p.nsub = int(cfg.get("subrings", 0))
    p.model = MODEL_IDS[cfg["model"]] if isinstance(cfg["model"], str) else int(cfg["model"])
    p.freq = float(cfg.get("freq_hz", 230e9))
    p.L_cm = length_unit_cm(float(cfg.get("mass_msun", 4.0e6)))
    mp = list(cfg.get("mp", []))
    for i in range(16):
        p.mp[i] = float(mp[i]) if i < len(mp) else 0.0
    if grid is not None:
        p.grid = grid.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        p.n1, p.n2, p.n3 = grid.shape[3], grid.shape[2], grid.shape[1]
        gp = list(cfg.get("gp", []))
        for i in range(8):
            p.gp[i] = float(gp[i]) if i < len(gp) else 0.0
    return p


def trace(cfg, alpha, beta, nthreads=None, grid=None):
    """Trace rays through screen points (alpha, beta) [M].

    Returns (S, feat): S is (n, nstokes + subrings) float64 (Stokes, then the
    subring planes of I), feat a structured array with fields rmin, ncross,
    steps, status.
    """
    alpha = np.ascontiguousarray(alpha, dtype=np.float64).ravel()
    beta = np.ascontiguousarray(beta, dtype=np.float64).ravel()
    n = alpha.size
    p = make_params(cfg, grid)
    S = np.zeros((n, p.nstokes + p.nsub), dtype=np.float64)
    feat = np.zeros(n, dtype=FEAT_DTYPE)
    if n == 0:
        return S, feat
    if nthreads is None:
        nthreads = default_threads()
    lib().or_trace(ctypes.byref(p), n, _dp(alpha), _dp(beta), _dp(S),
                   feat.ctypes.data_as(ctypes.c_void_p), int(nthreads))
    return S, feat


def screen_coords(fov, nx, ny, i, j):
    """Screen coordinates of vertex (i, j) on an nx x ny vertex grid spanning
    [-fov/2, fov/2] in x with square cells (Sec. 3.2 grid of n0x x n0y points)."""
    dx = fov / (nx - 1)
    x0 = -0.5 * fov
    y0 = -0.5 * dx * (ny - 1)
    return x0 + np.asarray(i, dtype=np.float64) * dx, y0 + np.asarray(j, dtype=np.float64) * dx


def trace_path(cfg, alpha, beta, cap=200000, grid=None):
    """Trace one ray and return (S, feat, states, kt, kph): states is (n, 6)
    with columns r, theta, phi, k_r (Kerr-Schild), k_theta, step length."""
    p = make_params(cfg, grid)
    S = np.zeros(4 + MAX_SUB)
    feat = np.zeros(1, dtype=FEAT_DTYPE)
    rec = np.zeros((cap, 6))
    kk = np.zeros(2)
    n = lib().or_trace_path(ctypes.byref(p), float(alpha), float(beta), _dp(S),
                            feat.ctypes.data_as(ctypes.c_void_p), _dp(rec), cap, _dp(kk))
    return S[:p.nstokes], feat[0], rec[:n].copy(), kk[0], kk[1]


def plasma_point(cfg, alpha, beta, y, grid=None):
    """Coefficients per unit affine length at state y = (r, theta, phi, k_r,
    k_theta) of the ray through (alpha, beta): (emits, J[4], alpha_I,
    alpha_QUV[3], rho_QUV[3])."""
    p = make_params(cfg, grid)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(11)
    ok = lib().or_plasma_point(ctypes.byref(p), float(alpha), float(beta), _dp(yy), _dp(out))
    return bool(ok), out[:4], out[4], out[5:8], out[8:11]


_count_lib = None


def count_ops(cfg, alpha, beta, grid=None):
    """Operation counts of the oracle's rays through (alpha, beta), from its
    instrumented build (opcount.cpp): structured array with steps, emitting
    steps and the operations (+, -, *, /, sqrt and transcendental calls) of
    the geodesic, of the plasma point (its non-emitting calls separately)
    and of the transfer update."""
    global _count_lib
    if _count_lib is None:
        L = ctypes.CDLL(_build.build_count())
        L.or_count_ray.argtypes = [ctypes.POINTER(OrParams), ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]
        L.or_count_ray.restype = ctypes.c_int
        L.or_count_probe.argtypes = [ctypes.c_int]
        L.or_count_probe.restype = ctypes.c_longlong
        _count_lib = L
    p = make_params(cfg, grid)
    alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    dt = np.dtype([("steps", np.int64), ("emit", np.int64), ("geo", np.int64), ("plasma", np.int64),
                   ("transfer", np.int64), ("plasma_noemit", np.int64), ("S", np.float64, 4)])
    out = np.zeros(alpha.size, dtype=dt)
    buf = np.zeros(6, dtype=np.int64)
    sb = np.zeros(4)
    for k in range(alpha.size):
        _count_lib.or_count_ray(ctypes.byref(p), float(alpha[k]), float(beta[k]),
                                buf.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), _dp(sb))
        out[k] = tuple(buf) + (sb.copy(),)
    return out


def count_probe(which):
    """Operations the counter records for one oracle routine (0: a 4x4
    matrix product, 1: the horizon radius)."""
    count_ops({"a": 0.0, "r_cam": 1000.0, "inc_deg": 60.0, "model": "toy_disk"}, [], [])
    return int(_count_lib.or_count_probe(int(which)))
