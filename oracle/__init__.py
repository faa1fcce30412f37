"""Plain double-precision oracle for "Points as Tori" (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.  The C++ source is ``pts_oracle.cpp`` in this folder.
Each function there cites the passage of the paper it follows (Sec. 4.1 torus
fitting, Sec. 4.2 Eqs. (BasicFormulaShifted)/(RelationshipBetweenLambdaAndRadius),
Sec. 5.3 sphere tracing, Sec. 4.2 radius-limited evaluation).  Derivatives
(in x, the coefficients a, the points p and normals n, and the Laplacian in x)
are exact derivatives of the same code, via forward-mode dual and hyper-dual
numbers.

Parity pins (see ``tests/test_oracle_pins.py``): sphere closed form (values and
Laplacian 2/|x|), single torus vs. brute-force surface distance, torus round
trip, principal curvatures vs. a generic shape-operator computation,
orientation/scale/translation/permutation invariances, the large-C
nearest-point limit, finite differences for every gradient and the Laplacian,
brute-force nearest neighbours for the radius-limited evaluation, and for the
two baselines the planar closed form, the screened Laplace equation the
double-layer sum satisfies, area-weight and orientation identities and the
nearest-point limit.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pts_oracle.cpp")
_LIB = os.path.join(_HERE, "_pts_oracle.so")

C_DEFAULT = 64.0          # Sec. 4.2: "We use C = 64"
KFLOOR_REL = 1e-6         # R-floor: kappa_floor = 1e-6 / bbox diagonal
TSTRIDE = 32

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/_pts_oracle.so`` (g++, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.orc_version.restype = ctypes.c_int
        L.orc_threads.argtypes = [ctypes.c_int]
        L.orc_threads.restype = ctypes.c_int
        L.orc_bbox_diag.argtypes = [i64, P]
        L.orc_bbox_diag.restype = ctypes.c_double
        L.orc_frame.argtypes = [i64, P, P]
        L.orc_frame.restype = None
        L.orc_fit.argtypes = [i64, P, P, P, ctypes.c_double, ctypes.c_int, P]
        L.orc_fit.restype = ctypes.c_int
        L.orc_torus_g.argtypes = [i64, P, i64, P, P]
        L.orc_torus_g.restype = None
        L.orc_eval.argtypes = [i64, P, P, i64, P, ctypes.c_double, ctypes.c_int, P, P, P]
        L.orc_eval.restype = ctypes.c_int
        L.orc_grad_a.argtypes = [i64, P, P, P, ctypes.c_double, ctypes.c_int, i64, P,
                                 ctypes.c_double, P, ctypes.c_int, P]
        L.orc_grad_a.restype = ctypes.c_int
        L.orc_trace.argtypes = [i64, P, P, i64, P, P, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int, P, P, P, P]
        L.orc_trace.restype = ctypes.c_int
        L.orc_eval_baseline.argtypes = [i64, P, P, P, i64, P, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int, P, P, P]
        L.orc_eval_baseline.restype = ctypes.c_int
        L.orc_laplacian.argtypes = [i64, P, P, i64, P, ctypes.c_double, ctypes.c_int, P]
        L.orc_laplacian.restype = ctypes.c_int
        L.orc_grad_points.argtypes = [i64, P, P, P, ctypes.c_double, ctypes.c_int, i64, P, ctypes.c_double, P,
                                      ctypes.c_int, P, P, P]
        L.orc_grad_points.restype = ctypes.c_int
        L.orc_knn_mean.argtypes = [i64, P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.orc_knn_mean.restype = ctypes.c_int
        L.orc_eval_radius.argtypes = [i64, P, P, i64, P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, P, P]
        L.orc_eval_radius.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a, shape_last=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape_last is not None:
        a = a.reshape(-1, shape_last)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def threads(n: int = 0) -> int:
    """Set (n > 0) and return the number of OpenMP threads the oracle uses."""
    return lib().orc_threads(int(n))


def bbox_diag(p) -> float:
    p = _f64(p, 3)
    return float(lib().orc_bbox_diag(p.shape[0], _ptr(p)))


def kfloor_for(p) -> float:
    """R-floor: kappa_floor = 1e-6 / D with D the bbox diagonal (D = 1 when it is 0)."""
    D = bbox_diag(p)
    return KFLOOR_REL / (D if D > 0.0 else 1.0)


def frame(n):
    """(s, t, n_hat) per point, the fixed tangent frame reading (R-frame)."""
    n = _f64(n, 3)
    out = np.zeros((n.shape[0], 9))
    lib().orc_frame(n.shape[0], _ptr(n), _ptr(out))
    return out[:, 0:3], out[:, 3:6], out[:, 6:9]


class Tori:
    """Fitted tori of Sec. 4.1, one row per point (double precision)."""

    def __init__(self, raw: np.ndarray):
        self.raw = raw
        self.c = raw[:, 0:3]
        self.u = raw[:, 3:6]
        self.R = raw[:, 6]
        self.r = raw[:, 7]
        self.sgn = raw[:, 8]
        self.kmin = raw[:, 9]
        self.kmax = raw[:, 10]
        self.kminf = raw[:, 11]
        self.kmaxf = raw[:, 12]
        self.nstar = raw[:, 13:16]
        self.vmin = raw[:, 16:19]
        self.o = raw[:, 19:22]
        self.H = raw[:, 22]
        self.K = raw[:, 23]
        self.umbilic = raw[:, 24].astype(bool)
        self.kplus = raw[:, 25]
        self.kminus = raw[:, 26]

    def __len__(self):
        return self.raw.shape[0]


def fit(p, n, a, kfloor: float | None = None, center_mode: int = 0) -> Tori:
    """Torus fitting (Sec. 4.1).  a is [N,6] = (a00, a01, a10, a11, a02, a20)."""
    p = _f64(p, 3)
    n = _f64(n, 3)
    a = _f64(a, 6)
    if kfloor is None:
        kfloor = kfloor_for(p)
    out = np.zeros((p.shape[0], TSTRIDE))
    rc = lib().orc_fit(p.shape[0], _ptr(p), _ptr(n), _ptr(a), float(kfloor), int(center_mode), _ptr(out))
    if rc != 0:
        raise ValueError("oracle fit: zero-length normal")
    return Tori(out)


def torus_g(tori: Tori, x) -> np.ndarray:
    """g_i(x_q) = sign(T_i) phi_T_i(x_q) for all pairs, [Q, N] (Eq. SingleTorusSDF)."""
    x = _f64(x, 3)
    N = len(tori)
    out = np.zeros((x.shape[0], N))
    lib().orc_torus_g(N, _ptr(tori.raw), x.shape[0], _ptr(x), _ptr(out))
    return out


def eval_sdf(p, tori: Tori, x, C: float = C_DEFAULT, grad: bool = False, stats: bool = False,
             nthreads: int = 0):
    """phi(x) of Eq. (BasicFormulaShifted); optionally grad phi and (M, W, phi)."""
    p = _f64(p, 3)
    x = _f64(x, 3)
    Q = x.shape[0]
    phi = np.zeros(Q)
    g = np.zeros((Q, 3)) if grad else None
    st = np.zeros((Q, 3)) if stats else None
    rc = lib().orc_eval(p.shape[0], _ptr(p), _ptr(tori.raw), Q, _ptr(x), float(C), int(nthreads),
                        _ptr(phi), _ptr(g), _ptr(st))
    if rc != 0:
        raise ValueError("oracle eval: empty cloud")
    out = [phi]
    if grad:
        out.append(g)
    if stats:
        out.append(st)
    return out[0] if len(out) == 1 else tuple(out)


def sdf(p, n, a, x, C: float = C_DEFAULT, kfloor: float | None = None, center_mode: int = 0,
        grad: bool = False, stats: bool = False, nthreads: int = 0):
    """Fit tori, then evaluate phi at x (Algorithm 1, both stages)."""
    return eval_sdf(p, fit(p, n, a, kfloor, center_mode), x, C, grad, stats, nthreads)


def grad_a(p, n, a, x, gout, C: float = C_DEFAULT, kfloor: float | None = None,
           center_mode: int = 0, nthreads: int = 0) -> np.ndarray:
    """dL/da, [N,6], for L = sum_q gout_q phi(x_q)."""
    p = _f64(p, 3)
    n = _f64(n, 3)
    a = _f64(a, 6)
    x = _f64(x, 3)
    gout = _f64(gout).reshape(-1)
    if kfloor is None:
        kfloor = kfloor_for(p)
    ga = np.zeros((p.shape[0], 6))
    rc = lib().orc_grad_a(p.shape[0], _ptr(p), _ptr(n), _ptr(a), float(kfloor), int(center_mode),
                          x.shape[0], _ptr(x), float(C), _ptr(gout), int(nthreads), _ptr(ga))
    if rc != 0:
        raise ValueError("oracle grad_a: empty cloud")
    return ga


BASELINE_KINDS = {"sspd": 0, "shc": 1}


def eval_baseline(p, n, x, kind: str, area=None, C: float = C_DEFAULT, lam_fixed: float = 0.0,
                  raw: bool = False, nthreads: int = 0):
    """Smoothed signed planar distance ('sspd', Eq. SmoothedSignedPlanarDistance) or signed Hopf-Cole
    distance ('shc', Eq. ScreenedWindingNumber) at x [Q,3]; with raw, also the weighted sum itself and
    the sum of the absolute values of its terms: (phi, sum, abs_sum)."""
    p = _f64(p, 3)
    n = _f64(n, 3)
    x = _f64(x, 3)
    A = None if area is None else np.ascontiguousarray(np.asarray(area, dtype=np.float64).reshape(-1))
    if A is not None and A.shape[0] != p.shape[0]:
        raise ValueError("area must have one value per point")
    out = np.zeros(x.shape[0])
    r = np.zeros(x.shape[0]) if raw else None
    ra = np.zeros(x.shape[0]) if raw else None
    rc = lib().orc_eval_baseline(p.shape[0], _ptr(p), _ptr(n), _ptr(A), x.shape[0], _ptr(x), float(C),
                                 BASELINE_KINDS[kind], float(lam_fixed), int(nthreads), _ptr(out), _ptr(r),
                                 _ptr(ra))
    if rc != 0:
        raise ValueError("oracle baseline: empty cloud or unknown kind")
    return (out, r, ra) if raw else out


def laplacian(p, tori: Tori, x, C: float = C_DEFAULT, nthreads: int = 0) -> np.ndarray:
    """Laplacian of phi (Eq. BasicFormulaShifted, lambda_x moving with x; App. D), [Q]."""
    p = _f64(p, 3)
    x = _f64(x, 3)
    lap = np.zeros(x.shape[0])
    if lib().orc_laplacian(p.shape[0], _ptr(p), _ptr(tori.raw), x.shape[0], _ptr(x), float(C), int(nthreads),
                           _ptr(lap)) != 0:
        raise ValueError("oracle laplacian: empty cloud")
    return lap


def grad_points(p, n, a, x, gout, C: float = C_DEFAULT, kfloor: float | None = None, center_mode: int = 0,
                nthreads: int = 0):
    """(dL/da [N,6], dL/dp [N,3], dL/dn [N,3]) for L = sum_q gout_q phi(x_q): exact derivatives through
    each point's torus fit, its weight and (as the farthest point of a query) lambda_x."""
    p = _f64(p, 3)
    n = _f64(n, 3)
    a = _f64(a, 6)
    x = _f64(x, 3)
    gout = _f64(gout).reshape(-1)
    if kfloor is None:
        kfloor = kfloor_for(p)
    N = p.shape[0]
    ga, gp, gn = np.zeros((N, 6)), np.zeros((N, 3)), np.zeros((N, 3))
    rc = lib().orc_grad_points(N, _ptr(p), _ptr(n), _ptr(a), float(kfloor), int(center_mode), x.shape[0],
                               _ptr(x), float(C), _ptr(gout), int(nthreads), _ptr(ga), _ptr(gp), _ptr(gn))
    if rc != 0:
        raise ValueError("oracle grad_points: empty cloud")
    return ga, gp, gn


def trace(p, tori: Tori, org, dirs, steps: int, eps: float, tmax: float, C: float = C_DEFAULT,
          nthreads: int = 0):
    """Sphere tracing (Sec. 5.3): returns (t, hit, nsteps, normal)."""
    p = _f64(p, 3)
    org = _f64(org, 3)
    dirs = _f64(dirs, 3)
    R = org.shape[0]
    t = np.zeros(R)
    hit = np.zeros(R, dtype=np.int32)
    ns = np.zeros(R, dtype=np.int32)
    nrm = np.zeros((R, 3))
    rc = lib().orc_trace(p.shape[0], _ptr(p), _ptr(tori.raw), R, _ptr(org), _ptr(dirs), int(steps),
                         float(eps), float(tmax), float(C), int(nthreads), _ptr(t), _ptr(hit),
                         _ptr(ns), _ptr(nrm))
    if rc != 0:
        raise ValueError("oracle trace: empty cloud")
    return t, hit.astype(bool), ns, nrm


def knn_mean(p, k: int = 64, nthreads: int = 0) -> float:
    """Mean over points of the mean distance to their k nearest other points
    (Sec. 4.2, "Acceleration and adaptive lambda"); 1.0 for a single point."""
    p = _f64(p, 3)
    out = ctypes.c_double(0.0)
    if lib().orc_knn_mean(p.shape[0], _ptr(p), int(k), int(nthreads), ctypes.byref(out)) != 0:
        raise ValueError("oracle knn_mean: empty cloud")
    return float(out.value)


def radius_params(p, C: float = C_DEFAULT, k: int = 64, nthreads: int = 0):
    """(D, lambda, R_eval) of the radius-limited evaluation: lambda = 1e3 / D,
    R_eval = 2 C / lambda (Sec. 4.2)."""
    D = knn_mean(p, k, nthreads)
    lam = 1e3 / D
    return D, lam, 2.0 * C / lam


def eval_radius(p, tori: Tori, x, lam: float, reval: float, kfb: int = 32, nthreads: int = 0):
    """Radius-limited phi (Sec. 4.2): blend over the points within reval of x
    with the constant lambda, else over the kfb nearest.  Returns (phi, count),
    count = points blended, negative for the nearest-point fallback."""
    p = _f64(p, 3)
    x = _f64(x, 3)
    Q = x.shape[0]
    phi = np.zeros(Q)
    cnt = np.zeros(Q, dtype=np.int32)
    rc = lib().orc_eval_radius(p.shape[0], _ptr(p), _ptr(tori.raw), Q, _ptr(x), float(lam), float(reval),
                               int(kfb), int(nthreads), _ptr(phi), _ptr(cnt))
    if rc != 0:
        raise ValueError("oracle eval_radius: empty cloud")
    return phi, cnt
