"""FP64 rounding of the oracle against a 50-digit evaluation (mpmath), N <= 8.

This is a precision check of the oracle's arithmetic, not a pin of its
formulas (the closed forms, worked examples and brute-force checks in
test_oracle_pins.py pin those): the definition is evaluated here a second time
at 50 digits -- the frame, the curvatures of Eq. (MeanAndGaussCurvatures), the
principal direction of Eq. (PrincipalDirections) with the longer-row reading,
the floored radii, the center Q*(0,0) + n*/kappa_min, the torus distance of
Eq. (SingleTorusSDF) and the blend of Eq. (BasicFormulaShifted) with
lambda_x = 2C/M -- on inputs chosen away from the readings' thresholds (ties,
the umbilic fallback, the frame switch), so both sides take the same branches.
The cases include nearly flat points, whose floored radii (about 1e6 D) make
the plain FP64 torus distance cancel.
"""

import numpy as np
import pytest

import oracle

mp = pytest.importorskip("mpmath")
mp.mp.dps = 50


def _vec(v):
    return [mp.mpf(float(c)) for c in v]


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _unit(a):
    l = mp.sqrt(_dot(a, a))
    return [c / l for c in a]


def _torus(p, n, a, kfloor):
    """(c, u, R, r, sign) of one point at 50 digits."""
    a00, a01, a10, a11, a02, a20 = [mp.mpf(float(c)) for c in a]
    nh = _unit(_vec(n))
    e = [mp.mpf(1), mp.mpf(0), mp.mpf(0)] if abs(nh[0]) < mp.mpf("0.9") else [mp.mpf(0), mp.mpf(1), mp.mpf(0)]
    en = _dot(e, nh)
    s = _unit([e[i] - en * nh[i] for i in range(3)])
    t = _cross(nh, s)
    E, G, F = 1 + a10 ** 2, 1 + a01 ** 2, a10 * a01
    A = mp.sqrt(1 + a01 ** 2 + a10 ** 2)
    H = (a02 * E + a20 * G - a11 * F) / A ** 3
    K = (4 * a02 * a20 - a11 ** 2) / A ** 4
    root = mp.sqrt(max(H * H - K, mp.mpf(0)))
    kp, km = H + root, H - root
    kmin, kmax = (kp, km) if abs(kp) < abs(km) else (km, kp)
    r1 = (kmin * F * A - a11, 2 * a20 - kmin * E * A)
    r2 = (2 * a02 - kmin * G * A, kmin * F * A - a11)
    w = r2 if r2[0] ** 2 + r2[1] ** 2 > r1[0] ** 2 + r1[1] ** 2 else r1
    v = _unit([w[0] * (s[i] + a10 * nh[i]) + w[1] * (t[i] + a01 * nh[i]) for i in range(3)])
    ns = [(nh[i] - a10 * s[i] - a01 * t[i]) / A for i in range(3)]

    def floor(k):
        sg = mp.mpf(1) if k > 0 else mp.mpf(-1)
        return sg * max(abs(k), kfloor)

    kminf, kmaxf = floor(kmin), floor(kmax)
    L, r = 1 / abs(kminf), 1 / abs(kmaxf)
    zeta = 1 if kminf * kmaxf > 0 else -1
    R = L - zeta * r
    sign = 1 if kmaxf < 0 else -1
    o = [mp.mpf(float(p[i])) + a00 * nh[i] for i in range(3)]
    c = [o[i] + ns[i] / kminf for i in range(3)]
    u = _unit(_cross(ns, v))
    return c, u, R, r, sign


def _phi(p, n, a, x, C=64):
    pts = np.asarray(p, np.float64)
    D = float(np.linalg.norm(pts.max(0) - pts.min(0))) or 1.0
    kfloor = mp.mpf(1e-6) / mp.mpf(D)
    tori = [_torus(p[i], n[i], a[i], kfloor) for i in range(len(p))]
    P = [_vec(q) for q in p]
    out = []
    for xq in x:
        X = _vec(xq)
        d = [mp.sqrt(_dot([X[j] - Pi[j] for j in range(3)], [X[j] - Pi[j] for j in range(3)])) for Pi in P]
        M = max(d)
        lam = 2 * C / M
        num = den = mp.mpf(0)
        for (c, u, R, r, sign), di in zip(tori, d):
            v = [X[j] - c[j] for j in range(3)]
            h = _dot(v, u)
            rho = mp.sqrt(max(_dot(v, v) - h * h, mp.mpf(0)))
            g = sign * (mp.sqrt((rho - R) ** 2 + h * h) - r)
            wgt = mp.exp(-lam * (di - M / 2))
            num += wgt * g
            den += wgt
        out.append(num / den)
    return np.array([float(v) for v in out]), max(float(t[2]) for t in tori)


def _case(seed, N, flat=0):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1.0, 1.0, size=(N, 3))
    n = rng.normal(size=(N, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    a = np.zeros((N, 6))
    a[:, 0] = rng.uniform(-0.02, 0.02, N)               # a00
    a[:, 1:3] = rng.uniform(-0.3, 0.3, (N, 2))          # a01, a10
    a[:, 3] = rng.uniform(0.1, 0.4, N) * rng.choice([-1, 1], N)   # a11
    a[:, 4] = rng.uniform(-0.9, -0.2, N)                # a02
    a[:, 5] = rng.uniform(0.2, 0.9, N) * rng.choice([-1, 1], N)   # a20 (elliptic and saddle points)
    for i in range(flat):                                # nearly flat: both curvatures floored
        a[i, 3:6] = (1e-9, -3e-9, 2e-9)
    x = rng.uniform(-1.5, 1.5, size=(12, 3))
    # keep the frame choice and the curvature ordering away from their switches
    assert np.all(np.abs(np.abs(n[:, 0]) - 0.9) > 1e-3)
    return p, n, a, x


@pytest.mark.parametrize("seed,N,flat", [(1, 1, 0), (2, 3, 0), (3, 8, 0), (4, 8, 2), (5, 5, 5)])
def test_oracle_fp64_against_50_digits(seed, N, flat):
    p, n, a, x = _case(seed, N, flat)
    ref, Rmax = _phi(p, n, a, x)
    got = oracle.sdf(p, n, a, x)
    err = np.abs(got - ref)
    # FP64 rounding of the plain torus distance: a few ulp of |x - c| + R, i.e.
    # of the largest radius (1e6 D for floored curvatures), passed through the
    # normalised weights
    tol = 1e-13 + 32 * np.finfo(np.float64).eps * Rmax
    print(f"N={N} flat={flat}: max |oracle - 50 digits| {err.max():.3e}, largest R {Rmax:.3e}, tol {tol:.3e}",
          flush=True)
    assert np.all(err <= tol)
