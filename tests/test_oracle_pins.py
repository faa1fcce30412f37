"""Pins of the double-precision oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each compares it with a closed
form, a worked example, an invariance of the definition, an independent
generic computation (shape operator of a parametrised surface, brute-force
distance to a sampled torus) or finite differences.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2607_16946_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "torus_cases.json")


def _sphere(N, radius=1.0, seed=0, shift=0.0, inward=False):
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(N, 3))
    u = z / np.linalg.norm(z, axis=1, keepdims=True)
    p = radius * u
    n = -u if inward else u.copy()
    k = 1.0 / (radius + shift)          # curvature of the shifted sphere
    a = np.zeros((N, 6))
    a[:, 0] = shift
    a[:, 4] = a[:, 5] = (0.5 * k) if inward else (-0.5 * k)
    return p, n, a


def _rot(seed):
    return synth.random_rotation(np.random.default_rng(seed))


# ---------------------------------------------------------------------------
# Closed forms and worked examples
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("radius,shift,C", [(1.0, 0.0, 64.0), (2.5, 0.0, 64.0), (1.0, 0.3, 64.0),
                                             (0.7, -0.2, 20.0)])
def test_sphere_closed_form(radius, shift, C):
    # Sec. 5.1 initialisation a02 = a20 = -1/2 is the tangent unit sphere; every
    # fitted torus is then the same sphere, so the blend (a partition of unity)
    # returns |x| - (radius + shift) exactly, for any weights.
    p, n, a = _sphere(600, radius, seed=1, shift=shift)
    x = np.random.default_rng(2).uniform(-2.5, 2.5, size=(300, 3)) * radius
    phi = oracle.sdf(p, n, a, x, C=C)
    ref = np.linalg.norm(x, axis=1) - (radius + shift)
    assert np.max(np.abs(phi - ref)) < 1e-12 * max(1.0, radius)


def test_sphere_inward_normals_negate():
    p, n, a = _sphere(400, 1.3, seed=3, inward=True)
    x = np.random.default_rng(4).uniform(-2, 2, size=(200, 3))
    phi = oracle.sdf(p, n, a, x)
    assert np.max(np.abs(phi + (np.linalg.norm(x, axis=1) - 1.3))) < 1e-12


def test_golden_worked_examples():
    cases = json.load(open(GOLDEN))["cases"]
    for cs in cases:
        tor = oracle.fit([cs["p"]], [cs["n"]], [cs["a"]], kfloor=cs["kfloor"])
        ex = cs["expect"]
        assert np.allclose(tor.c[0], ex["c"], atol=1e-9, rtol=1e-12), cs["name"]
        assert abs(tor.R[0] - ex["R"]) < 1e-9 * max(1.0, ex["R"]), cs["name"]
        assert abs(tor.r[0] - ex["r"]) < 1e-12, cs["name"]
        assert tor.sgn[0] == ex["sgn"], cs["name"]
        if "axis" in ex:
            assert abs(abs(np.dot(tor.u[0], ex["axis"])) - 1.0) < 1e-12, cs["name"]
        g = oracle.torus_g(tor, cs["queries"])[:, 0]
        tol = cs.get("g_tol", 1e-12)
        assert np.max(np.abs(g - np.array(cs["g"]))) < tol, (cs["name"], g, cs["g"])
        # N = 1: the blend returns g itself (the single weight cancels).
        phi = oracle.eval_sdf([cs["p"]], tor, cs["queries"])
        assert np.max(np.abs(phi - np.array(cs["g"]))) < tol, cs["name"]


WEIGHTS = os.path.join(os.path.dirname(__file__), "golden", "blend_weights.json")


def test_blend_weights_three_spheres_hand_derived():
    """Sec. 4.2, Eqs. (BasicFormulaShifted), (RelationshipBetweenLambdaAndRadius); App. D: a hand-derived
    blend of three exact spheres whose two near points differ in distance by M/(2C), so that the
    weight ratio e^-(lambda delta) depends on the factor in lambda_x = 2C/M.  Checks the fit, phi,
    the statistics (M and the shifted weight sum W) and grad phi with its lambda_x term."""
    G = json.load(open(WEIGHTS))
    p, n, a, x = (np.array(G[k], dtype=np.float64) for k in ("p", "n", "a", "x"))
    tor = oracle.fit(p, n, a)
    assert np.allclose(tor.c, [[0.75, 0, 0], [0, 3 / 128 - 1, 0], [0, 0, -2]], atol=1e-14)
    assert np.allclose(tor.R, 0.0, atol=1e-14) and np.allclose(tor.r, [0.25, 2.0, 1.0], atol=1e-14)
    assert np.all(tor.sgn == 1.0)
    assert np.allclose(oracle.torus_g(tor, x[None])[0], G["cases"][0]["g"], atol=1e-14)
    for case in G["cases"]:
        phi, g, st = oracle.eval_sdf(p, tor, x[None], C=case["C"], grad=True, stats=True)
        assert abs(phi[0] - case["phi"]) <= 1e-13, (case["C"], phi[0], case["phi"])
        assert np.abs(g[0] - np.array(case["grad"])).max() <= 1e-11 * max(1.0, np.abs(case["grad"]).max())
        assert st[0, 0] == case["M"]
        assert abs(st[0, 1] - case["W"]) <= 1e-12 * case["W"]
        assert abs(st[0, 2] - case["phi"]) <= 1e-13


def test_blend_weights_pin_rejects_planted_misreadings():
    """The pin above fails for the plausible misreadings: lambda = C/M (the oracle run with C halved
    computes exactly that) moves phi by >= 0.027 and grad phi by >= 0.5; a dropped shift
    (w = exp(-lambda d)) leaves phi but scales W by e^-C."""
    G = json.load(open(WEIGHTS))
    p, n, a, x = (np.array(G[k], dtype=np.float64) for k in ("p", "n", "a", "x"))
    tor = oracle.fit(p, n, a)
    for case in G["cases"]:
        C = case["C"]
        phi, g, st = oracle.eval_sdf(p, tor, x[None], C=C / 2, grad=True, stats=True)
        assert abs(phi[0] - G["misreading_lambda_C_over_M_phi"][str(int(C))]) <= 1e-13
        assert abs(phi[0] - case["phi"]) > 0.025
        # grad of the misread phi at lambda = C/M differs in every component
        assert np.abs(g[0] - np.array(case["grad"])).max() > 0.1
        # dropped shift: W would be sum exp(-lambda d_i) = W exp(-lambda sigma) = W e^-C
        unshifted = sum(math.exp(-case["lambda"] * di) for di in case["d"])
        assert abs(unshifted - case["W"] * math.exp(-C)) <= 1e-12 * unshifted
        assert abs(unshifted - case["W"]) > 0.5 * case["W"]


def test_printed_center_fails_on_saddle():
    # The inner-equator case separates the two center readings: the printed
    # formula puts the torus axis on the wrong side (planted-mistake check).
    cs = json.load(open(GOLDEN))["cases"][1]
    tor = oracle.fit([cs["p"]], [cs["n"]], [cs["a"]], kfloor=cs["kfloor"], center_mode=1)
    assert np.allclose(tor.c[0], [4.0, 0.0, 0.0], atol=1e-12)
    g = oracle.torus_g(tor, cs["queries"][:1])[0, 0]
    assert abs(g - (-0.01)) < 1e-12
    # ... and on elliptic points both readings coincide.
    cs0 = json.load(open(GOLDEN))["cases"][0]
    t0 = oracle.fit([cs0["p"]], [cs0["n"]], [cs0["a"]], kfloor=cs0["kfloor"], center_mode=0)
    t1 = oracle.fit([cs0["p"]], [cs0["n"]], [cs0["a"]], kfloor=cs0["kfloor"], center_mode=1)
    assert np.allclose(t0.c, t1.c, atol=1e-12)


# ---------------------------------------------------------------------------
# Brute force: Eq. (SingleTorusSDF) is the distance to the torus surface
# ---------------------------------------------------------------------------

def _torus_surface_distance(c, u, R, r, x):
    """Unsigned distance from x to the ring torus (c, u, R, r) by dense sampling + local refinement."""
    from scipy.optimize import minimize
    u = u / np.linalg.norm(u)
    e1 = np.cross(u, [1.0, 0.0, 0.0])
    if np.linalg.norm(e1) < 0.5:
        e1 = np.cross(u, [0.0, 1.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)

    def surf(th, ps):
        rr = R + r * np.cos(th)
        return c + rr[..., None] * (np.cos(ps)[..., None] * e1 + np.sin(ps)[..., None] * e2) + \
            (r * np.sin(th))[..., None] * u

    th, ps = np.meshgrid(np.linspace(0, 2 * np.pi, 721), np.linspace(0, 2 * np.pi, 721), indexing="ij")
    S = surf(th, ps).reshape(-1, 3)
    out = []
    for xi in x:
        d = np.linalg.norm(S - xi, axis=1)
        j = int(np.argmin(d))
        t0 = np.array([th.reshape(-1)[j], ps.reshape(-1)[j]])
        f = lambda v: np.sum((surf(np.array(v[0]), np.array(v[1])) - xi) ** 2)  # noqa: E731
        res = minimize(f, t0, method="Nelder-Mead", options={"xatol": 1e-13, "fatol": 1e-26, "maxiter": 4000})
        out.append(math.sqrt(res.fun))
    return np.array(out)


@pytest.mark.parametrize("a", [
    [0.0, 0.0, 0.0, 0.0, -0.2, -0.6],     # elliptic, both convex
    [0.05, 0.0, 0.0, 0.1, 0.15, -0.7],    # saddle with a shift and a twist term
    [0.0, 0.0, 0.0, 0.0, -0.45, -0.1],    # elliptic, ring-dominant
])
def test_single_torus_matches_bruteforce_distance(a):
    p = np.array([[0.1, -0.2, 0.3]])
    n = np.array([[0.3, 0.5, 0.81]])
    tor = oracle.fit(p, n, [a], kfloor=1e-9)
    assert tor.R[0] > tor.r[0]  # ring torus: the formula is its exact SDF
    x = np.random.default_rng(5).normal(size=(12, 3)) * 2.0 + p
    g = oracle.torus_g(tor, x)[:, 0]
    dist = _torus_surface_distance(tor.c[0], tor.u[0], tor.R[0], tor.r[0], x)
    # inside/outside of the solid ring torus, from its own definition
    v = x - tor.c[0]
    h = v @ tor.u[0]
    rho = np.linalg.norm(v - h[:, None] * tor.u[0], axis=1)
    inside = (rho - tor.R[0]) ** 2 + h ** 2 < tor.r[0] ** 2
    signed = np.where(inside, -dist, dist) * tor.sgn[0]
    assert np.max(np.abs(g - signed)) < 1e-7
    # N = 1 blend is the single torus
    phi = oracle.eval_sdf(p, tor, x)
    assert np.max(np.abs(phi - g)) < 1e-13


# ---------------------------------------------------------------------------
# Torus fitting vs. independent geometry
# ---------------------------------------------------------------------------

def _monge_shape_operator(p, n, a):
    """Principal curvatures/directions of Q*(s,t) at (0,0) from the textbook
    shape operator of a parametrised surface, computed generically."""
    n = np.asarray(n, dtype=np.float64) / np.linalg.norm(n)
    s, t = synth.tangent_frame(n[None])
    s, t = s[0], t[0]
    a00, a01, a10, a11, a02, a20 = a
    Qs, Qt = a10, a01
    Qss, Qst, Qtt = 2 * a20, a11, 2 * a02
    Xs = s + Qs * n
    Xt = t + Qt * n
    N = np.cross(Xs, Xt)
    N /= np.linalg.norm(N)
    I = np.array([[Xs @ Xs, Xs @ Xt], [Xt @ Xs, Xt @ Xt]])
    II = np.array([[Qss * (n @ N), Qst * (n @ N)], [Qst * (n @ N), Qtt * (n @ N)]])
    S = np.linalg.solve(I, II)
    vals, vecs = np.linalg.eig(S)
    vals = vals.real
    vecs = vecs.real
    dirs = [vecs[0, k] * Xs + vecs[1, k] * Xt for k in range(2)]
    dirs = [d / np.linalg.norm(d) for d in dirs]
    return vals, dirs, N


def test_curvatures_and_directions_vs_shape_operator():
    rng = np.random.default_rng(7)
    for _ in range(300):
        a = rng.normal(size=6) * np.array([0.1, 0.6, 0.6, 0.8, 0.8, 0.8])
        n = rng.normal(size=3)
        p = rng.normal(size=3)
        tor = oracle.fit([p], [n], [a], kfloor=1e-12)
        vals, dirs, N = _monge_shape_operator(p, n, a)
        got = np.sort([tor.kplus[0], tor.kminus[0]])
        assert np.allclose(got, np.sort(vals), atol=1e-10, rtol=1e-10)
        assert np.allclose(tor.nstar[0], N, atol=1e-12)
        k_min_ref = vals[np.argmin(np.abs(vals))]
        assert abs(tor.kmin[0] - k_min_ref) < 1e-10 * max(1, abs(k_min_ref))
        if abs(abs(vals[0]) - abs(vals[1])) > 1e-6:
            dref = dirs[int(np.argmin(np.abs(vals)))]
            assert abs(abs(np.dot(tor.vmin[0], dref)) - 1.0) < 1e-8


def test_ellipsoid_curvatures_closed_form():
    # Gaussian and mean curvature of x^2/A^2 + y^2/B^2 + z^2/C^2 = 1 (textbook):
    # K = 1 / (A B C)^2 / h^4, |H| = |x|^2 - A^2 - B^2 - C^2 ... / (2 (ABC)^2 h^3),
    # with h^2 = x^2/A^4 + y^2/B^4 + z^2/C^4.  Coefficients from the workload
    # generator's Hessian (an independent route).
    rng = np.random.default_rng(8)
    ax = np.array([0.3, 0.5, 0.9])
    ell = synth.Ellipsoid(np.zeros(3), np.eye(3), ax)
    x = ell.sample(rng, 200)
    grad, hess = ell.grad_hess(x)
    n, a = synth.coeffs_from_implicit(grad, hess)
    tor = oracle.fit(x, n, a, kfloor=1e-12)
    A, B, C = ax
    h2 = x[:, 0] ** 2 / A ** 4 + x[:, 1] ** 2 / B ** 4 + x[:, 2] ** 2 / C ** 4
    K = 1.0 / ((A * B * C) ** 2 * h2 ** 2)
    H = (np.sum(x ** 2, axis=1) - A * A - B * B - C * C) / (2 * (A * B * C) ** 2 * h2 ** 1.5)
    assert np.allclose(tor.K, K, rtol=1e-9)
    # outward normal: convex surface has negative curvature in the paper's sign convention
    assert np.allclose(tor.H, H, rtol=1e-9)
    assert np.all(tor.sgn == 1.0)


def _torus_coeffs_closed_form(R0, r0, theta, psi, Rm, c0):
    """Point, outward normal and coefficients on a ring torus from its principal
    curvatures (tube -1/r0, ring -cos(theta)/(R0 + r0 cos(theta))) and directions."""
    ct, st, cp, sp = math.cos(theta), math.sin(theta), math.cos(psi), math.sin(psi)
    rr = R0 + r0 * ct
    y = np.array([rr * cp, rr * sp, r0 * st])
    nl = np.array([ct * cp, ct * sp, st])
    e_ring = np.array([-sp, cp, 0.0])
    e_tube = np.array([-st * cp, -st * sp, ct])
    k_tube = -1.0 / r0
    k_ring = -ct / rr
    p = Rm @ y + c0
    n = Rm @ nl
    e_ring = Rm @ e_ring
    e_tube = Rm @ e_tube
    s, t = synth.tangent_frame(n[None])
    s, t = s[0], t[0]
    II = lambda v, w: k_tube * (v @ e_tube) * (w @ e_tube) + k_ring * (v @ e_ring) * (w @ e_ring)  # noqa: E731
    a = np.array([0.0, 0.0, 0.0, II(s, t), 0.5 * II(t, t), 0.5 * II(s, s)])
    return p, n, a


def test_torus_round_trip_equators():
    Rm = _rot(11)
    c0 = np.array([0.3, -0.1, 0.2])
    R0, r0 = 3.0, 1.0
    for theta in (0.0, math.pi):
        for psi in np.linspace(0, 2 * math.pi, 7, endpoint=False):
            p, n, a = _torus_coeffs_closed_form(R0, r0, theta, psi, Rm, c0)
            tor = oracle.fit([p], [n], [a], kfloor=1e-12)
            assert np.allclose(tor.c[0], c0, atol=1e-10)
            assert abs(abs(tor.u[0] @ (Rm @ [0, 0, 1.0])) - 1) < 1e-10
            assert abs(tor.R[0] - R0) < 1e-10 and abs(tor.r[0] - r0) < 1e-12
            assert tor.sgn[0] == 1.0


def test_torus_fit_osculates_to_second_order():
    # At a general torus point the fitted torus is not the original one, but
    # it matches the surface to second order: the error of g against the true
    # torus SDF shrinks like |y|^3 for offsets y around the point.
    Rm = _rot(12)
    c0 = np.zeros(3)
    R0, r0 = 2.0, 0.7
    p, n, a = _torus_coeffs_closed_form(R0, r0, 0.9, 0.4, Rm, c0)
    tor = oracle.fit([p], [n], [a], kfloor=1e-12)
    rng = np.random.default_rng(13)
    dirs = rng.normal(size=(20, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)

    def true_sdf(x):
        y = (x - c0) @ Rm
        rho = np.linalg.norm(y[:, :2], axis=1)
        return np.sqrt((rho - R0) ** 2 + y[:, 2] ** 2) - r0

    errs = []
    for eps in (4e-2, 2e-2, 1e-2):
        x = p + eps * dirs
        errs.append(np.max(np.abs(oracle.torus_g(tor, x)[:, 0] - true_sdf(x))))
    assert errs[1] / errs[0] < 0.2 and errs[2] / errs[1] < 0.2   # ~1/8 per halving


# ---------------------------------------------------------------------------
# Invariances of the definition
# ---------------------------------------------------------------------------

def _mixed_cloud(N=1500, seed=21):
    cl, _ = synth.mid(N=N, grid=4)
    rng = np.random.default_rng(seed)
    a = cl.a.astype(np.float64)
    a[:, 0] += rng.normal(scale=0.01, size=N)      # shifts
    a[:, 1:3] += rng.normal(scale=0.05, size=(N, 2))  # tilted supporting planes
    return cl.p.astype(np.float64), cl.n.astype(np.float64), a


def test_orientation_flip_negates():
    # (n, a) -> (-n, a') describes the same surface with the opposite
    # orientation.  The input frame becomes (s, -t, -n), hence
    # a' = (-a00, a01, -a10, a11, -a02, -a20), and phi must change sign.
    p, n, a = _mixed_cloud()
    ap = a * np.array([-1, 1, -1, 1, -1, -1])
    x = np.random.default_rng(22).uniform(-1.2, 1.2, size=(200, 3))
    kf = oracle.kfloor_for(p)
    phi = oracle.sdf(p, n, a, x, kfloor=kf)
    phi2 = oracle.sdf(p, -n, ap, x, kfloor=kf)
    assert np.max(np.abs(phi + phi2)) < 1e-11


def test_scale_invariance():
    # Sec. 4.3 rescaling: p -> alpha p, a00 -> alpha a00, a11, a02, a20 -> a / alpha
    # (a01, a10 unchanged); lambda_x scales as 1/alpha, so phi(alpha x) = alpha phi(x).
    p, n, a = _mixed_cloud()
    alpha = 2.75
    sa = a * np.array([alpha, 1, 1, 1 / alpha, 1 / alpha, 1 / alpha])
    x = np.random.default_rng(23).uniform(-1.2, 1.2, size=(200, 3))
    phi = oracle.sdf(p, n, a, x)
    phi2 = oracle.sdf(alpha * p, n, sa, alpha * x)
    assert np.max(np.abs(phi2 - alpha * phi)) < 1e-11


def test_translation_and_permutation_invariance():
    p, n, a = _mixed_cloud()
    x = np.random.default_rng(24).uniform(-1.2, 1.2, size=(200, 3))
    phi = oracle.sdf(p, n, a, x)
    b = np.array([0.7, -1.9, 3.3])
    assert np.max(np.abs(oracle.sdf(p + b, n, a, x + b) - phi)) < 1e-11
    perm = np.random.default_rng(25).permutation(p.shape[0])
    assert np.max(np.abs(oracle.sdf(p[perm], n[perm], a[perm], x) - phi)) < 1e-12


def test_rotation_invariance_isotropic():
    p, n, a = _sphere(500, 1.0, seed=26)
    a[:, 4:6] *= (1.0 + 0.1 * np.random.default_rng(27).normal(size=(500, 1)))  # isotropic jitter
    a[:, 0] = 0.02
    Rm = _rot(28)
    x = np.random.default_rng(29).uniform(-1.5, 1.5, size=(100, 3))
    phi = oracle.sdf(p, n, a, x)
    phi2 = oracle.sdf(p @ Rm.T, n @ Rm.T, a, x @ Rm.T)
    assert np.max(np.abs(phi - phi2)) < 1e-11


def test_large_C_limit_is_nearest_torus():
    # Laplace's method (Sec. 2.3): as C grows the weights concentrate on the
    # nearest point and phi tends to that point's g.
    p, n, a = _mixed_cloud(N=120)
    rng = np.random.default_rng(30)
    pick = rng.choice(p.shape[0], size=150)
    x = p[pick] + 0.02 * rng.normal(size=(150, 3))
    tor = oracle.fit(p, n, a)
    g = oracle.torus_g(tor, x)
    d = np.linalg.norm(x[:, None, :] - p[None], axis=2)
    order = np.argsort(d, axis=1)
    gap = (d[np.arange(len(x)), order[:, 1]] - d[np.arange(len(x)), order[:, 0]]) / d.max(axis=1)
    ok = gap > 0.03                      # lambda * gap > 2 C * 0.03 = 36 at C = 600
    gnear = g[np.arange(len(x)), order[:, 0]]
    phi600 = oracle.eval_sdf(p, tor, x, C=600.0)
    assert ok.sum() > 20
    assert np.max(np.abs(phi600[ok] - gnear[ok])) < 1e-7
    phi64 = oracle.eval_sdf(p, tor, x, C=64.0)
    assert np.max(np.abs(phi64[ok] - gnear[ok])) > 1e-6   # finite C genuinely blends


def test_degenerate_queries():
    p, n, a = _sphere(50, 1.0, seed=31)
    tor = oracle.fit(p, n, a)
    x = np.array([[np.nan, 0.0, 0.0], [0.1, 0.2, 0.3]])
    phi = oracle.eval_sdf(p, tor, x)
    assert np.isnan(phi[0]) and np.isfinite(phi[1])
    # N = 1 and x = p: the max distance is 0 and the weights are uniform.
    t1 = oracle.fit(p[:1], n[:1], a[:1])
    assert abs(oracle.eval_sdf(p[:1], t1, p[:1])[0] - 0.0) < 1e-12


# ---------------------------------------------------------------------------
# Gradients vs. central finite differences
# ---------------------------------------------------------------------------

def test_grad_x_matches_finite_differences():
    p, n, a = _mixed_cloud(N=1000)
    tor = oracle.fit(p, n, a)
    x = np.random.default_rng(32).uniform(-1.0, 1.0, size=(60, 3))
    phi, g = oracle.eval_sdf(p, tor, x, grad=True)
    h = 1e-6
    fd = np.zeros_like(g)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd[:, k] = (oracle.eval_sdf(p, tor, x + e) - oracle.eval_sdf(p, tor, x - e)) / (2 * h)
    # skip queries whose farthest point is nearly tied (lambda_x kinks there)
    d = np.linalg.norm(x[:, None, :] - p[None], axis=2)
    ds = np.sort(d, axis=1)
    ok = (ds[:, -1] - ds[:, -2]) > 1e-4
    assert ok.sum() > 40
    assert np.max(np.abs(g[ok] - fd[ok])) < 2e-7


def test_grad_x_includes_lambda_term():
    # App. D holds lambda fixed; with lambda_x = 2C / max_i |x - p_i| the exact
    # derivative differs from it by (2C/M^2) e_{i*} sum_i (w_i/W)(g_i - phi) d_i.
    p, n, a = _mixed_cloud(N=600)
    tor = oracle.fit(p, n, a)
    x = np.random.default_rng(33).uniform(-1.0, 1.0, size=(20, 3))
    phi, g, st = oracle.eval_sdf(p, tor, x, grad=True, stats=True)
    h = 1e-6
    # frozen-lambda derivative by finite differences at the frozen lambda (C scaled)
    fz = np.zeros_like(g)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        for sgn in (+1, -1):
            xs = x + sgn * e
            dd = np.linalg.norm(xs[:, None, :] - p[None], axis=2)
            lam = 2 * 64.0 / st[:, 0]
            w = np.exp(-lam[:, None] * (dd - 0.5 * st[:, :1]))
            gg = oracle.torus_g(tor, xs)
            fz[:, k] += sgn * np.sum(w * gg, axis=1) / np.sum(w, axis=1) / (2 * h)
    assert np.max(np.abs(g - fz)) > 1e-6      # the lambda_x term is not negligible
    d = np.linalg.norm(x[:, None, :] - p[None], axis=2)
    istar = np.argmax(d, axis=1)
    e_star = (x - p[istar]) / d[np.arange(len(x)), istar][:, None]
    lam = 2 * 64.0 / st[:, 0]
    w = np.exp(-lam[:, None] * (d - 0.5 * st[:, :1]))
    W = w.sum(axis=1, keepdims=True)
    gg = oracle.torus_g(tor, x)
    extra = (2 * 64.0 / st[:, 0] ** 2)[:, None] * e_star * np.sum(w / W * (gg - phi[:, None]) * d, axis=1)[:, None]
    assert np.max(np.abs(g - (fz + extra))) < 1e-6


def test_grad_a_matches_finite_differences():
    p, n, a = _mixed_cloud(N=300)
    rng = np.random.default_rng(34)
    x = rng.uniform(-1.0, 1.0, size=(80, 3))
    gout = rng.normal(size=80)
    kf = oracle.kfloor_for(p)
    ga = oracle.grad_a(p, n, a, x, gout, kfloor=kf)
    h = 1e-6
    idx = rng.choice(p.shape[0], size=12, replace=False)
    for i in idx:
        for j in range(6):
            ap = a.copy()
            am = a.copy()
            ap[i, j] += h
            am[i, j] -= h
            Lp = gout @ oracle.sdf(p, n, ap, x, kfloor=kf)
            Lm = gout @ oracle.sdf(p, n, am, x, kfloor=kf)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - ga[i, j]) < 1e-6 * max(1.0, abs(fd)), (i, j, fd, ga[i, j])


def test_grad_points_matches_finite_differences():
    # dL/dp and dL/dn move the torus, the weight and, for a query's farthest
    # point, lambda_x; central differences of the oracle's phi pin all three
    p, n, a = _mixed_cloud(N=300)
    rng = np.random.default_rng(36)
    x = rng.uniform(-1.0, 1.0, size=(80, 3))
    gout = rng.normal(size=80)
    kf = oracle.kfloor_for(p)
    ga, gp, gn = oracle.grad_points(p, n, a, x, gout, kfloor=kf)
    assert np.allclose(ga, oracle.grad_a(p, n, a, x, gout, kfloor=kf), rtol=1e-10, atol=1e-12)
    far = np.argmax(np.linalg.norm(x[:, None, :] - p[None], axis=2), axis=1)
    idx = list(rng.choice(p.shape[0], size=10, replace=False)) + list(np.unique(far)[:4])
    h = 1e-6
    for i in idx:
        for arr, g in ((p, gp), (n, gn)):
            for k in range(3):
                ap, am = arr.copy(), arr.copy()
                ap[i, k] += h
                am[i, k] -= h
                if arr is p:
                    Lp = gout @ oracle.sdf(ap, n, a, x, kfloor=kf)
                    Lm = gout @ oracle.sdf(am, n, a, x, kfloor=kf)
                else:
                    Lp = gout @ oracle.sdf(p, ap, a, x, kfloor=kf)
                    Lm = gout @ oracle.sdf(p, am, a, x, kfloor=kf)
                fd = (Lp - Lm) / (2 * h)
                assert abs(fd - g[i, k]) < 2e-6 * max(1.0, abs(fd)), (i, k, arr is p, fd, g[i, k])


def test_laplacian_sphere_closed_form():
    # every torus of the exact unit sphere is the sphere itself, so phi = |x| - 1
    # and its Laplacian is 2 / |x| wherever the weights move
    p, n, a = _sphere(400, 1.0, seed=37)
    tor = oracle.fit(p, n, a)
    rng = np.random.default_rng(38)
    x = rng.uniform(-2.5, 2.5, size=(40, 3))
    x = x[np.linalg.norm(x, axis=1) > 0.05]
    lap = oracle.laplacian(p, tor, x)
    assert np.allclose(lap, 2.0 / np.linalg.norm(x, axis=1), rtol=1e-9, atol=1e-9)


def test_laplacian_matches_second_differences():
    # the sum of the three second central differences of the oracle's phi
    # (Richardson-extrapolated over h and h/2 to cancel the h^2 error)
    p, n, a = _mixed_cloud(N=300)
    tor = oracle.fit(p, n, a)
    rng = np.random.default_rng(39)
    x = rng.uniform(-1.0, 1.0, size=(24, 3))
    lap = oracle.laplacian(p, tor, x)
    phi0 = oracle.eval_sdf(p, tor, x)

    def second_diff(h):
        out = np.zeros(len(x))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            out += (oracle.eval_sdf(p, tor, x + e) - 2 * phi0 + oracle.eval_sdf(p, tor, x - e)) / (h * h)
        return out

    fd = (4 * second_diff(5e-4) - second_diff(1e-3)) / 3
    assert np.abs(fd).max() > 5.0
    assert np.allclose(lap, fd, rtol=1e-5, atol=1e-5 * np.abs(fd).max())


# ---------------------------------------------------------------------------
# Baselines: smoothed signed planar distance and signed Hopf-Cole distance
# ---------------------------------------------------------------------------

def _plane_cloud(N, seed):
    rng = np.random.default_rng(seed)
    p = np.zeros((N, 3))
    p[:, :2] = rng.uniform(-1, 1, size=(N, 2))
    n = np.zeros((N, 3))
    n[:, 2] = rng.uniform(0.5, 2.0, size=N)      # not unit: the planar distance uses n / |n|
    return p, n


def test_sspd_plane_closed_form():
    # every point's planar distance is x_z, and the weights sum to one
    p, n = _plane_cloud(300, 40)
    x = np.random.default_rng(41).uniform(-1.5, 1.5, size=(200, 3))
    assert np.allclose(oracle.eval_baseline(p, n, x, "sspd"), x[:, 2], rtol=1e-12, atol=1e-12)
    assert np.allclose(oracle.eval_baseline(p, -n, x, "sspd"), -x[:, 2], rtol=1e-12, atol=1e-12)


def test_sspd_area_weights_and_single_point():
    p, n, _ = _mixed_cloud(N=200)
    x = np.random.default_rng(42).uniform(-1, 1, size=(50, 3))
    phi = oracle.eval_baseline(p, n, x, "sspd")
    # a common factor on the areas cancels
    assert np.allclose(oracle.eval_baseline(p, n, x, "sspd", area=np.full(200, 7.5)), phi, rtol=1e-12, atol=1e-14)
    # all weight on one point gives that point's planar distance
    A = np.zeros(200)
    A[17] = 1.0
    nh = n[17] / np.linalg.norm(n[17])
    assert np.allclose(oracle.eval_baseline(p, n, x, "sspd", area=A), (x - p[17]) @ nh, rtol=1e-12, atol=1e-12)


def test_shc_satisfies_screened_laplace():
    # with lambda fixed, the double-layer sum is a sum of screened (Yukawa)
    # dipoles, so Lap w = lambda^2 w away from the points (Eq. ScreenedLaplace)
    rng = np.random.default_rng(43)
    p = rng.uniform(-0.5, 0.5, size=(40, 3))
    n = rng.normal(size=(40, 3))
    lam = 3.0
    x = rng.uniform(-2, 2, size=(400, 3))
    x = x[np.linalg.norm(x[:, None, :] - p[None], axis=2).min(axis=1) > 0.5][:30]
    _, w0, _ = oracle.eval_baseline(p, n, x, "shc", lam_fixed=lam, raw=True)

    def second_diff(h):
        out = np.zeros(len(x))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            _, wp, _ = oracle.eval_baseline(p, n, x + e, "shc", lam_fixed=lam, raw=True)
            _, wm, _ = oracle.eval_baseline(p, n, x - e, "shc", lam_fixed=lam, raw=True)
            out += (wp - 2 * w0 + wm) / (h * h)
        return out

    lap = (4 * second_diff(1e-4) - second_diff(2e-4)) / 3
    scale = np.abs(lam * lam * w0).max()
    assert np.abs(lap - lam * lam * w0).max() <= 1e-7 * scale
    # phi is -(1/lambda) log|w| with the sign of w (sigma = 0 at fixed lambda)
    phi = oracle.eval_baseline(p, n, x, "shc", lam_fixed=lam)
    assert np.allclose(phi, np.sign(w0) * (-np.log(np.abs(w0)) / lam), rtol=1e-12, atol=1e-12)


def test_shc_orientation_areas_and_sign():
    p, n, _ = _mixed_cloud(N=200)
    x = np.random.default_rng(44).uniform(-1, 1, size=(60, 3))
    phi, w, _ = oracle.eval_baseline(p, n, x, "shc", raw=True)
    assert np.allclose(oracle.eval_baseline(p, -n, x, "shc"), -phi, rtol=1e-12, atol=1e-12)
    # scaling every area by k multiplies w by k: phi moves by -sign(w) log(k) / lambda_x
    M = np.linalg.norm(x[:, None, :] - p[None], axis=2).max(axis=1)
    lam = 2 * 64.0 / M
    k = 3.0
    assert np.allclose(oracle.eval_baseline(p, n, x, "shc", area=np.full(200, k)),
                       phi - np.sign(w) * np.log(k) / lam, rtol=1e-12, atol=1e-12)
    # one point: outside along its normal the distance is positive, inside negative
    q = np.array([[0.0, 0.0, 0.3], [0.0, 0.0, -0.3]])
    one = oracle.eval_baseline([[0.0, 0.0, 0.0]], [[0.0, 0.0, 2.0]], q, "shc")
    assert one[0] > 0 and one[1] < 0


def test_baselines_nearest_point_limit():
    # as C grows the weights concentrate on the nearest point: SSPD tends to its
    # planar distance and |SHC| to the distance itself, with error O(1/C)
    p, n, _ = _mixed_cloud(N=150)
    rng = np.random.default_rng(45)
    x = rng.uniform(-1, 1, size=(40, 3))
    d = np.linalg.norm(x[:, None, :] - p[None], axis=2)
    srt = np.sort(d, axis=1)
    x = x[srt[:, 1] - srt[:, 0] > 0.05 * srt[:, -1]]
    d = np.linalg.norm(x[:, None, :] - p[None], axis=2)
    nn = np.argmin(d, axis=1)
    nh = n[nn] / np.linalg.norm(n[nn], axis=1, keepdims=True)
    planar = np.sum((x - p[nn]) * nh, axis=1)
    errs_s, errs_h = [], []
    for C in (50.0, 200.0, 600.0):
        errs_s.append(np.abs(oracle.eval_baseline(p, n, x, "sspd", C=C) - planar).max())
        errs_h.append(np.abs(np.abs(oracle.eval_baseline(p, n, x, "shc", C=C)) - d.min(axis=1)).max())
    assert errs_s[2] < 1e-6 and errs_s[0] > errs_s[1] > errs_s[2]
    assert errs_h[2] < errs_h[0] / 4 and errs_h[2] < 0.02


def test_baselines_rigid_invariance():
    p, n, _ = _mixed_cloud(N=120)
    x = np.random.default_rng(46).uniform(-1, 1, size=(40, 3))
    R = _rot(47)
    t = np.array([0.3, -1.2, 2.0])
    for kind in ("sspd", "shc"):
        a = oracle.eval_baseline(p, n, x, kind)
        b = oracle.eval_baseline(p @ R.T + t, n @ R.T, x @ R.T + t, kind)
        assert np.allclose(a, b, rtol=1e-9, atol=1e-10), kind


# ---------------------------------------------------------------------------
# Sphere tracing on the exact sphere
# ---------------------------------------------------------------------------

def test_trace_sphere_closed_form():
    p, n, a = _sphere(300, 1.0, seed=35)
    tor = oracle.fit(p, n, a)
    org, dirs = synth.camera_rays(8, radius=3.0, fov_deg=30.0)
    o = org.astype(np.float64)
    d = dirs.astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t, hit, ns, nrm = oracle.trace(p, tor, o, d, steps=64, eps=1e-9, tmax=8.0)
    b = np.sum(o * d, axis=1)
    disc = b * b - (np.sum(o * o, axis=1) - 1.0)
    expect_hit = disc > 0
    assert np.array_equal(hit, expect_hit)
    tstar = -b - np.sqrt(np.where(expect_hit, disc, 0.0))
    assert np.max(np.abs(t[hit] - tstar[hit])) < 1e-8
    xh = o + t[:, None] * d
    assert np.max(np.abs(nrm[hit] - xh[hit] / np.linalg.norm(xh[hit], axis=1, keepdims=True))) < 1e-7


# ---------------------------------------------------------------------------
# Radius-limited evaluation (Sec. 4.2, "Acceleration and adaptive lambda")
# ---------------------------------------------------------------------------

def test_knn_mean_matches_brute_force():
    rng = np.random.default_rng(3)
    for N in (2, 5, 80, 300):
        p = rng.normal(size=(N, 3))
        dm = np.linalg.norm(p[:, None, :] - p[None, :, :], axis=2)
        np.fill_diagonal(dm, np.inf)
        k = min(64, N - 1)
        want = np.sort(dm, axis=1)[:, :k].mean(axis=1).mean()
        assert abs(oracle.knn_mean(p) - want) <= 1e-12 * want
    assert oracle.knn_mean(np.zeros((1, 3))) == 1.0
    # two points: each one's only neighbour is the other
    assert abs(oracle.knn_mean(np.array([[0.0, 0.0, 0.0], [0.0, 3.0, 4.0]])) - 5.0) < 1e-15
    D, lam, reval = oracle.radius_params(np.array([[0.0, 0.0, 0.0], [0.0, 3.0, 4.0]]))
    assert abs(lam - 200.0) < 1e-12 and abs(reval - 2 * 64.0 / 200.0) < 1e-15


@pytest.mark.parametrize("shift", [0.0, 0.2])
def test_radius_eval_sphere_closed_form(shift):
    # every torus of a sphere cloud is the sphere itself, so any blend of them --
    # within R_eval or over the 32 nearest -- is |x| - (1 + shift)
    p, n, a = _sphere(3000, seed=4, shift=shift)
    tor = oracle.fit(p, n, a)
    D, lam, reval = oracle.radius_params(p)
    rng = np.random.default_rng(9)
    near = p[:40] * (1.0 + 0.3 * reval * rng.uniform(-1, 1, size=(40, 1)))
    u = rng.normal(size=(60, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    far = u * rng.choice([0.3, 1.6, 2.5], size=(60, 1))
    x = np.vstack([near, far])
    phi, cnt = oracle.eval_radius(p, tor, x, lam, reval)
    assert np.all(cnt[:40] > 0) and np.all(cnt[40:] == -32)
    assert np.abs(phi - (np.linalg.norm(x, axis=1) - 1.0 - shift)).max() < 1e-12


def test_radius_eval_single_point_counts_and_limits():
    rng = np.random.default_rng(6)
    p, n, a = _sphere(50, seed=6)
    a[:, 5] = -0.5 * (1.0 + 0.5 * rng.random(50))     # anisotropic, point-specific tori
    a[:, 3] = 0.2 * rng.normal(size=50)
    tor = oracle.fit(p, n, a)
    # a query within R_eval of exactly one point blends that point's torus alone
    # (R_eval below a third of the smallest spacing, lambda = 2C / R_eval)
    dm = np.linalg.norm(p[:, None, :] - p[None, :, :], axis=2)
    np.fill_diagonal(dm, np.inf)
    reval = 0.3 * dm.min()
    lam = 2 * 64.0 / reval
    v = rng.normal(size=(10, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    x = p[:10] + 0.5 * reval * v
    phi, cnt = oracle.eval_radius(p, tor, x, lam, reval)
    g = oracle.torus_g(tor, x)
    assert np.all(cnt == 1)
    assert np.allclose(phi, g[np.arange(10), np.arange(10)], rtol=1e-14, atol=1e-15)
    # far queries fall back to the 32 nearest (all points if fewer)
    far = 10.0 * v
    _, cnt = oracle.eval_radius(p, tor, far, lam, reval)
    assert np.all(cnt == -32)
    _, cnt = oracle.eval_radius(p[:10], oracle.fit(p[:10], n[:10], a[:10]), far, lam, reval)
    assert np.all(cnt == -10)
    # a very large lambda leaves the nearest point's torus (Laplace limit)
    xq = 1.5 * v
    phi, cnt = oracle.eval_radius(p, tor, xq, 1e9, 1e-12)
    gq = oracle.torus_g(tor, xq)
    nearest = np.argmin(np.linalg.norm(xq[:, None, :] - p[None], axis=2), axis=1)
    assert np.all(cnt == -32)
    assert np.allclose(phi, gq[np.arange(10), nearest], rtol=1e-12, atol=1e-14)
    # a NaN query gives NaN and blends nothing
    phi, cnt = oracle.eval_radius(p, tor, np.array([[np.nan, 0.0, 0.0]]), lam, reval)
    assert np.isnan(phi[0]) and cnt[0] == 0
