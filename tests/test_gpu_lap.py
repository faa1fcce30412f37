"""Parity of the Laplacian, gradient and eikonal residual sweep with the oracle.

The oracle's Laplacian is the exact second derivative of its own phi
(hyper-dual numbers, lambda_x moving with x); it is pinned in the CPU tests by
the unit sphere's closed form 2/|x| and by second differences.

Tolerances, from the arithmetic.  Laplacian, per query:
    |err| <= 2e-4 max(1, |Lap phi|) + 4e-7 lambda / d_min.
The first term covers FP32 rounding of the per-pair terms (each O(2 lambda)
before they cancel; the sums themselves are carried in FP64).  The second is
the input precision: phi has a cusp at every point (the weight's |x - p|), so
the term -2 lambda <(g - phi)/d> turns the FP32 error of one torus value
(about 2e-7 here) into 2 lambda 2e-7 / d for a query at distance d from its
nearest point.  Gradient and eikonal residual |err| <= 1e-4 (both O(1)).  As
for the gradient, queries whose two farthest points are within FP32 rounding
of each other are left out: there lambda_x has a kink and e_* may be either
point.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_16946_amd import binding, synth

pytestmark = pytest.mark.gpu

LREL = 2e-4
LCUSP = 4e-7
GTOL = 1e-4


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def _far_decided(p, x):
    d = np.linalg.norm(x.astype(np.float64)[:, None, :] - p.astype(np.float64)[None], axis=2)
    top = np.sort(d, axis=1)[:, -2:]
    return top[:, 1] - top[:, 0] > 1e-5 * top[:, 1]


def _lap_tol(p, x, lref, C=64.0):
    d = np.linalg.norm(x.astype(np.float64)[:, None, :] - p.astype(np.float64)[None], axis=2)
    lam = 2.0 * C / d.max(axis=1)
    return LREL * np.maximum(1.0, np.abs(lref)) + LCUSP * lam / np.maximum(d.min(axis=1), 1e-12)


def _run(cl, x):
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x)
    _, g_eval, st = c(xs, grad=True, stats=True)
    lap, g, eik = binding.laplacian(c.rec, c.N, xs, st, c.params)
    return c, xs, st, g_eval, lap.cpu().numpy(), g.cpu().numpy(), eik.cpu().numpy()


@pytest.mark.parametrize("name", ["tiny", "mid", "diff", "cap"])
def test_laplacian_vs_oracle(name):
    if name == "tiny":
        cl, x = synth.tiny(Q=1200, N=900)
    elif name == "mid":
        cl, x = synth.mid(N=1500, grid=10)
    elif name == "cap":  # nearly flat: every point takes the anchored torus form
        cl, x = synth.cap_cloud(N=1200, Q=1500)
    else:
        cl, x, _ = synth.diff_workload(N=2048, Q=2000)
    x = x[_far_decided(cl.p, x)]
    c, xs, st, g_eval, lap, g, eik = _run(cl, x)
    tor = oracle.fit(cl.p, cl.n, cl.a)
    lref = oracle.laplacian(cl.p, tor, x)
    _, gref = oracle.eval_sdf(cl.p, tor, x, grad=True)
    rel = np.abs(lap - lref) / np.maximum(1.0, np.abs(lref))
    tol = _lap_tol(cl.p, x, lref)
    gerr = np.abs(g - gref).max()
    eerr = np.abs(eik - (np.linalg.norm(gref, axis=1) - 1.0)).max()
    w = int(np.argmax(rel))
    dq = np.linalg.norm(x[w].astype(np.float64) - cl.p.astype(np.float64), axis=1)
    print(f"{name}: {len(x)} queries, |Lap| up to {np.abs(lref).max():.3e}; Laplacian max rel err "
          f"{rel.max():.3e} (99th pct {np.quantile(rel, 0.99):.3e}; worst query: Lap {lref[w]:.4g}, nearest point "
          f"{dq.min():.3e}, lambda {128.0 / dq.max():.4g}); grad err {gerr:.3e}; eikonal err {eerr:.3e}; "
          f"largest err / tol {(np.abs(lap - lref) / tol).max():.3f}", flush=True)
    assert np.all(np.abs(lap - lref) <= tol)
    assert gerr <= GTOL and eerr <= GTOL
    # the gradient of this sweep and of pts_eval agree (two summation orders of the same sums)
    assert (g_eval.cpu().numpy() - g).__abs__().max() <= GTOL
    # outputs alone equal the same outputs of the combined call
    lap1, _, _ = binding.laplacian(c.rec, c.N, xs, st, c.params, want="l")
    _, _, eik1 = binding.laplacian(c.rec, c.N, xs, st, c.params, want="e")
    assert np.array_equal(lap1.cpu().numpy(), lap) and np.array_equal(eik1.cpu().numpy(), eik)


def test_laplacian_sphere_closed_form():
    # every torus of the exact unit sphere is the sphere: phi = |x| - 1,
    # Lap phi = 2/|x| and |grad phi| = 1
    cl = synth.sphere_cloud(3000, seed=14, jitter=0.0)
    rng = np.random.default_rng(15)
    u = rng.normal(size=(2000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    x = (u * rng.uniform(0.3, 2.5, size=(2000, 1))).astype(np.float32)
    x = x[_far_decided(cl.p, x)]
    _, _, _, _, lap, g, eik = _run(cl, x)
    ref = 2.0 / np.linalg.norm(x.astype(np.float64), axis=1)
    rel = np.abs(lap - ref) / np.maximum(1.0, ref)
    print(f"sphere: Laplacian max rel err {rel.max():.3e}; eikonal residual max {np.abs(eik).max():.3e}", flush=True)
    assert np.all(np.abs(lap - ref) <= _lap_tol(cl.p, x, ref))
    assert np.abs(eik).max() <= GTOL


def test_laplacian_edge_cases():
    cl, x = synth.tiny(Q=300, N=257)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x)
    _, st = c(xs, stats=True)
    # no queries: a no-op
    out = binding.laplacian(c.rec, c.N, xs[:0], st[:0], c.params)
    assert all(t.numel() == 0 for t in out if t is not None)
    # deterministic
    a = binding.laplacian(c.rec, c.N, xs, st, c.params)
    b = binding.laplacian(c.rec, c.N, xs, st, c.params)
    assert all(torch.equal(u, v) for u, v in zip(a, b))
    # a single point: phi = g, the torus's own Laplacian and a unit gradient
    one = synth.Cloud(cl.p[:1].copy(), cl.n[:1].copy(), cl.a[:1].copy(), {})
    lap, _, eik = _run(one, x[:50])[4:]
    lref = oracle.laplacian(one.p, oracle.fit(one.p, one.n, one.a), x[:50])
    assert np.all(np.abs(lap - lref) <= _lap_tol(one.p, x[:50], lref))
    assert np.abs(eik).max() <= GTOL
