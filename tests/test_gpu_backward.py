"""Parity of the parameter backward (dL/da, dL/dp, dL/dn) and of the autograd
module with the oracle.

Tolerance: |dL/dtheta_gpu - dL/dtheta_oracle| <= 1e-4 * max|dL/dtheta_oracle|
per output (FP32 sweeps, FP64 chain rule).  The oracle differentiates its own
torus fit, weights and lambda_x with dual numbers; it is pinned by finite
differences in the CPU tests.

dL/dp moves with the farthest point of each query, which FP32 cannot tell
apart from the runner-up when their distances agree to within its rounding;
at such a tie phi is not differentiable in p.  Those queries (top two
distances within 1e-5 relative) get a zero upstream gradient on both sides.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_16946_amd import autograd, binding, synth

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def _tilted(cl, seed):
    """Add shifts and tilted supporting planes so that every coefficient matters."""
    rng = np.random.default_rng(seed)
    a = cl.a.astype(np.float64).copy()
    a[:, 0] += rng.normal(scale=0.01, size=cl.N)
    a[:, 1:3] += rng.normal(scale=0.05, size=(cl.N, 2))
    return synth.Cloud(cl.p, cl.n, a.astype(np.float32), cl.meta)


def _far_decided(p, x):
    """Queries whose farthest point is separated from the runner-up by more than FP32 rounding."""
    d = np.linalg.norm(x.astype(np.float64)[:, None, :] - p.astype(np.float64)[None], axis=2)
    top = np.sort(d, axis=1)[:, -2:]
    return top[:, 1] - top[:, 0] > 1e-5 * top[:, 1]


def _case(name):
    if name == "tiny":
        return synth.tiny(Q=1500, N=1200)
    if name == "mid":
        cl, x = synth.mid(N=1500, grid=11)
        return _tilted(cl, 1), x
    if name == "cap":  # every torus radius L is 20 to 30 bbox diagonals: all anchored
        cl, x = synth.cap_cloud()
        return _tilted(cl, 12), x
    cl, q, mask = synth.diff_workload(N=2048, Q=3000)
    return cl, q


@pytest.mark.parametrize("name", ["tiny", "mid", "diff", "cap"])
def test_backward_params_vs_oracle(name):
    cl, x = _case(name)
    gout = np.random.default_rng(2).normal(size=x.shape[0]).astype(np.float32)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x)
    sdf, st = c(xs, stats=True)
    ga = binding.backward_params(c.rec, c.p, c.n, c.a, xs, st, _dev(gout), c.params).cpu().numpy().astype(np.float64)
    ref = oracle.grad_a(cl.p, cl.n, cl.a, x, gout)
    scale = np.abs(ref).max()
    err = np.abs(ga - ref).max()
    print(f"{name}: dL/da max err {err:.3e}, scale {scale:.3e}", flush=True)
    assert err <= 1e-4 * scale


@pytest.mark.parametrize("name", ["tiny", "mid", "diff", "cap"])
def test_backward_points_vs_oracle(name):
    cl, x = _case(name)
    if name not in ("mid", "cap"):
        cl = _tilted(cl, 3)
    gout = np.random.default_rng(4).normal(size=x.shape[0]).astype(np.float32)
    gout[~_far_decided(cl.p, x)] = 0.0
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x)
    _, st = c(xs, stats=True)
    go = _dev(gout)
    ga, gp, gn = binding.backward_points(c.rec, c.p, c.n, c.a, xs, st, go, c.params)
    refs = oracle.grad_points(cl.p, cl.n, cl.a, x, gout)
    for what, g, ref in zip("apn", (ga, gp, gn), refs):
        g = g.cpu().numpy().astype(np.float64)
        scale = np.abs(ref).max()
        err = np.abs(g - ref).max()
        print(f"{name}: dL/d{what} max err {err:.3e}, scale {scale:.3e}", flush=True)
        assert err <= 1e-4 * scale, what
    # the coefficient part is the coefficient-only entry point's, bit for bit
    assert torch.equal(ga, binding.backward_params(c.rec, c.p, c.n, c.a, xs, st, go, c.params))
    # each output alone equals the same output of the combined call
    assert torch.equal(binding.backward_points(c.rec, c.p, c.n, c.a, xs, st, go, c.params, want="p")[1], gp)
    assert torch.equal(binding.backward_points(c.rec, c.p, c.n, c.a, xs, st, go, c.params, want="n")[2], gn)


def _farthest_term(cl, x, gout, C=64.0):
    """The farthest-point part of dL/dp alone, in FP64 from the tori: per query
    -gout (2C/M^2) V e_* on its farthest point, V = <(g - phi) d>."""
    tor = oracle.fit(cl.p, cl.n, cl.a)
    p = cl.p.astype(np.float64)
    xd = x.astype(np.float64)
    g = oracle.torus_g(tor, xd)                                  # [Q, N]
    d = np.linalg.norm(xd[:, None, :] - p[None], axis=2)
    far = np.argmax(d, axis=1)
    M = d[np.arange(len(x)), far]
    w = np.exp(-(2 * C / M)[:, None] * (d - 0.5 * M[:, None]))
    W = w.sum(axis=1)
    phi = (w * g).sum(axis=1) / W
    V = (w * (g - phi[:, None]) * d).sum(axis=1) / W
    es = (xd - p[far]) / M[:, None]
    out = np.zeros_like(p)
    np.add.at(out, far, -(gout * 2 * C / M ** 2 * V)[:, None] * es)
    return out, np.unique(far)


def test_backward_points_farthest_point_term():
    # queries on one side of an elongated cloud share a few farthest points;
    # the GPU must carry their term: its error there is far below the term
    cl, _ = synth.tiny(Q=10, N=900)
    p = cl.p.astype(np.float64) * np.array([3.0, 1.0, 1.0])
    cl = synth.Cloud(p.astype(np.float32), cl.n, cl.a, cl.meta)
    rng = np.random.default_rng(9)
    x = (rng.normal(size=(2000, 3)) * 0.2 + np.array([-2.0, 0.0, 0.0])).astype(np.float32)
    x = x[_far_decided(cl.p, x)]
    gout = np.ones(x.shape[0], np.float32)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x)
    _, st = c(xs, stats=True)
    _, gp, _ = binding.backward_points(c.rec, c.p, c.n, c.a, xs, st, None, c.params, want="p")
    _, gp_ref, _ = oracle.grad_points(cl.p, cl.n, cl.a, x, gout)
    term, far = _farthest_term(cl, x, gout)
    gp = gp.cpu().numpy().astype(np.float64)
    err_far = np.abs(gp[far] - gp_ref[far]).max()
    print(f"{len(far)} farthest points; their term up to {np.abs(term[far]).max():.3e}, "
          f"GPU error there {err_far:.3e}; |dL/dp| overall up to {np.abs(gp_ref).max():.3e}", flush=True)
    assert np.abs(gp - gp_ref).max() <= 1e-4 * np.abs(gp_ref).max()
    assert err_far <= 1e-2 * np.abs(term[far]).max()


def test_backward_points_no_queries_and_determinism():
    cl, x = synth.tiny(Q=700, N=500)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x)
    _, st = c(xs, stats=True)
    r1 = binding.backward_points(c.rec, c.p, c.n, c.a, xs, st, None, c.params)
    r2 = binding.backward_points(c.rec, c.p, c.n, c.a, xs, st, None, c.params)
    assert all(torch.equal(u, v) for u, v in zip(r1, r2))
    z = binding.backward_points(c.rec, c.p, c.n, c.a, xs[:0], st[:0], None, c.params)
    assert all(torch.count_nonzero(t) == 0 for t in z)


def test_backward_params_no_queries_and_determinism():
    cl, x = synth.tiny(Q=500, N=700)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x)
    _, st = c(xs, stats=True)
    g1 = binding.backward_params(c.rec, c.p, c.n, c.a, xs, st, None, c.params)
    g2 = binding.backward_params(c.rec, c.p, c.n, c.a, xs, st, None, c.params)
    assert torch.equal(g1, g2)
    z = binding.backward_params(c.rec, c.p, c.n, c.a, xs[:0], st[:0], None, c.params)
    assert torch.count_nonzero(z) == 0


def test_autograd_module_matches_oracle():
    # L = sum phi^2 over near-surface queries of the differentiation workload
    cl, q, mask = synth.diff_workload(N=1500, Q=2000)
    x = q[mask]
    m = autograd.TorusSDF(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x).requires_grad_(True)
    phi = m(xs)
    loss = (phi * phi).sum()
    loss.backward()
    phi_np = phi.detach().cpu().numpy().astype(np.float64)
    ref_phi, ref_g = oracle.sdf(cl.p, cl.n, cl.a, x, grad=True)
    gx_ref = 2.0 * ref_phi[:, None] * ref_g
    assert np.abs(xs.grad.cpu().numpy() - gx_ref).max() <= 1e-4
    ga_ref = oracle.grad_a(cl.p, cl.n, cl.a, x, 2.0 * ref_phi)
    ga = m.a.grad.cpu().numpy().astype(np.float64)
    assert np.abs(ga - ga_ref).max() <= 1e-4 * np.abs(ga_ref).max()
    # an optimiser step refits the tori on the next forward
    with torch.no_grad():
        m.a -= 1e-3 * m.a.grad
    phi2 = m(xs.detach())
    a2 = m.a.detach().cpu().numpy()
    ref2 = oracle.sdf(cl.p, cl.n, a2, x)
    assert np.abs(phi2.detach().cpu().numpy() - ref2).max() <= 1e-5 * oracle.bbox_diag(cl.p)


def test_autograd_points_and_normals_match_oracle():
    cl, q, mask = synth.diff_workload(N=1200, Q=1500)
    x = q[mask]
    x = x[_far_decided(cl.p, x)]
    m = autograd.TorusSDF(_dev(cl.p), _dev(cl.n), _dev(cl.a), learn_points=True, learn_normals=True)
    phi = m(_dev(x))
    (phi * phi).sum().backward()
    ref_phi = oracle.sdf(cl.p, cl.n, cl.a, x)
    refs = oracle.grad_points(cl.p, cl.n, cl.a, x, 2.0 * ref_phi)
    for what, g, ref in zip("apn", (m.a.grad, m.p.grad, m.n.grad), refs):
        err = np.abs(g.cpu().numpy().astype(np.float64) - ref).max()
        assert err <= 1e-4 * np.abs(ref).max(), what
    # moving the points refits the tori
    with torch.no_grad():
        m.p -= 1e-3 * m.p.grad
    phi2 = m(_dev(x))
    ref2 = oracle.sdf(m.p.detach().cpu().numpy(), cl.n, cl.a, x)
    assert np.abs(phi2.detach().cpu().numpy() - ref2).max() <= 1e-5 * oracle.bbox_diag(cl.p)
