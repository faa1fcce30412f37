"""Sphere tracing with every step's phi from the error-bounded evaluation
(pts_trace_bounded) against the exact device trace, the closed form of an
exact sphere and the oracle's tracer.

Each step's phi is within eval_eps of the exact one, so with eval_eps far
below the hit threshold the two marches take the same steps up to t
differences of order steps x eval_eps; rays whose final |phi| sits at the
threshold may stop one step apart, so hits are compared on all but a small
fraction of rays and t and normals on rays that hit in both.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_16946_amd import binding, synth

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def _rays(res, radius=3.0, fov=40.0, seed=0, target=(0.0, 0.0, 0.0)):
    org, d = synth.camera_rays(res, radius=radius, fov_deg=fov, seed=seed, target=target)
    d = d.astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return org, d.astype(np.float32)


def _both(c, org, d, steps, eps, tmax, eval_eps):
    ex = binding.trace(c.rec, c.N, _dev(org), _dev(d), steps=steps, eps=eps, tmax=tmax)
    bd = binding.trace(c.rec, c.N, _dev(org), _dev(d), steps=steps, eps=eps, tmax=tmax, eval_eps=eval_eps)
    return [[v.cpu().numpy() for v in r] for r in (ex, bd)]


def _compare(ex, bd, steps, eval_eps, D, what):
    (te, he, nse, ne), (tb, hb, nsb, nb) = ex, bd
    agree = he == hb
    both = he & hb
    dt = np.abs(tb[both] - te[both]).max() if both.any() else 0.0
    print(f"{what}: {he.sum()} exact hits, {hb.sum()} bounded hits, {(~agree).sum()} disagree, "
          f"max |dt| {dt:.3e} ({dt / D:.2e} D), steps equal {np.mean(nse[both] == nsb[both]):.4f}", flush=True)
    assert (~agree).sum() <= max(2, 0.01 * len(he))
    # the march's error: eval_eps per step, not amplified (|dphi/dt| <= 1 along a ray)
    assert dt <= 2.0 * steps * eval_eps + 2e-5 * D
    assert np.abs(nb[both] - ne[both]).max() < 1e-3
    assert np.all(nb[~hb] == 0)
    return both


def test_bounded_trace_sphere_closed_form():
    cl = synth.sphere_cloud(2000, seed=9, jitter=0.0)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    org, d = _rays(32)
    t, hit, ns, nrm = binding.trace(c.rec, c.N, _dev(org), _dev(d), steps=64, eps=1e-5, tmax=8.0, eval_eps=1e-7)
    t, hit, nrm = t.cpu().numpy(), hit.cpu().numpy(), nrm.cpu().numpy()
    o, dd = org.astype(np.float64), d.astype(np.float64)
    b = np.sum(o * dd, axis=1)
    disc = b * b - (np.sum(o * o, axis=1) - 1.0)
    expect = disc > 0.05
    assert np.array_equal(hit[expect], np.ones(expect.sum(), bool))
    tstar = -b - np.sqrt(np.where(disc > 0, disc, 0))
    assert np.abs(t[expect] - tstar[expect]).max() < 1e-4
    xh = o + t[:, None] * dd
    nref = xh / np.linalg.norm(xh, axis=1, keepdims=True)
    assert np.abs(nrm[expect] - nref[expect]).max() < 1e-3
    assert not hit[disc < -1e-2].any()


@pytest.mark.parametrize("eval_eps_rel", [0.0, 1e-6])
def test_bounded_trace_small_cloud_vs_exact_and_oracle(eval_eps_rel):
    cl, _ = synth.mid(N=3000, grid=4)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    org, d = _rays(24, radius=2.5, seed=3)
    D = oracle.bbox_diag(cl.p)
    eps, tmax, steps = 1e-4 * D, 6.0, 48
    ex, bd = _both(c, org, d, steps, eps, tmax, eval_eps_rel * D)
    _compare(ex, bd, steps, eval_eps_rel * D, D, f"3k cloud, eval_eps {eval_eps_rel:g} D")
    tor = oracle.fit(cl.p, cl.n, cl.a)
    to, ho, nso, no = oracle.trace(cl.p, tor, org, d, steps=steps, eps=eps, tmax=tmax)
    tb, hb = bd[0], bd[1]
    assert hb.sum() > 50 and (hb != ho).sum() <= max(2, 0.02 * len(hb))
    both = hb & ho
    assert np.abs(tb[both] - to[both]).max() < 1e-3 * D


def test_bounded_trace_benchmark_cloud_vs_exact():
    # the 131072-point cloud, where the bounded evaluation skips most units
    cl, _ = synth.mid(N=131072, grid=4)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    D = oracle.bbox_diag(cl.p)
    org, d = _rays(48, radius=1.5 * D, fov=45.0, seed=5)
    steps, eval_eps = 48, 1e-6 * D
    ex, bd = _both(c, org, d, steps, 1e-4 * D, 3.0 * D, eval_eps)
    both = _compare(ex, bd, steps, eval_eps, D, "131k cloud, eval_eps 1e-6 D")
    assert both.sum() > 200


def test_bounded_trace_edges_and_determinism():
    cl = synth.sphere_cloud(500, seed=10, jitter=0.0)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    org, d = _rays(8)
    t, hit, ns, _ = binding.trace(c.rec, c.N, _dev(org), _dev(d), steps=0, eps=1e-5, tmax=8.0, eval_eps=1e-6)
    assert torch.count_nonzero(t) == 0 and not hit.any() and torch.all(ns == 0)
    # ragged ray count, twice: the same bits
    o37, d37 = _dev(org[:37]), _dev(d[:37])
    a = binding.trace(c.rec, c.N, o37, d37, steps=40, eps=1e-5, tmax=8.0, eval_eps=1e-6)
    b = binding.trace(c.rec, c.N, o37, d37, steps=40, eps=1e-5, tmax=8.0, eval_eps=1e-6)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    with pytest.raises(binding.PtsError):
        binding.trace(c.rec, c.N, o37, d37, steps=4, eps=1e-5, tmax=8.0, eval_eps=-1.0)
