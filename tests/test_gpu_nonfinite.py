"""Queries and rays with non-finite coordinates, scattered through a batch
and filling whole wavefronts, on a cloud of several 4096-point blocks: every
evaluator returns a non-finite value for them and, for the others, the same
result as the batch without them (bitwise where a query's result does not
depend on the other queries; within the error bound for the error-bounded
evaluation, whose wavefront votes do)."""

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


@pytest.fixture(scope="module")
def case():
    cl, _ = synth.mid(N=20000, grid=4)          # 313 units, 5 blocks
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    D = oracle.bbox_diag(cl.p)
    lo, hi = synth.padded_bbox(cl.p, 0.1)
    x = np.random.default_rng(31).uniform(lo, hi, size=(4096, 3)).astype(np.float32)
    bad_idx = np.array(sorted({0, 1, 17, 63, 64, 500, 4095} | set(range(1000, 1070))))
    xb = x.copy()
    xb[bad_idx[0::3], 0] = np.nan
    xb[bad_idx[1::3], 1] = np.inf
    xb[bad_idx[2::3], 2] = -np.inf
    good = np.ones(len(x), bool)
    good[bad_idx] = False
    return cl, c, D, x, xb, good


def _np(t):
    return t.cpu().numpy()


def test_eval_grad_stats_and_baselines(case):
    cl, c, D, x, xb, good = case
    for kw in ({}, {"grad": True, "stats": True}):
        a = binding.eval(c.rec, c.N, _dev(x), c.params, **kw)
        b = binding.eval(c.rec, c.N, _dev(xb), c.params, **kw)
        a = a if isinstance(a, tuple) else (a,)
        b = b if isinstance(b, tuple) else (b,)
        assert not np.isfinite(_np(b[0])[~good]).any()
        for u, v in zip(a, b):
            if u is not None:
                assert np.array_equal(_np(u)[good], _np(v)[good])
    for kind in ("sspd", "shc"):
        a = _np(binding.eval_baseline(c.rec, c.N, _dev(x), kind, c.params))
        b = _np(binding.eval_baseline(c.rec, c.N, _dev(xb), kind, c.params))
        assert not np.isfinite(b[~good]).any() and np.array_equal(a[good], b[good])


def test_bounded_and_radius(case):
    cl, c, D, x, xb, good = case
    for eps_rel in (1e-6, 1e-4):
        eps = eps_rel * D
        a = _np(binding.eval_bounded(c.rec, c.N, _dev(x), eps, c.params))
        b = _np(binding.eval_bounded(c.rec, c.N, _dev(xb), eps, c.params))
        assert not np.isfinite(b[~good]).any()
        assert np.abs(a[good].astype(np.float64) - b[good]).max() <= 2 * eps + 2e-6 * D
    binding.radius_prepare(c.rec, c.N, c.params)
    a = _np(binding.eval_radius(c.rec, c.N, _dev(x)))
    b = _np(binding.eval_radius(c.rec, c.N, _dev(xb)))
    assert not np.isfinite(b[~good]).any() and np.array_equal(a[good], b[good])


def test_traces(case):
    cl, c, D, x, xb, good = case
    ctr = 0.5 * (cl.p.min(0) + cl.p.max(0))
    org, d = synth.camera_rays(32, radius=1.5 * D, fov_deg=45.0, seed=6, target=tuple(ctr))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    orb = org.astype(np.float32).copy()
    bad = np.array([0, 5, 300] + list(range(600, 680)))
    orb[bad, 0] = np.nan
    ok = np.ones(len(orb), bool)
    ok[bad] = False
    kw = dict(steps=48, eps=1e-4 * D, tmax=3.0 * D)
    ta, ha, _, na = (_np(v) for v in binding.trace(c.rec, c.N, _dev(org), _dev(d), **kw))
    tb, hb, _, nb = (_np(v) for v in binding.trace(c.rec, c.N, _dev(orb), _dev(d), **kw))
    assert not hb[~ok].any()
    assert np.array_equal(ta[ok], tb[ok]) and np.array_equal(ha[ok], hb[ok]) and np.array_equal(na[ok], nb[ok])
    ee = 1e-6 * D
    ta, ha, _, _ = (_np(v) for v in binding.trace(c.rec, c.N, _dev(org), _dev(d), eval_eps=ee, **kw))
    tb, hb, _, _ = (_np(v) for v in binding.trace(c.rec, c.N, _dev(orb), _dev(d), eval_eps=ee, **kw))
    assert not hb[~ok].any()
    assert (ha[ok] != hb[ok]).sum() <= max(2, 0.01 * ok.sum())
    both = ha & hb & ok
    assert np.abs(ta[both] - tb[both]).max() <= 2 * 48 * ee + 2e-5 * D
