"""Offset surfaces and Booleans (Sec. 5.2, "Offset surfaces and Booleans").

With pts_params.offset = c every evaluator returns phi - c: checked bitwise
against phi - c computed from the plain result (the same FP32 subtraction),
with the statistics still holding phi.  Tracing the offset sphere hits radius
1 + c (closed-form ray intersection).  Booleans of two exact sphere SDFs equal
min/max of the closed forms; the elementwise compositions equal NumPy's.
"""

import numpy as np
import pytest
import torch

from paper_2607_16946_amd import binding, synth

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def test_offset_is_phi_minus_c_everywhere():
    cl, x = synth.tiny(Q=3000, N=2000)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xs = _dev(x)
    off = 0.137
    p0 = binding.make_params()
    p1 = binding.make_params(offset=off)
    cf = torch.tensor(off, dtype=torch.float32, device="cuda")
    phi = binding.eval(c.rec, c.N, xs, p0)
    assert torch.equal(binding.eval(c.rec, c.N, xs, p1), phi - cf)
    s0, st0 = binding.eval(c.rec, c.N, xs, p0, stats=True)
    s1, st1 = binding.eval(c.rec, c.N, xs, p1, stats=True)
    assert torch.equal(s1, s0 - cf) and torch.equal(st1, st0)
    for kind in ("sspd", "shc"):
        b0 = binding.eval_baseline(c.rec, c.N, xs, kind, p0)
        assert torch.equal(binding.eval_baseline(c.rec, c.N, xs, kind, p1), b0 - cf)
    e0 = binding.eval_bounded(c.rec, c.N, xs, 1e-6, p0)
    assert torch.equal(binding.eval_bounded(c.rec, c.N, xs, 1e-6, p1), e0 - cf)
    with pytest.raises(binding.PtsError):
        binding.eval(c.rec, c.N, xs, binding.make_params(offset=float("inf")))


@pytest.mark.parametrize("off", [0.25, -0.3])
@pytest.mark.parametrize("eval_eps", [None, 1e-7])
def test_trace_offset_sphere(off, eval_eps):
    # eval_eps: the march on the error-bounded phi (pts_trace_bounded)
    cl = synth.sphere_cloud(2000, seed=9, jitter=0.0)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    org, d = synth.camera_rays(32, radius=3.0, fov_deg=40.0, seed=0)
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    t, hit, _, nrm = binding.trace(c.rec, c.N, _dev(org), _dev(d), steps=64, eps=1e-5, tmax=8.0,
                                   params=binding.make_params(offset=off), eval_eps=eval_eps)
    t, hit, nrm = t.cpu().numpy(), hit.cpu().numpy(), nrm.cpu().numpy()
    o, dd = org.astype(np.float64), d.astype(np.float64)
    R = 1.0 + off
    b = np.sum(o * dd, axis=1)
    disc = b * b - (np.sum(o * o, axis=1) - R * R)
    expect = disc > 0.05 * R * R
    print(f"offset {off}: {hit.sum()} hits, {expect.sum()} expected", flush=True)
    assert expect.sum() > 100 and hit[expect].all()
    tstar = -b - np.sqrt(np.where(disc > 0, disc, 0))
    assert np.abs(t[expect] - tstar[expect]).max() < 1e-4
    xh = o + t[:, None] * dd
    assert np.abs(nrm[expect] - xh[expect] / np.linalg.norm(xh[expect], axis=1, keepdims=True)).max() < 1e-3
    assert not hit[disc < -1e-2].any()


def test_booleans_of_two_spheres():
    a = synth.sphere_cloud(3000, seed=21, jitter=0.0)
    bcl = synth.sphere_cloud(3000, seed=22, jitter=0.0)
    shift = np.array([0.8, 0.0, 0.0], np.float32)
    b = synth.Cloud(bcl.p + shift, bcl.n, bcl.a, {})
    ca = binding.Cloud(_dev(a.p), _dev(a.n), _dev(a.a))
    cb = binding.Cloud(_dev(b.p), _dev(b.n), _dev(b.a))
    x = np.random.default_rng(23).uniform(-2.0, 2.8, size=(4000, 3)).astype(np.float32)
    xs = _dev(x)
    fa, fb = ca(xs), cb(xs)
    xd = x.astype(np.float64)
    ta = np.linalg.norm(xd, axis=1) - 1.0
    tb = np.linalg.norm(xd - shift, axis=1) - 1.0
    for op, ref in (("union", np.minimum(ta, tb)), ("intersect", np.maximum(ta, tb)),
                    ("subtract", np.maximum(ta, -tb))):
        got = binding.compose(fa, fb, op).cpu().numpy()
        err = np.abs(got - ref).max()
        print(f"{op}: max err {err:.3e}", flush=True)
        assert err <= 1e-5 * 4.0


def test_compose_elementwise():
    rng = np.random.default_rng(24)
    a = rng.normal(size=5003).astype(np.float32)
    b = rng.normal(size=5003).astype(np.float32)
    a[7] = np.nan
    b[11] = np.nan
    A, B = _dev(a), _dev(b)
    with np.errstate(invalid="ignore"):
        refs = {"union": np.minimum(a, b), "intersect": np.maximum(a, b), "subtract": np.maximum(a, -b),
                "offset": a - np.float32(0.5)}
    for op, ref in refs.items():
        got = binding.compose(A, None if op == "offset" else B, op, c=0.5).cpu().numpy()
        assert np.array_equal(got, ref, equal_nan=True), op
    # in place, and empty
    binding.compose(A, B, "union", out=A)
    assert np.array_equal(A.cpu().numpy(), refs["union"], equal_nan=True)
    assert binding.compose(A[:0], B[:0], "union").numel() == 0
    with pytest.raises(ValueError):
        binding.compose(A, None, "union")
