"""The upper end of the accepted screening constant (C <= 75) against the FP64 oracle.

phi does not depend on the additive shift of Eq. (BasicFormulaShifted); the
FP32 kernels shift the exponents by min(C, 64) instead of C (Sec. 4.2 fixes
C = 64), so for 64 < C <= 75 every weighted sum, the gradient (which reuses
the forward's weight sum W), the signed Hopf-Cole baseline (whose -log|s|
undoes the shift) and the radius-limited evaluation (its own shift) must still
agree with the oracle.  The clouds are dense near the queries (the case where
the largest weights add up), and one query sits at the centre of a sphere
cloud, equidistant from every point (the case where the smallest weights must
not underflow).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_16946_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
EPS32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _queries(cl, n, seed):
    """Half within 0.02 of the surface along the normal, half uniform in the padded bbox, plus the bbox centre."""
    rng = np.random.default_rng(seed)
    i = rng.integers(cl.N, size=n // 2)
    near = cl.p[i] + cl.n[i] * rng.uniform(-0.02, 0.02, size=(n // 2, 1))
    lo, hi = synth.padded_bbox(cl.p, 0.1)
    far = rng.uniform(lo, hi, size=(n - n // 2, 3))
    ctr = 0.5 * (cl.p.min(0) + cl.p.max(0))
    return np.vstack([near, far, ctr[None]]).astype(np.float32)


def _cases():
    mid, _ = synth.mid(N=6000, grid=4)
    sph, _ = synth.tiny(Q=16, N=4096)
    return {"mid-6000": mid, "sphere-4096": sph}


@pytest.mark.parametrize("C", [70.0, 75.0])
def test_eval_and_gradient_at_large_C(C):
    for name, cl in _cases().items():
        x = _queries(cl, 3000, 7)
        c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a), C=C)
        phi, g = binding.eval(c.rec, c.N, _dev(x), c.params, grad=True)
        phi, g = phi.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
        tor = oracle.fit(cl.p, cl.n, cl.a)
        ref, gref = oracle.eval_sdf(cl.p, tor, x, C=C, grad=True)
        D = oracle.bbox_diag(cl.p)
        err = np.abs(phi - ref)
        # grad phi is not defined where FP32 cannot order the two farthest points (the lambda_x term)
        d = np.linalg.norm(x.astype(np.float64)[:, None, :] - cl.p.astype(np.float64)[None], axis=2)
        top = np.sort(d, axis=1)[:, -2:]
        decided = top[:, 1] - top[:, 0] > 2e-6 * top[:, 1]
        gerr = np.abs(g - gref).max(axis=1)[decided]
        print(f"C={C} {name}: max |phi err| {err.max():.3e} (tol {TOL * D:.3e}), centre query phi {phi[-1]:.6f} "
              f"(oracle {ref[-1]:.6f}); grad max err {gerr.max():.3e} over {decided.sum()} queries", flush=True)
        assert np.all(np.isfinite(phi)) and np.all(np.isfinite(g))
        assert err.max() <= TOL * D
        assert gerr.max() <= 1e-4


def test_hopf_cole_baseline_at_large_C():
    C = 75.0
    cl, _ = synth.mid(N=2000, grid=4)
    x = _queries(cl, 1500, 11)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a), C=C)
    for kind in ("sspd", "shc"):
        phi = binding.eval_baseline(c.rec, c.N, _dev(x), kind, c.params).cpu().numpy().astype(np.float64)
        ref, s, sabs = oracle.eval_baseline(cl.p, cl.n, x, kind, C=C, raw=True)
        D = max(oracle.bbox_diag(cl.p), 1.0)
        if kind == "sspd":
            ok = np.ones(len(x), bool)
            tol = np.full(len(x), TOL * D)
        else:
            M = np.linalg.norm(x.astype(np.float64)[:, None, :] - cl.p.astype(np.float64)[None], axis=2).max(axis=1)
            lam = 2 * C / M
            ok = np.abs(s) > 1e-4 * sabs
            tol = TOL * D + 64 * EPS32 * sabs / (np.abs(s) * lam)
        err = np.abs(phi - ref)
        print(f"C={C} {kind}: {ok.sum()}/{len(x)} compared, max err {err[ok].max():.3e}", flush=True)
        assert ok.sum() > 0.9 * len(x)
        assert np.all(err[ok] <= tol[ok])


def test_radius_limited_at_large_C():
    C = 75.0
    cl, _ = synth.mid(N=3000, grid=4)
    x = _queries(cl, 1500, 13)
    prm = binding.make_params(C=C)
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a), C=C)
    binding.radius_prepare(c.rec, c.N, prm)
    info = binding.radius_info(c.rec)
    assert abs(info.reval * info.lam - 2 * C) <= 1e-4 * 2 * C
    tor = oracle.fit(cl.p, cl.n, cl.a)
    ref, cnt_o = oracle.eval_radius(cl.p, tor, x, float(info.lam), float(info.reval), 32)
    phi, cnt = binding.eval_radius(c.rec, c.N, _dev(x), count=True)
    phi, cnt = phi.cpu().numpy().astype(np.float64), cnt.cpu().numpy()
    # queries whose selection FP32 decides the same way (none within 1e-4 R_eval of the radius, a gap after the 32nd)
    d = np.linalg.norm(x.astype(np.float64)[:, None, :] - cl.p.astype(np.float64)[None], axis=2)
    edge = np.any(np.abs(d - info.reval) <= 1e-4 * info.reval, axis=1)
    ds = np.sort(d, axis=1)[:, :33]
    gap = ds[:, 32] - ds[:, 31] > 1e-5 * ds[:, 31]
    m = ~edge & (np.any(d <= info.reval, axis=1) | gap)
    D = max(oracle.bbox_diag(cl.p), 1.0)
    err = np.abs(phi - ref)[m]
    print(f"radius C={C}: {m.sum()} decided ({(cnt_o[m] > 0).sum()} within R_eval), max err {err.max():.3e}",
          flush=True)
    assert m.sum() > 0.9 * len(x)
    assert np.array_equal(cnt[m], cnt_o[m])
    assert err.max() <= TOL * D
