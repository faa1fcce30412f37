"""Invariances of the definition on the device path (the oracle's pins of the
same names in test_oracle_pins.py, here through the C ABI in FP32).

Each comparison is between two GPU evaluations, each within 1e-5 D of the
oracle, so the bound is twice that (scaled with the cloud for the scaling
case):

* orientation flip: (n, a) -> (-n, a'), a' = (-a00, a01, -a10, a11, -a02, -a20)
  (the input frame becomes (s, -t, -n)) negates phi;
* scaling by alpha = 2 (exact in FP32): p -> alpha p, a00 -> alpha a00,
  a11, a02, a20 -> a / alpha gives phi(alpha x) = alpha phi(x);
* translation of points and queries leaves phi unchanged;
* a permutation of the points leaves phi unchanged;
* a rotation of an isotropic cloud (a01 = a10 = a11 = 0, a02 = a20) leaves
  phi unchanged;
* every point taken twice doubles every weight and leaves phi (a ratio of
  weighted sums) and grad phi unchanged; the error-bounded evaluation of the
  doubled cloud stays within its eps of it.

The first four run on a curved cloud (mostly direct tori) and on a nearly
flat cap (every torus in the anchored form).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_16946_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL_REL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _phi(p, n, a, x):
    c = binding.Cloud(_dev(p), _dev(n), _dev(a))
    return c(_dev(x)).cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


@pytest.fixture(scope="module", params=["mid", "cap"])
def cloud(request):
    """A curved cloud (mostly direct tori) and a nearly flat one (all anchored)."""
    rng = np.random.default_rng(41)
    if request.param == "mid":
        cl, _ = synth.mid(N=3000, grid=4)
        x = rng.uniform(-1.2, 1.2, size=(2500, 3))
    else:
        cl, x = synth.cap_cloud(N=2000, Q=2500)
    a = cl.a.astype(np.float64)
    a[:, 0] += rng.normal(scale=0.01, size=cl.N)
    a[:, 1:3] += rng.normal(scale=0.05, size=(cl.N, 2))
    p, n, a, x = (v.astype(np.float32) for v in (cl.p, cl.n, a, x))
    return p, n, a, x, oracle.bbox_diag(p)


def _report(what, err, tol):
    print(f"{what}: max deviation {err:.3e} (bound {tol:.3e})", flush=True)
    assert err <= tol, what


def test_orientation_flip_negates(cloud):
    p, n, a, x, D = cloud
    ap = (a * np.array([-1, 1, -1, 1, -1, -1], np.float32)).astype(np.float32)
    err = np.abs(_phi(p, n, a, x) + _phi(p, -n, ap, x)).max()
    _report("flip", err, 2 * TOL_REL * D)


def test_scale_by_two(cloud):
    p, n, a, x, D = cloud
    al = 2.0
    sa = (a * np.array([al, 1, 1, 1 / al, 1 / al, 1 / al], np.float32)).astype(np.float32)
    err = np.abs(_phi(al * p, n, sa, al * x) - al * _phi(p, n, a, x)).max()
    _report("scale", err, 2 * al * TOL_REL * D)


def test_translation_and_permutation(cloud):
    p, n, a, x, D = cloud
    phi = _phi(p, n, a, x)
    b = np.array([0.7, -1.9, 3.3], np.float32)
    _report("translation", np.abs(_phi(p + b, n, a, x + b) - phi).max(), 2 * TOL_REL * D)
    perm = np.random.default_rng(42).permutation(p.shape[0])
    _report("permutation", np.abs(_phi(p[perm], n[perm], a[perm], x) - phi).max(), 2 * TOL_REL * D)


def test_rotation_of_an_isotropic_cloud():
    cl = synth.sphere_cloud(3000, seed=43, jitter=0.01)
    p, n = cl.p.astype(np.float64), cl.n.astype(np.float64)
    a = np.zeros((cl.N, 6))
    k = -0.5 * (1.0 + 0.05 * np.random.default_rng(44).normal(size=cl.N))
    a[:, 4] = a[:, 5] = k
    a[:, 0] = 0.02
    q, _ = np.linalg.qr(np.random.default_rng(45).normal(size=(3, 3)))
    x = np.random.default_rng(46).uniform(-1.5, 1.5, size=(2000, 3))
    D = oracle.bbox_diag(p)
    phi = _phi(p, n, a, x)
    phi2 = _phi(p @ q.T, n @ q.T, a, x @ q.T)
    _report("rotation", np.abs(phi - phi2).max(), 2 * TOL_REL * D)


def test_duplicated_points(cloud):
    p, n, a, x, D = cloud
    c1 = binding.Cloud(_dev(p), _dev(n), _dev(a))
    c2 = binding.Cloud(_dev(np.concatenate([p, p])), _dev(np.concatenate([n, n])), _dev(np.concatenate([a, a])))
    xs = _dev(x)
    phi1, g1 = (t.cpu().numpy().astype(np.float64) for t in c1(xs, grad=True))
    phi2, g2 = (t.cpu().numpy().astype(np.float64) for t in c2(xs, grad=True))
    _report("duplicated points", np.abs(phi2 - phi1).max(), 2 * TOL_REL * D)
    _report("duplicated points, grad", np.abs(g2 - g1).max(), 2e-4)
    eps = 1e-6 * D
    pb = binding.eval_bounded(c2.rec, c2.N, xs, eps, c2.params).cpu().numpy().astype(np.float64)
    _report("duplicated points, bounded", np.abs(pb - phi1).max(), eps + 2 * TOL_REL * D)
