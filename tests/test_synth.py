"""Seeded workload generators: determinism and shape of the synthetic inputs."""

import hashlib

import numpy as np

from paper_2607_16946_amd import synth


def _h(*arrs):
    m = hashlib.sha256()
    for a in arrs:
        m.update(np.ascontiguousarray(a).tobytes())
    return m.hexdigest()


def test_generators_are_deterministic():
    c1, x1 = synth.tiny(Q=256, N=512)
    c2, x2 = synth.tiny(Q=256, N=512)
    assert _h(c1.p, c1.n, c1.a, x1) == _h(c2.p, c2.n, c2.a, x2)
    m1, y1 = synth.mid(N=2048, grid=8)
    m2, y2 = synth.mid(N=2048, grid=8)
    assert _h(m1.p, m1.n, m1.a, y1) == _h(m2.p, m2.n, m2.a, y2)


def test_workload_shapes():
    cl, x = synth.tiny()
    assert cl.p.shape == (4096, 3) and x.shape == (4096, 3)
    assert cl.p.dtype == np.float32 and cl.a.shape == (4096, 6)
    assert np.allclose(np.linalg.norm(cl.p, axis=1), 1.0, atol=1e-6)
    # curvature 1 with 1% jitter, convex with outward normals: a02, a20 ~ -1/2
    assert abs(cl.a[:, 4:6].mean() + 0.5) < 1e-3 and 0.003 < cl.a[:, 4:6].std() < 0.007
    m, y = synth.mid(N=4096, grid=16)
    assert m.N == 4096 and y.shape == (16 ** 3, 3)
    assert np.allclose(np.linalg.norm(m.n, axis=1), 1.0, atol=1e-6)
    lo, hi = m.p.min(0), m.p.max(0)
    assert np.all(y.min(0) < lo) and np.all(y.max(0) > hi)    # padded lattice
    cl3, q3, mask = synth.diff_workload(N=1024, Q=2048)
    assert cl3.N == 1024 and q3.shape == (2048, 3) and mask.sum() == 1024
    c4 = synth.serving_cloud(3)
    assert 1024 <= c4.N <= 262144
    org, d = synth.camera_rays(16)
    assert org.shape == (256, 3) and np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)


def test_large_outliers_and_density():
    cl, x = synth.large(N=20000, Q=1000)
    assert cl.N == 20000 and cl.meta["outliers"] == 600
    assert x.shape == (1000, 3)


def test_cap_cloud_is_nearly_flat():
    """The cap generator: points on the sphere of radius 50, unit outward
    normals, unequal curvatures -(1 +- e)/50; by the oracle's fit every torus
    radius L = 1/|kappa_min| exceeds 4 bbox diagonals (the anchored form's range)."""
    import oracle

    cl, x = synth.cap_cloud(N=600, Q=300)
    c2, x2 = synth.cap_cloud(N=600, Q=300)
    assert _h(cl.p, cl.n, cl.a, x) == _h(c2.p, c2.n, c2.a, x2)
    assert cl.N == 600 and x.shape == (300, 3)
    p = cl.p.astype(np.float64)
    assert np.allclose(np.linalg.norm(p - [0.0, 0.0, -50.0], axis=1), 50.0, atol=1e-4)
    assert np.allclose(np.linalg.norm(cl.n, axis=1), 1.0, atol=1e-6)
    assert np.all(cl.a[:, 4] < cl.a[:, 5]) and np.all(cl.a[:, 5] < 0)
    tor = oracle.fit(cl.p, cl.n, cl.a)
    L = 1.0 / np.abs(np.asarray(tor.kminf))
    assert np.all(L > 4.0 * oracle.bbox_diag(cl.p))
