"""Parity of the HIP path (through the C ABI) with the FP64 oracle: torus fitting and evaluation.

Tolerance for phi: |phi_gpu - phi_oracle| <= 1e-5 * D, D = bounding-box
diagonal of the cloud (FP32 evaluation of an FP64 definition; derivation in
the design notes).  Inputs are the seeded synthetic workloads.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2607_16946_amd import binding, synth

pytestmark = pytest.mark.gpu

TOL_REL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _say(*a):
    print(*a, flush=True)


def _build(cl, **kw):
    return binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a), **kw)


def _oracle_phi(cl, x, nthreads=0):
    tor = oracle.fit(cl.p, cl.n, cl.a)
    return oracle.eval_sdf(cl.p, tor, x, nthreads=nthreads), tor


def _check_close(got, ref, D, what):
    err = np.abs(got.astype(np.float64) - ref)
    tol = TOL_REL * D
    _say(f"{what}: max err {err.max():.3e} (p99 {np.percentile(err, 99):.3e}) tol {tol:.3e}")
    assert np.all(np.isfinite(got))
    assert err.max() <= tol, what


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def test_decode_matches_oracle_tori():
    for name, (cl, _) in {"tiny": synth.tiny(Q=16), "mid-8k": synth.mid(N=8192, grid=4)}.items():
        _say("decode", name)
        c = _build(cl)
        dec = c.decode().cpu().numpy().astype(np.float64)
        tor = oracle.fit(cl.p, cl.n, cl.a)
        L = 1.0 / np.abs(tor.kminf)
        scale = np.abs(tor.c).max(axis=1) + 1.0
        assert np.all(np.abs(dec[:, 0:3] - tor.c).max(axis=1) <= 2e-6 * scale), name
        assert np.all(np.abs(np.abs(np.sum(dec[:, 3:6] * tor.u, axis=1)) - 1.0) < 1e-5), name
        assert np.all(np.abs(dec[:, 6] - tor.R) <= 1e-6 * (tor.R + 1.0)), name
        assert np.all(np.abs(dec[:, 7] - tor.r) <= 1e-6 * tor.r), name
        assert np.array_equal(dec[:, 8], tor.sgn), name
        assert np.all(np.abs(dec[:, 9] - L) <= 1e-6 * L), name
        info = c.info()
        D = oracle.bbox_diag(cl.p)
        assert abs(info.diag - D) < 1e-6 * D and info.N == cl.N
        assert info.n_direct + info.n_anchored == cl.N
        assert np.array_equal(dec[:, 10] > 0, L > 4.0 * D), name


def test_tiny_full_parity():
    cl, x = synth.tiny()
    _say("tiny full", cl.N, x.shape)
    c = _build(cl)
    got = c(_dev(x)).cpu().numpy()
    ref, _ = _oracle_phi(cl, x)
    _check_close(got, ref, oracle.bbox_diag(cl.p), "tiny")


def test_sphere_closed_form_on_device():
    cl = synth.sphere_cloud(3000, seed=7, jitter=0.0)
    x = np.random.default_rng(8).uniform(-1.5, 1.5, size=(3000, 3)).astype(np.float32)
    _say("sphere closed form")
    got = _build(cl)(_dev(x)).cpu().numpy().astype(np.float64)
    ref = np.linalg.norm(x.astype(np.float64), axis=1) - 1.0
    assert np.max(np.abs(got - ref)) <= TOL_REL * oracle.bbox_diag(cl.p)


def test_mid_small_full_parity():
    cl, x = synth.mid(N=8192, grid=16)
    _say("mid small", cl.N, x.shape)
    got = _build(cl)(_dev(x)).cpu().numpy()
    ref, _ = _oracle_phi(cl, x)
    _check_close(got, ref, oracle.bbox_diag(cl.p), "mid-8k")


def test_mid_full_size_sampled():
    # full 131072-point cloud and 128^3 lattice, in the launch configuration
    # the benchmark times; the oracle checks a seeded sample of queries.
    cl, x = synth.mid()
    _say("mid full", cl.N, x.shape)
    c = _build(cl)
    got = c(_dev(x)).cpu().numpy()
    idx = np.random.default_rng(11).choice(x.shape[0], size=1536, replace=False)
    ref, _ = _oracle_phi(cl, x[idx])
    _check_close(got[idx], ref, oracle.bbox_diag(cl.p), "mid full (sampled)")
    info = c.info()
    _say("anchored points:", info.n_anchored)


def test_mixed_coefficients_and_forms():
    cl = synth.mixed_forms_cloud()
    c = _build(cl)
    info = c.info()
    tor = oracle.fit(cl.p, cl.n, cl.a)
    D = oracle.bbox_diag(cl.p)
    L = 1.0 / np.abs(tor.kminf)
    _say(f"mixed coefficients: direct {info.n_direct}, anchored {info.n_anchored}")
    assert info.n_direct == int(np.sum(L <= 4.0 * D)) and 0 < info.n_anchored < cl.N
    dec = c.decode().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(dec[:, 0:3] - tor.c).max(axis=1) <= 2e-6 * (np.abs(tor.c).max(axis=1) + 1.0))
    assert np.all(np.abs(dec[:, 9] - L) <= 1e-6 * L)
    x = np.random.default_rng(5).uniform(-1.2, 1.2, size=(2500, 3)).astype(np.float32)
    got = c(_dev(x)).cpu().numpy()
    ref = oracle.eval_sdf(cl.p, tor, x)
    _check_close(got, ref, D, "mixed coefficients")


@pytest.mark.parametrize("Q", [1, 7, 255, 1000, 1025, 70001])
def test_ragged_query_counts(Q):
    cl, _ = synth.mid(N=3000, grid=4)
    x = np.random.default_rng(Q).uniform(-1.2, 1.2, size=(Q, 3)).astype(np.float32)
    _say("ragged Q", Q)
    got = _build(cl)(_dev(x)).cpu().numpy()
    sub = slice(0, min(Q, 600))
    ref, _ = _oracle_phi(cl, x[sub])
    _check_close(got[sub], ref, oracle.bbox_diag(cl.p), f"Q={Q}")


@pytest.mark.parametrize("N", [1, 2, 63, 513, 5000])
def test_ragged_point_counts(N):
    cl, _ = synth.mid(N=max(N, 16), grid=4)
    cl = synth.Cloud(cl.p[:N].copy(), cl.n[:N].copy(), cl.a[:N].copy(), {})
    x = np.random.default_rng(N).uniform(-1.2, 1.2, size=(777, 3)).astype(np.float32)
    _say("ragged N", N)
    got = _build(cl)(_dev(x)).cpu().numpy()
    ref, _ = _oracle_phi(cl, x)
    D = max(oracle.bbox_diag(cl.p), 1.0)
    _check_close(got, ref, D, f"N={N}")


def test_split_count_only_changes_rounding():
    cl, x = synth.mid(N=20000, grid=12)
    ref, tor = _oracle_phi(cl, x[:400])
    D = oracle.bbox_diag(cl.p)
    c0 = _build(cl)
    dec = c0.decode().cpu().numpy().astype(np.float64)
    bad = np.abs(dec[:, 0:3] - tor.c).max(axis=1) > 2e-6 * (np.abs(tor.c).max(axis=1) + 1.0)
    _say("splits: torus mismatches", int(bad.sum()), np.nonzero(bad)[0][:10])
    outs = {}
    for S in (0, 1, 2, 8, 16, 32):  # 16 and 32: the split-major blend
        plan = binding.eval_plan(cl.N, x.shape[0], binding.make_params(splits=S))
        o = _build(cl, splits=S)(_dev(x)).cpu().numpy().astype(np.float64)
        outs[S] = o
        _say(f"splits={S} plan={plan} max err {np.max(np.abs(o[:400] - ref)):.3e} tol {TOL_REL * D:.3e}")
    for S, o in outs.items():
        assert np.max(np.abs(o[:400] - ref)) <= TOL_REL * D, S
        assert np.max(np.abs(o - outs[0])) <= TOL_REL * D, S


def test_far_sweep_over_splits_is_exact():
    """A call with few query blocks sweeps the farthest point over the point
    splits and folds the rows; a call with many sweeps once per query block.
    The farthest distance M and the farthest point (through e_*) of a query
    must be the same bits either way (W and phi may differ by rounding: the
    blend's split count depends on the number of queries)."""
    cl, _ = synth.mid(N=40000, grid=4)
    c = _build(cl)
    lo, hi = synth.padded_bbox(cl.p, 0.1)
    big = np.random.default_rng(31).uniform(lo, hi, size=(1 << 19, 3)).astype(np.float32)
    small = big[:3000]
    assert binding.eval_plan(cl.N, small.shape[0])[1] > 1
    _, st_small = c(_dev(small), stats=True)
    _, st_big = c(_dev(big), stats=True)
    a = st_small.cpu().numpy()
    b = st_big[:3000].cpu().numpy()
    _say("far sweep split vs unsplit: M equal", np.array_equal(a[:, 0], b[:, 0]),
         "e_* equal", np.array_equal(a[:, 3:6], b[:, 3:6]))
    assert np.array_equal(a[:, 0].view(np.uint32), b[:, 0].view(np.uint32))
    assert np.array_equal(a[:, 3:6].view(np.uint32), b[:, 3:6].view(np.uint32))


def test_deterministic_bitwise():
    cl, x = synth.mid(N=10000, grid=10)
    c = _build(cl)
    xs = _dev(x)
    a = c(xs).cpu().numpy()
    b = c(xs).cpu().numpy()
    c2 = _build(cl)
    d = c2(xs).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.array_equal(a.view(np.uint32), d.view(np.uint32))


def test_degenerate_queries_and_stats():
    cl, _ = synth.tiny(Q=4)
    c = _build(cl)
    x = np.array([[np.nan, 0, 0], [np.inf, 0, 0], [0.1, 0.2, 0.3], cl.p[5]], dtype=np.float32)
    sdf, st = c(_dev(x), stats=True)
    sdf = sdf.cpu().numpy()
    st = st.cpu().numpy().astype(np.float64)
    assert np.isnan(sdf[0]) and np.isnan(sdf[1]) and np.all(np.isfinite(sdf[2:]))
    ref, rst = oracle.eval_sdf(cl.p, oracle.fit(cl.p, cl.n, cl.a), x[2:], stats=True)
    assert np.allclose(st[2:, 0], rst[:, 0], rtol=1e-6)            # M
    assert np.allclose(st[2:, 1], rst[:, 1], rtol=1e-4)            # shifted weight sum W
    assert np.allclose(st[2:, 2], sdf[2:], rtol=0, atol=0)         # phi
    # one-point cloud queried at the point itself: uniform weights, phi = g = 0 there
    one = synth.Cloud(cl.p[:1].copy(), cl.n[:1].copy(), cl.a[:1].copy(), {})
    v = _build(one)(_dev(cl.p[:1].copy())).cpu().numpy()
    assert abs(v[0]) < 1e-6


def test_degenerate_clouds():
    """Coincident points (zero bounding box: D = 1; at the point M = 0 and the
    weights are uniform), collinear points (zero-extent axes of the spatial
    sort) and a flat cloud (both curvatures floored, every point in the
    anchored torus form), each against the oracle."""
    rng = np.random.default_rng(51)
    # five copies of one point with different normals and coefficients
    p = np.repeat(np.array([[0.3, -0.2, 0.1]], np.float32), 5, axis=0)
    n = rng.normal(size=(5, 3)).astype(np.float32)
    a = np.zeros((5, 6), np.float32)
    a[:, 4:6] = rng.uniform(-0.8, -0.2, size=(5, 2))
    x = np.vstack([p[:1], rng.uniform(-1, 1, size=(200, 3))]).astype(np.float32)
    cases = {"coincident": synth.Cloud(p, n, a, {})}
    # points on a line
    tl = np.linspace(-1, 1, 300, dtype=np.float32)[:, None]
    pl = (tl * np.array([[0.6, 0.8, 0.0]], np.float32)).astype(np.float32)
    nl = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (300, 1))
    al = np.zeros((300, 6), np.float32)
    al[:, 4] = -0.5
    cases["collinear"] = synth.Cloud(pl, nl, al, {})
    # a flat square patch with a = 0
    g = np.stack(np.meshgrid(np.linspace(-1, 1, 40), np.linspace(-1, 1, 40)), -1).reshape(-1, 2)
    pf = np.c_[g, np.zeros(len(g))].astype(np.float32)
    nf = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (len(g), 1))
    cases["flat"] = synth.Cloud(pf, nf, np.zeros((len(g), 6), np.float32), {})
    for name, cl in cases.items():
        c = _build(cl)
        if name == "flat":
            assert c.info().n_anchored == cl.N
        got = c(_dev(x)).cpu().numpy()
        ref, _ = _oracle_phi(cl, x)
        D = max(oracle.bbox_diag(cl.p), 1.0)
        _check_close(got, ref, D, name)


def test_invalid_inputs_rejected():
    cl, _ = synth.tiny(Q=4)
    n = cl.n.copy()
    n[17] = 0.0
    with pytest.raises(binding.PtsError) as e:
        binding.Cloud(_dev(cl.p), _dev(n), _dev(cl.a))
    assert e.value.code == binding.PTS_EINVAL
    a = cl.a.copy()
    a[3, 2] = np.nan
    with pytest.raises(binding.PtsError):
        binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(a))
    c = _build(cl)
    x = _dev(np.zeros((10, 3), np.float32))
    out = torch.empty(10, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    import ctypes
    rc = binding.lib().pts_eval(binding._ptr(c.rec), c.N, binding._ptr(x), 10, binding._ptr(out), None, None,
                                ctypes.byref(c.params), binding._ptr(ws), 16, binding._stream())
    assert rc == binding.PTS_EINVAL and b"workspace" in binding.lib().pts_last_error()


def test_blend_weights_three_spheres_hand_derived():
    """The hand-derived three-sphere blend (Sec. 4.2, Eqs. BasicFormulaShifted and
    RelationshipBetweenLambdaAndRadius; App. D) through pts_eval: phi, its statistics and grad phi
    against the stored closed forms, at C = 64 and C = 4."""
    import json
    import os
    G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "blend_weights.json")))
    p, n, a = (np.array(G[k], dtype=np.float32) for k in ("p", "n", "a"))
    x = np.array([G["x"]], dtype=np.float32)
    D = float(np.linalg.norm(p.max(0).astype(np.float64) - p.min(0)))
    for case in G["cases"]:
        _say(f"three spheres, C = {case['C']}")
        prm = binding.make_params(C=case["C"])
        c = binding.Cloud(_dev(p), _dev(n), _dev(a), C=case["C"])
        phi, g, st = binding.eval(c.rec, 3, _dev(x), prm, grad=True, stats=True)
        phi, g, st = phi.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
        _say(f"  phi {phi[0]:.8f} (closed form {case['phi']:.8f}), grad {g[0]} ({case['grad']})")
        assert abs(phi[0] - case["phi"]) <= TOL_REL * D
        assert np.abs(g[0] - np.array(case["grad"])).max() <= 1e-4 * max(1.0, np.abs(case["grad"]).max())
        assert abs(st[0, 0] - case["M"]) <= 1e-6 * case["M"]
        assert abs(st[0, 2] - case["phi"]) <= TOL_REL * D


@pytest.mark.parametrize("N,Q", [(4096, 4096), (1537, 777), (20000, 300001), (8192, 1 << 20), (3000, 1),
                                 (65536, 100), (65536, 3000)])
def test_eval_equals_the_three_stages(N, Q):
    """pts_eval leaves the farthest-point sweep's per-split maxima unfolded and lets the blend take their
    maximum; it must equal pts_eval_far + pts_eval_blend + pts_eval_combine bit for bit, whether the
    farthest-point sweep ran split (few query blocks) or not, and on repeated calls."""
    cl, _ = synth.mid(N=N, grid=4)
    x = np.random.default_rng(N + Q).uniform(-1.2, 1.2, size=(Q, 3)).astype(np.float32)
    prm = binding.make_params()
    c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a))
    xd = _dev(x)
    ws = torch.empty(binding.eval_ws_bytes(N, Q, prm), dtype=torch.uint8, device="cuda")
    staged = torch.empty(Q, dtype=torch.float32, device="cuda")
    binding.eval_far(c.rec, N, xd, prm, ws)
    binding.eval_blend(c.rec, N, xd, prm, ws)
    binding.eval_combine(N, Q, staged, prm, ws)
    ws.fill_(0xA5)  # the fused path must not depend on what the workspace held
    for rep in range(3):
        fused = binding.eval(c.rec, N, xd, prm, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(fused.view(torch.int32), staged.view(torch.int32)), (N, Q, rep)
    _say(f"eval N={N} Q={Q}: plan {binding.eval_plan(N, Q, prm)}, bitwise equal to the stages")
