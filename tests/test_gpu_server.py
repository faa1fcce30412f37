"""The serving engine on the device.

* Each request's result is bitwise the same alone and in a mix of uneven
  requests against different clouds, submitted from several threads.
* Query results equal pts_eval with the cloud's serving split, trace results
  equal pts_trace with its default splits, and phi agrees with the FP64 oracle
  (within 1e-5 of the bbox diagonal on a sample of queries).
* Admission keeps admitted buffers within the budget while requests queue.
* A second packed launch is issued while the first is in flight.
"""

import threading
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2607_16946_amd import binding, synth
from paper_2607_16946_amd.server import Server

pytestmark = pytest.mark.gpu

TOL = 1e-5  # of the bbox diagonal


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.lib()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _clouds():
    return [synth.sphere_cloud(3000, seed=11, jitter=0.01),
            synth.mid(N=20000, grid=4)[0],
            synth.serving_cloud(3, nmax=70000),
            synth.mixed_forms_cloud(6000)]   # direct, anchored and R = 0 tori


def _queries(cl, q, seed):
    rng = np.random.default_rng(seed)
    lo, hi = synth.padded_bbox(cl.p, 0.1)
    return rng.uniform(lo, hi, size=(q, 3)).astype(np.float32)


def _rays(res, seed):
    o, d = synth.camera_rays(res, radius=3.0, fov_deg=45.0, seed=seed)
    d = d.astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


def _requests(clouds, ids):
    """(kind, cloud index, inputs) for a mix of uneven query and trace requests."""
    reqs = []
    qs = [1, 7, 511, 512, 513, 5000, 40000, 3]
    for i, q in enumerate(qs):
        k = i % len(clouds)
        reqs.append(("eval", k, _queries(clouds[k], q, 100 + i)))
    for i in range(3):
        k = (i + 1) % len(clouds)
        reqs.append(("trace", k, _rays(40 + 8 * i, 7 + i)))
    return reqs


def _submit(S, ids, r):
    kind, k, inp = r
    if kind == "eval":
        return S.submit_eval(ids[k], inp)
    o, d = inp
    return S.submit_trace(ids[k], o, d, steps=24, eps=1e-4, tmax=6.0, normals=True)


def _same(a, b):
    if isinstance(a, dict):
        return all(_same(a[k], b[k]) for k in a)
    return np.array_equal(a, b)


def test_alone_vs_mixed_is_bitwise_identical():
    clouds = _clouds()
    with Server(budget_bytes=4 << 30) as S:
        ids = [S.add_cloud(c.p, c.n, c.a) for c in clouds]
        reqs = _requests(clouds, ids)
        print(f"server: {len(reqs)} requests on clouds N={[c.N for c in clouds]}", flush=True)
        alone = [S.wait(_submit(S, ids, r)) for r in reqs]
        S.reset_stats()
        order = np.random.default_rng(0).permutation(len(reqs))
        mixed = [None] * len(reqs)
        errors = []

        def client(part):
            try:
                ts = [(i, _submit(S, ids, reqs[i])) for i in part]
                for i, t in ts:
                    mixed[i] = S.wait(t)
            except Exception as e:  # noqa: BLE001 -- re-raised below
                errors.append(e)

        th = [threading.Thread(target=client, args=(order[j::3],)) for j in range(3)]
        for x in th:
            x.start()
        for x in th:
            x.join(120)
        assert not errors, errors[0]
        st = S.stats()
        print(f"mixed run: launches={st['launches']} max_batch={st['max_batch_requests']} "
              f"overlapped={st['overlapped_launches']} p50={st['p50_ms']:.2f} ms p99={st['p99_ms']:.2f} ms",
              flush=True)
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["max_batch_requests"] >= 2
        for i, (a, m) in enumerate(zip(alone, mixed)):
            assert _same(a, m), f"request {i} ({reqs[i][0]}) differs alone vs mixed"


def test_server_equals_direct_calls_and_oracle():
    clouds = _clouds()
    with Server(budget_bytes=4 << 30) as S:
        ids = [S.add_cloud(c.p, c.n, c.a) for c in clouds]
        for k, (cl, cid) in enumerate(zip(clouds, ids)):
            N, split = S.cloud_plan(cid)
            assert N == cl.N
            prm = binding.make_params(splits=split)
            c = binding.Cloud(_dev(cl.p), _dev(cl.n), _dev(cl.a), splits=split)
            x = _queries(cl, 3000 + 517 * k, 300 + k)
            got = S.wait(S.submit_eval(cid, x))
            # query requests use pts_eval's own plan (default parameters); traces the cloud's split
            ref = binding.eval(c.rec, c.N, _dev(x)).cpu().numpy()
            assert np.array_equal(got, ref), f"cloud {k}: server != pts_eval (plan {binding.eval_plan(c.N, len(x))})"
            for n_small in (1, 37, 300):  # few queries: many short splits, the wavefront combine beyond 64
                xs = x[:n_small]
                assert np.array_equal(S.wait(S.submit_eval(cid, xs)), binding.eval(c.rec, c.N, _dev(xs)).cpu().numpy())
            D = oracle.bbox_diag(cl.p)
            tor = oracle.fit(cl.p, cl.n, cl.a)
            sub = x[:600]
            phi_o = oracle.eval_sdf(cl.p, tor, sub)
            err = np.abs(got[:600].astype(np.float64) - phi_o).max() / D
            print(f"cloud {k}: N={N} split={split} max|phi-oracle|/D = {err:.2e}", flush=True)
            assert err <= TOL
            o, d = _rays(32, 20 + k)
            r = S.wait(S.submit_trace(cid, o, d, steps=24, eps=1e-4, tmax=6.0, normals=True))
            t, hit, ns, nrm = binding.trace(c.rec, c.N, _dev(o), _dev(d), steps=24, eps=1e-4, tmax=6.0, params=prm)
            assert np.array_equal(r["t"], t.cpu().numpy())
            assert np.array_equal(r["hit"], hit.cpu().numpy().astype(np.int32))
            assert np.array_equal(r["steps"], ns.cpu().numpy())
            assert np.array_equal(r["normal"], nrm.cpu().numpy())
            assert r["hit"].sum() > 0


def _request_bytes(N, q):
    """Device bytes of one query request: the mock executor uses the same layouts."""
    with Server(budget_bytes=1 << 30, mock=True, max_batch_work=2048, mock_pairs_per_s=N * q / 0.2) as M:
        c = M.add_cloud(np.zeros((N, 3), np.float32), np.tile(np.float32([0, 0, 1]), (N, 1)),
                        np.zeros((N, 6), np.float32))
        t = M.submit_eval(c, np.zeros((q, 3), np.float32))
        seen = 0
        for _ in range(2000):
            seen = M.stats()["bytes_inflight"]
            if seen:
                break
            time.sleep(0.001)
        M.wait(t)
        return seen, M.stats()["bytes_resident"], M.stats()["bytes_reserved"]


def test_budget_admission_on_device():
    cl = synth.serving_cloud(5, nmax=60000)
    q = 30000
    rb, resident, reserved = _request_bytes(cl.N, q)
    budget = reserved + resident + int(2.5 * rb)
    with Server(budget_bytes=budget, max_batch_work=2048) as S:
        cid = S.add_cloud(cl.p, cl.n, cl.a)
        xs = [_queries(cl, q, 500 + i) for i in range(8)]
        alone = S.wait(S.submit_eval(cid, xs[0]))
        ts = [S.submit_eval(cid, x) for x in xs]
        peak = 0
        queued_seen = False
        while not all(S.poll(t) in ("done", "failed", "cancelled") for t in ts):
            st = S.stats()
            assert st["bytes_inflight"] <= 2 * rb
            assert st["bytes_inflight"] + st["bytes_resident"] + st["bytes_reserved"] <= budget
            peak = max(peak, st["inflight"])
            queued_seen |= st["queued"] > 0 and st["inflight"] > 0
            time.sleep(0.0005)
        outs = [S.wait(t) for t in ts]
        print(f"budget {budget} B, request {rb} B: peak inflight {peak}, queued seen {queued_seen}", flush=True)
        assert peak <= 2
        assert np.array_equal(outs[0], alone)


def test_overlapping_launches_and_edge_requests():
    clouds = _clouds()
    with Server(budget_bytes=4 << 30) as S:
        ids = [S.add_cloud(c.p, c.n, c.a) for c in clouds]
        # edge requests: nothing to compute / no steps
        assert S.wait(S.submit_eval(ids[0], np.zeros((0, 3), np.float32))).shape == (0,)
        o, d = _rays(8, 1)
        r = S.wait(S.submit_trace(ids[0], o, d, steps=0, eps=1e-4, tmax=6.0))
        assert np.all(r["t"] == 0) and not r["hit"].any() and np.all(r["steps"] == 0) and np.all(r["normal"] == 0)
        # every ray misses (camera turned away): no hit rays to take normals at
        r = S.wait(S.submit_trace(ids[0], o, -d, steps=32, eps=1e-4, tmax=6.0))
        assert not r["hit"].any() and np.all(r["normal"] == 0) and np.all(r["t"] > 0)
        # a single ray that hits, and one that misses
        o1 = np.array([[0.0, 0.0, 3.0], [0.0, 0.0, 3.0]], np.float32)
        d1 = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, 1.0]], np.float32)
        r = S.wait(S.submit_trace(ids[0], o1, d1, steps=64, eps=1e-4, tmax=6.0))
        assert r["hit"].tolist() == [1, 0] and np.all(r["normal"][1] == 0)
        assert abs(float(r["normal"][0][2]) - 1.0) < 1e-2
        S.reset_stats()
        t0 = time.time()
        # a long launch first (about 10^10 pairs), then arrivals while it runs
        ts = [S.submit_eval(ids[2], _queries(clouds[2], 400000, 899))]
        time.sleep(0.002)
        for i in range(40):
            k = i % 3
            ts.append(S.submit_eval(ids[k], _queries(clouds[k], 2000 + 997 * i, 900 + i)))
            time.sleep(0.0005)
        for t in ts:
            S.wait(t)
        wall = time.time() - t0
        st = S.stats()
        print(f"stream: launches={st['launches']} overlapped={st['overlapped_launches']} "
              f"device busy {st['busy_s'] * 1e3:.1f} ms over {wall * 1e3:.1f} ms wall", flush=True)
        assert st["completed"] == 41
        assert st["overlapped_launches"] > 0


def test_nonfinite_queries_and_rays_in_requests():
    # NaN / inf queries inside a query request and NaN ray origins inside a
    # trace request: non-finite results (no hit) for them, and the others
    # bitwise those of the clean requests
    cl = synth.mid(N=20000, grid=4)[0]
    x = _queries(cl, 3000, 55)
    xb = x.copy()
    bad = np.array([0, 9, 700, 2999] + list(range(1200, 1270)))
    xb[bad[0::2], 0] = np.nan
    xb[bad[1::2], 2] = np.inf
    good = np.ones(len(x), bool)
    good[bad] = False
    o, d = _rays(32, 3)
    ob = o.copy()
    rbad = np.array([1, 100, 500])
    ob[rbad, 1] = np.nan
    ok = np.ones(len(o), bool)
    ok[rbad] = False
    with Server(budget_bytes=1 << 30) as S:
        cid = S.add_cloud(cl.p, cl.n, cl.a)
        a = S.wait(S.submit_eval(cid, x))
        b = S.wait(S.submit_eval(cid, xb))
        assert not np.isfinite(b[~good]).any() and np.array_equal(a[good], b[good])
        ta = S.wait(S.submit_trace(cid, o, d, steps=24, eps=1e-4, tmax=6.0, normals=True))
        tb = S.wait(S.submit_trace(cid, ob, d, steps=24, eps=1e-4, tmax=6.0, normals=True))
        assert not tb["hit"][~ok].any()
        for k in ("t", "hit", "steps", "normal"):
            assert np.array_equal(ta[k][ok], tb[k][ok]), k
