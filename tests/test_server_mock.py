"""The serving scheduler on a host without a GPU (mock executor).

In mock mode the server runs its real scheduler -- admission by budget and
slots, FIFO order, packing, two launches in flight, trace re-enqueue,
cancellation, failure isolation, latency accounting -- while a cost model
(pairs / mock_pairs_per_s seconds per launch) stands in for the kernels and
outputs are a fixed pattern (query requests: cloud + 1e-3 (j mod 1000); trace
requests: t = cloud, hit = j mod 2, every ray stops after min(steps, 3)).
"""

import threading
import time

import numpy as np
import pytest

from paper_2607_16946_amd import binding
from paper_2607_16946_amd.server import Server
from paper_2607_16946_amd.binding import PtsError


def _cloud(N):
    p = np.zeros((N, 3), np.float32)
    n = np.tile(np.float32([0, 0, 1]), (N, 1))
    a = np.zeros((N, 6), np.float32)
    return p, n, a


def _x(q):
    return np.zeros((q, 3), np.float32)


def _pattern(cid, q):
    return np.float32(cid) + np.float32(1e-3) * (np.arange(q) % 1000).astype(np.float32)


def _sample_until_done(S, tickets, fn, timeout=20.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        fn(S.stats(), [S.poll(t) for t in tickets])
        if all(S.poll(t) in ("done", "failed", "cancelled") for t in tickets):
            return
        time.sleep(0.001)
    raise AssertionError("requests did not finish")


def test_results_are_routed_to_their_requests():
    with Server(budget_bytes=64 << 20, mock=True, max_batch_work=4096, mock_pairs_per_s=1e11) as S:
        c1 = S.add_cloud(*_cloud(1000))
        c2 = S.add_cloud(*_cloud(5000))
        qs = [1, 7, 300, 4096, 9, 0]
        ts = [S.submit_eval(c1 if i % 2 else c2, _x(q)) for i, q in enumerate(qs)]
        tr = S.submit_trace(c2, _x(100), np.ones((100, 3), np.float32), steps=10, eps=1e-3, tmax=5.0)
        for i, (t, q) in enumerate(zip(ts, qs)):
            out = S.wait(t)
            assert out.shape == (q,)
            np.testing.assert_allclose(out, _pattern(c1 if i % 2 else c2, q), rtol=1e-6)
        r = S.wait(tr)
        assert np.all(r["t"] == c2)
        assert np.array_equal(r["hit"], np.arange(100) % 2)
        assert np.all(r["steps"] == 3) and np.all(r["normal"] == 0)
        st = S.stats()
        assert st["completed"] == 7 and st["failed"] == 0 and st["cancelled"] == 0
        assert st["launches"] >= 3                 # the trace advanced one step per launch
        assert st["max_batch_requests"] >= 2       # requests were packed into one launch
        assert 0 <= st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
        S.reset_stats()
        st = S.stats()
        assert st["completed"] == 0 and st["launches"] == 0 and st["p99_ms"] == 0


def _request_bytes(N, q):
    """Device bytes one query request takes (measured on a throwaway server)."""
    with Server(budget_bytes=64 << 20, mock=True, max_batch_work=1024, mock_pairs_per_s=N * q / 0.2) as S:
        c = S.add_cloud(*_cloud(N))
        t = S.submit_eval(c, _x(q))
        seen = 0
        for _ in range(2000):
            seen = max(seen, S.stats()["bytes_inflight"])
            if seen:
                break
            time.sleep(0.001)
        S.wait(t)
        st = S.stats()
        return seen, st["bytes_resident"], st["bytes_reserved"]


def test_admission_by_budget_and_fifo():
    N, q = 4096, 4096
    rb, resident, reserved = _request_bytes(N, q)
    assert rb > 0
    budget = reserved + resident + int(2.5 * rb)
    rate = N * q / 0.03  # 30 ms per single-request launch
    with Server(budget_bytes=budget, mock=True, max_batch_work=1024, mock_pairs_per_s=rate) as S:
        c = S.add_cloud(*_cloud(N))
        assert S.stats()["bytes_resident"] == resident
        small = [S.submit_eval(c, _x(q)) for _ in range(6)]
        seen = {"queued": 0, "max_inflight": 0}

        def check(st, states):
            assert st["bytes_inflight"] <= 2 * rb
            assert st["bytes_inflight"] + st["bytes_resident"] + st["bytes_reserved"] <= budget
            assert st["inflight"] <= 2
            seen["max_inflight"] = max(seen["max_inflight"], st["inflight"])
            if st["queued"] and st["inflight"]:
                seen["queued"] += 1

        _sample_until_done(S, small, check)
        assert seen["max_inflight"] == 2 and seen["queued"] > 0   # back-pressure happened
        for t in small:
            np.testing.assert_allclose(S.wait(t), _pattern(c, q), rtol=1e-6)

        # FIFO: a request that needs both slots' memory is not overtaken
        a, b = S.submit_eval(c, _x(q)), S.submit_eval(c, _x(q))
        big = S.submit_eval(c, _x(2 * q))
        d = S.submit_eval(c, _x(q))

        def fifo(st, states):
            sa, sb, sbig, sd = states
            if sbig == "queued":
                assert sd == "queued"

        _sample_until_done(S, [a, b, big, d], fifo)
        for t in (a, b, big, d):
            S.wait(t)

        # a request larger than the budget is refused at once (64 q queries fit one launch of this server
        # only with 2 splits, 40 bytes per query: more than the 2.5 requests of q queries leave room for)
        with pytest.raises(PtsError) as e:
            S.submit_eval(c, _x(64 * q))
        assert e.value.code == binding.PTS_EBUDGET
        with pytest.raises(PtsError) as e:
            S.add_cloud(*_cloud(1 << 20))
        assert e.value.code == binding.PTS_EBUDGET
        assert S.stats()["rejected"] >= 1


def test_slots_limit_and_overlap():
    with Server(budget_bytes=64 << 20, mock=True, max_inflight=3, max_batch_work=4096,
                mock_pairs_per_s=1e8) as S:
        c = S.add_cloud(*_cloud(2000))
        ts = []
        peak = 0
        for i in range(12):  # a stream of arrivals while launches run
            ts.append(S.submit_eval(c, _x(500 + 37 * i)))
            peak = max(peak, S.stats()["inflight"])
            time.sleep(0.002)

        def check(st, states):
            nonlocal peak
            assert st["inflight"] <= 3
            peak = max(peak, st["inflight"])

        _sample_until_done(S, ts, check)
        for i, t in enumerate(ts):
            np.testing.assert_allclose(S.wait(t), _pattern(c, 500 + 37 * i), rtol=1e-6)
        st = S.stats()
        assert peak == 3
        assert st["overlapped_launches"] > 0    # a second launch was issued while one was in flight
        assert st["completed"] == 12


def test_cancel_and_failure_isolation():
    with Server(budget_bytes=64 << 20, mock=True, max_inflight=1, max_batch_work=4096, mock_pairs_per_s=1e8,
                mock_fail_count=77) as S:
        c = S.add_cloud(*_cloud(1000))
        run = S.submit_eval(c, _x(5000))      # 50 ms
        queued = S.submit_eval(c, _x(10))
        bad = S.submit_eval(c, _x(77))
        good = S.submit_eval(c, _x(11))
        for _ in range(1000):
            if S.poll(run) == "running":
                break
            time.sleep(0.001)
        assert S.poll(queued) == "queued"
        S.cancel(queued)
        assert S.poll(queued) == "cancelled"
        S.cancel(run)
        with pytest.raises(PtsError) as e:
            S.wait(queued)
        assert e.value.code == binding.PTS_ECANCELLED
        with pytest.raises(PtsError) as e:
            S.wait(run)
        assert e.value.code == binding.PTS_ECANCELLED
        with pytest.raises(PtsError) as e:
            S.wait(bad)
        assert e.value.code == binding.PTS_EHIP
        np.testing.assert_allclose(S.wait(good), _pattern(c, 11), rtol=1e-6)
        st = S.stats()
        assert st["cancelled"] == 2 and st["failed"] == 1 and st["completed"] == 1


def test_errors_and_cloud_lifecycle():
    with Server(budget_bytes=64 << 20, mock=True, max_batch_work=64, mock_pairs_per_s=1e8) as S:
        c = S.add_cloud(*_cloud(3000))
        assert S.cloud_plan(c) == (3000, 2)
        with pytest.raises(PtsError) as e:
            S.submit_eval(c + 100, _x(5))
        assert e.value.code == binding.PTS_ENOTFOUND
        # more workgroups than one launch holds: spread over launches of at most 64 workgroups
        big = S.submit_eval(c, _x(64 * 512))
        n0 = S.stats()["launches"]
        np.testing.assert_allclose(S.wait(big), _pattern(c, 64 * 512), rtol=1e-6)
        assert S.stats()["launches"] - n0 >= 64 * 2 // 64
        with pytest.raises(PtsError) as e:
            S.submit_trace(c, _x(4), _x(4), steps=-1, eps=1e-3, tmax=1.0)
        assert e.value.code == binding.PTS_EINVAL
        t = S.submit_eval(c, _x(3000))          # 90 ms
        with pytest.raises(PtsError) as e:
            S.remove_cloud(c)
        assert e.value.code == binding.PTS_EBUSY
        with pytest.raises(PtsError) as e:
            S.wait(t, timeout_ms=1)
        assert e.value.code == binding.PTS_ETIMEOUT
        S.wait(t)
        S.remove_cloud(c)
        with pytest.raises(PtsError) as e:
            S.submit_eval(c, _x(5))
        assert e.value.code == binding.PTS_ENOTFOUND
        assert S.stats()["bytes_resident"] == 0
        # ids are not reused
        c2 = S.add_cloud(*_cloud(10))
        assert c2 != c
        assert S.cloud_plan(c2) == (10, 1)
    # one block of a trace on a cloud split 8 ways needs 8 workgroups: a 2-workgroup launch cannot hold
    # it (a query request falls back to a split that fits)
    with Server(budget_bytes=64 << 20, mock=True, max_batch_work=2, mock_pairs_per_s=1e8) as S:
        c = S.add_cloud(*_cloud(9000))
        assert S.cloud_plan(c) == (9000, 8)
        with pytest.raises(PtsError) as e:
            S.submit_trace(c, _x(4), np.ones((4, 3), np.float32), steps=2, eps=1e-3, tmax=1.0)
        assert e.value.code == binding.PTS_EINVAL
        np.testing.assert_allclose(S.wait(S.submit_eval(c, _x(5))), _pattern(c, 5), rtol=1e-6)


def test_close_cancels_waiters():
    S = Server(budget_bytes=64 << 20, mock=True, max_inflight=1, max_batch_work=4096, mock_pairs_per_s=1e7)
    c = S.add_cloud(*_cloud(1000))
    ts = [S.submit_eval(c, _x(2000)) for _ in range(4)]   # 200 ms each
    codes = []

    def waiter(t):
        try:
            S.wait(t)
            codes.append(binding.PTS_OK)
        except PtsError as e:
            codes.append(e.code)

    th = [threading.Thread(target=waiter, args=(t,)) for t in ts]
    for x in th:
        x.start()
    time.sleep(0.05)
    S.close()
    for x in th:
        x.join(10)
    assert sorted(codes) == [binding.PTS_ECANCELLED] * 4
    with pytest.raises(RuntimeError):
        S.submit_eval(c, _x(1))


def test_many_clients_many_clouds():
    """Several client threads submitting to many clouds; every result lands in its own request."""
    with Server(budget_bytes=256 << 20, mock=True, max_inflight=16, max_batch_work=8192,
                mock_pairs_per_s=5e10) as S:
        rng = np.random.default_rng(5)
        clouds = [S.add_cloud(*_cloud(int(N))) for N in rng.integers(512, 20000, 12)]
        errors = []

        def client(k):
            r = np.random.default_rng(100 + k)
            for _ in range(15):
                cid = clouds[int(r.integers(len(clouds)))]
                q = int(r.integers(0, 3000))
                try:
                    out = S.wait(S.submit_eval(cid, _x(q)))
                    np.testing.assert_allclose(out, _pattern(cid, q), rtol=1e-6)
                except Exception as e:  # noqa: BLE001 -- collected and re-raised below
                    errors.append(e)

        th = [threading.Thread(target=client, args=(k,)) for k in range(6)]
        for x in th:
            x.start()
        for x in th:
            x.join(60)
        assert not errors, errors[0]
        st = S.stats()
        assert st["completed"] == 90 and st["inflight"] == 0 and st["queued"] == 0
        assert st["bytes_inflight"] == 0


def test_quantum_spreads_long_requests_and_lets_short_ones_pass():
    """A launch takes at most quantum_pairs of work, except that one launch in flight may run a long
    request whole while it is the only runnable one: two long query requests are spread over launches
    of about one quantum each, and a short request submitted behind both finishes within a few quanta;
    every result lands in its own request whichever chunks carried it."""
    N, big = 4000, 65536                       # 128 blocks of 512 queries, 2.6e8 pairs
    quantum = 512 * N * 8                      # 8 blocks per launch
    rate = quantum / 0.02                      # 20 ms per full launch
    with Server(budget_bytes=256 << 20, mock=True, max_batch_work=1 << 16, mock_pairs_per_s=rate,
                quantum_pairs=quantum) as S:
        c = S.add_cloud(*_cloud(N))
        t_big1, t_big2 = S.submit_eval(c, _x(big)), S.submit_eval(c, _x(big))
        time.sleep(0.005)
        t0 = time.time()
        t_small = S.submit_eval(c, _x(100))
        np.testing.assert_allclose(S.wait(t_small), _pattern(c, 100), rtol=1e-6)
        small_s = time.time() - t0
        assert S.poll(t_big1) == "running" and S.poll(t_big2) == "running"
        for t in (t_big1, t_big2):
            np.testing.assert_allclose(S.wait(t), _pattern(c, big), rtol=1e-6)
        big_s = time.time() - t0
        st = S.stats()
        assert st["launches"] >= 1 + 128 // 8            # at most one whole, the rest in quanta
        assert small_s < 0.1 < big_s, (small_s, big_s)   # a few quanta against ~16
        # a trace step of many rays behind a whole launch: chunked, results intact
        t_big3 = S.submit_eval(c, _x(big))
        tr = S.submit_trace(c, _x(40000), np.ones((40000, 3), np.float32), steps=5, eps=1e-3, tmax=5.0)
        r = S.wait(tr)
        assert np.all(r["t"] == c) and np.array_equal(r["hit"], np.arange(40000) % 2)
        assert np.all(r["steps"] == 3)
        S.wait(t_big3)
    with pytest.raises(PtsError):
        Server(mock=True, quantum_pairs=-1.0)
