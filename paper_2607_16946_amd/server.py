"""Python face of the serving engine (``pts_server_*`` in include/pts.h).

Marshalling only: the scheduler, admission, packing and every kernel live in
libpts.  Requests take host (numpy) arrays; the server copies inputs at submit
and writes outputs before it reports a request finished.  This wrapper keeps
each request's output arrays alive until ``wait`` has returned for it.
"""

from __future__ import annotations

import ctypes
import threading

import numpy as np

from . import binding
from .binding import PtsError, PTS_OK, PTS_REQ_EVAL, PTS_REQ_TRACE, ServerCfg, ServerStats, Request


def _host(a, name, cols, dtype=np.float32):
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.ndim != 2 or a.shape[1] != cols:
        raise ValueError(f"{name} must have shape [n, {cols}], got {a.shape}")
    return a


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


class Ticket:
    """A submitted request: its id and the arrays its results land in."""

    def __init__(self, tid: int, kind: int, outputs: dict):
        self.id = tid
        self.kind = kind
        self.outputs = outputs

    def result(self):
        return self.outputs["sdf"] if self.kind == PTS_REQ_EVAL else self.outputs


class Server:
    """Resident-cloud SDF server with continuous batching.

    Parameters mirror ``pts_server_cfg``; ``mock=True`` runs the scheduler
    without a device (a cost model stands in for the kernels).  Consecutive
    packed launches overlap on the device only if HIP gives the server's two
    launch streams different hardware queues: start the process with
    ``GPU_MAX_HW_QUEUES=8`` (or more) when it creates other streams too.
    """

    def __init__(self, budget_bytes: int = 4 << 30, max_inflight: int = 64, max_queue: int = 0,
                 max_batch_work: int = 0, C: float = 64.0, kfloor_rel: float = 1e-6, mock: bool = False,
                 mock_fail_count: int = 0, mock_pairs_per_s: float = 0.0, quantum_pairs: float = 0.0):
        self._L = binding.lib()
        cfg = ServerCfg(int(budget_bytes), int(max_inflight), int(max_queue), int(max_batch_work), float(C),
                        float(kfloor_rel), int(bool(mock)), int(mock_fail_count), float(mock_pairs_per_s),
                        float(quantum_pairs))
        h = ctypes.c_void_p()
        self._rc(self._L.pts_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._live: dict[int, Ticket] = {}
        self._cond = threading.Condition()
        self._waiters = 0

    # -- plumbing
    def _rc(self, rc):
        if rc != PTS_OK:
            raise PtsError(rc, self._L.pts_last_error().decode(errors="replace"))

    def _handle(self):
        if self._h is None:
            raise RuntimeError("server is closed")
        return self._h

    # -- clouds
    def add_cloud(self, p, n, a) -> int:
        p, n, a = _host(p, "p", 3), _host(n, "n", 3), _host(a, "a", 6)
        if not (len(p) == len(n) == len(a)):
            raise ValueError("p, n, a must have the same length")
        cid = ctypes.c_int(0)
        self._rc(self._L.pts_server_add_cloud(self._handle(), _ptr(p), _ptr(n), _ptr(a), len(p), ctypes.byref(cid)))
        return int(cid.value)

    def cloud_plan(self, cid: int) -> tuple[int, int]:
        """(N, splits): pts_eval with params.splits = splits gives the server's query results bit for bit
        (trace requests match pts_trace with default splits)."""
        N, S = ctypes.c_int64(0), ctypes.c_int(0)
        self._rc(self._L.pts_server_cloud_plan(self._handle(), int(cid), ctypes.byref(N), ctypes.byref(S)))
        return int(N.value), int(S.value)

    def remove_cloud(self, cid: int) -> None:
        self._rc(self._L.pts_server_remove_cloud(self._handle(), int(cid)))

    # -- requests
    def _submit(self, req: Request, kind: int, outputs: dict) -> Ticket:
        tid = ctypes.c_uint64(0)
        with self._cond:  # the ticket must be registered before anyone can wait on it
            self._rc(self._L.pts_server_submit(self._handle(), ctypes.byref(req), ctypes.byref(tid)))
            t = Ticket(int(tid.value), kind, outputs)
            self._live[t.id] = t
        return t

    def submit_eval(self, cloud: int, x) -> Ticket:
        x = _host(np.asarray(x).reshape(-1, 3), "x", 3)
        out = np.empty(len(x), np.float32)
        req = Request(PTS_REQ_EVAL, int(cloud), len(x), _ptr(x), None, _ptr(out), None, None, None, 0, 0.0, 0.0, 0)
        return self._submit(req, PTS_REQ_EVAL, {"sdf": out})

    def submit_trace(self, cloud: int, origin, direction, steps: int, eps: float, tmax: float,
                     normals: bool = True) -> Ticket:
        o = _host(origin, "origin", 3)
        d = _host(direction, "direction", 3)
        if len(o) != len(d):
            raise ValueError("origin and direction must have the same length")
        R = len(o)
        outs = {"t": np.empty(R, np.float32), "hit": np.empty(R, np.int32), "steps": np.empty(R, np.int32),
                "normal": np.empty((R, 3), np.float32) if normals else None}
        req = Request(PTS_REQ_TRACE, int(cloud), R, _ptr(o), _ptr(d), _ptr(outs["t"]), _ptr(outs["normal"]),
                      _ptr(outs["hit"]), _ptr(outs["steps"]), int(steps), float(eps), float(tmax), 0)
        return self._submit(req, PTS_REQ_TRACE, outs)

    def poll(self, t: Ticket) -> str:
        st = ctypes.c_int(0)
        self._rc(self._L.pts_server_poll(self._handle(), t.id, ctypes.byref(st)))
        return binding.STATE_NAMES[int(st.value)]

    def wait(self, t: Ticket, timeout_ms: int = -1):
        """Block until t finishes; return its result (raises PtsError if it failed or was cancelled).

        A timeout raises PtsError(PTS_ETIMEOUT) and leaves the request running."""
        with self._cond:  # close() destroys the server only once no waiter is inside it
            h = self._handle()
            self._waiters += 1
        rc = -1
        try:
            rc = self._L.pts_server_wait(h, t.id, int(timeout_ms))
            msg = self._L.pts_last_error().decode(errors="replace") if rc != PTS_OK else ""
            if rc != binding.PTS_ETIMEOUT:
                self._L.pts_server_release(h, t.id)
        finally:
            with self._cond:
                self._waiters -= 1
                if rc != binding.PTS_ETIMEOUT:
                    self._live.pop(t.id, None)
                self._cond.notify_all()
        if rc != PTS_OK:
            raise PtsError(rc, msg)
        return t.result()

    def cancel(self, t: Ticket) -> None:
        self._rc(self._L.pts_server_cancel(self._handle(), t.id))

    def stats(self) -> dict:
        s = ServerStats()
        self._rc(self._L.pts_server_stats_get(self._handle(), ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def reset_stats(self) -> None:
        self._rc(self._L.pts_server_stats_reset(self._handle()))

    def close(self) -> None:
        """Destroy the server; unfinished requests end cancelled (waiters get PTS_ECANCELLED)."""
        with self._cond:
            if self._h is None:
                return
            h = self._h
            live = list(self._live.values())
        for t in live:
            self._L.pts_server_cancel(h, t.id)
        with self._cond:
            self._cond.wait_for(lambda: self._waiters == 0)
            self._h = None
            self._live.clear()
        self._L.pts_server_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
