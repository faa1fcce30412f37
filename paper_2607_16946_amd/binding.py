"""ctypes binding of libpts (include/pts.h): argument marshalling only.

Every function here checks tensor placement/dtype/shape, passes raw device
pointers and the current HIP stream to the C ABI, and raises ``PtsError`` on a
non-zero status.  All arithmetic runs in the library's HIP kernels; if the
library is not built this module raises instead of falling back to anything.
"""

from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpts.so")

PTS_OK = 0
PTS_EINVAL = 1
PTS_EBUDGET = 2
PTS_ENOMEM = 3
PTS_EHIP = 4
PTS_EBUSY = 5
PTS_ECANCELLED = 6
PTS_ENOTFOUND = 7
PTS_ETIMEOUT = 8


class PtsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pts error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("C", ctypes.c_float), ("kfloor_rel", ctypes.c_float), ("splits", ctypes.c_int),
                ("offset", ctypes.c_float)]


class CloudInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("n_direct", ctypes.c_int64), ("n_anchored", ctypes.c_int64),
                ("bbox_lo", ctypes.c_float * 3), ("bbox_hi", ctypes.c_float * 3), ("diag", ctypes.c_float),
                ("kfloor", ctypes.c_float), ("version", ctypes.c_int), ("reserved", ctypes.c_int)]


class RadiusInfo(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("lam", ctypes.c_float), ("reval", ctypes.c_float),
                ("ready", ctypes.c_int), ("reserved", ctypes.c_int)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int), ("max_queue", ctypes.c_int),
                ("max_batch_work", ctypes.c_int64), ("C", ctypes.c_float), ("kfloor_rel", ctypes.c_float),
                ("mock", ctypes.c_int), ("mock_fail_count", ctypes.c_int), ("mock_pairs_per_s", ctypes.c_double),
                ("quantum_pairs", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("cloud", ctypes.c_int), ("count", ctypes.c_int64),
                ("in0", ctypes.c_void_p), ("in1", ctypes.c_void_p), ("out_sdf", ctypes.c_void_p),
                ("out_normal", ctypes.c_void_p), ("out_hit", ctypes.c_void_p), ("out_steps", ctypes.c_void_p),
                ("steps", ctypes.c_int), ("eps", ctypes.c_float), ("tmax", ctypes.c_float), ("reserved", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "failed", "cancelled", "rejected",
                                              "launches", "overlapped_launches")] + \
               [("max_batch_requests", ctypes.c_int64)] + \
               [(k, ctypes.c_double) for k in ("pairs", "busy_s", "p50_ms", "p99_ms", "max_ms", "p50_eval_ms",
                                              "p99_eval_ms", "p50_trace_ms", "p99_trace_ms")] + \
               [(k, ctypes.c_size_t) for k in ("bytes_resident", "bytes_inflight", "bytes_reserved")] + \
               [("inflight", ctypes.c_int), ("queued", ctypes.c_int)]


PTS_REQ_EVAL = 0
PTS_REQ_TRACE = 1
STATE_NAMES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}

_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

# name -> (restype, argtypes); the list of symbols include/pts.h declares.
SIGNATURES = {
    "pts_version": (ctypes.c_int, []),
    "pts_last_error": (ctypes.c_char_p, []),
    "pts_record_bytes": (ctypes.c_int, [_I64, ctypes.POINTER(_SZ)]),
    "pts_cloud_build": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_cloud_info_get": (ctypes.c_int, [_P, ctypes.POINTER(CloudInfo), _P]),
    "pts_cloud_decode": (ctypes.c_int, [_P, _I64, _P, _P]),
    "pts_eval_plan": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_I64)]),
    "pts_eval_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(_SZ)]),
    "pts_eval": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _P, _P, ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_eval_noalloc": (ctypes.c_int, [_P, _I64, _P, _I64, _P, ctypes.POINTER(Params), _P]),
    "pts_eval_far": (ctypes.c_int, [_P, _I64, _P, _I64, ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_eval_blend": (ctypes.c_int, [_P, _I64, _P, _I64, ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_eval_combine": (ctypes.c_int, [_I64, _I64, _P, ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_eval_bounded_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(_SZ)]),
    "pts_eval_bounded": (ctypes.c_int, [_P, _I64, _P, _I64, ctypes.c_float, _P, _P, _P, ctypes.POINTER(Params), _P,
                                        _SZ, _P]),
    "pts_compose": (ctypes.c_int, [_P, _P, _I64, ctypes.c_int, ctypes.c_float, _P, _P]),
    "pts_set_areas": (ctypes.c_int, [_P, _I64, _P, _P]),
    "pts_eval_baseline": (ctypes.c_int, [_P, _I64, _P, _I64, ctypes.c_int, _P, ctypes.POINTER(Params), _P, _SZ,
                                         _P]),
    "pts_grad_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(_SZ)]),
    "pts_grad_x": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _P, _P, ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_laplacian_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(_SZ)]),
    "pts_laplacian": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _P, _P, _P, ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_backward_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(_SZ)]),
    "pts_backward_params": (ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _I64, _P, _P, _P, ctypes.POINTER(Params), _P,
                                           _SZ, _P]),
    "pts_backward_points_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(_SZ)]),
    "pts_backward_points": (ctypes.c_int, [_P, _I64, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P,
                                           ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_trace_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(_SZ)]),
    "pts_trace_bounded_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(Params), ctypes.POINTER(_SZ)]),
    "pts_trace": (ctypes.c_int, [_P, _I64, _P, _P, _I64, ctypes.c_int, ctypes.c_float, ctypes.c_float, _P, _P, _P, _P,
                                 ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_trace_bounded": (ctypes.c_int, [_P, _I64, _P, _P, _I64, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, _P, _P, _P, _P, ctypes.POINTER(Params), _P, _SZ, _P]),
    "pts_radius_prepare": (ctypes.c_int, [_P, _I64, ctypes.POINTER(Params), _P]),
    "pts_radius_info_get": (ctypes.c_int, [_P, ctypes.POINTER(RadiusInfo), _P]),
    "pts_eval_radius_ws_bytes": (ctypes.c_int, [_I64, _I64, ctypes.POINTER(_SZ)]),
    "pts_eval_radius": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _P, _P, _SZ, _P]),
    "pts_server_create": (ctypes.c_int, [ctypes.POINTER(ServerCfg), ctypes.POINTER(_P)]),
    "pts_server_add_cloud": (ctypes.c_int, [_P, _P, _P, _P, _I64, ctypes.POINTER(ctypes.c_int)]),
    "pts_server_cloud_plan": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_int)]),
    "pts_server_remove_cloud": (ctypes.c_int, [_P, ctypes.c_int]),
    "pts_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "pts_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]),
    "pts_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int]),
    "pts_server_cancel": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "pts_server_release": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "pts_server_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(ServerStats)]),
    "pts_server_stats_reset": (ctypes.c_int, [_P]),
    "pts_server_destroy": (ctypes.c_int, [_P]),
}


def lib():
    """Load libpts.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2607_16946_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != PTS_OK:
        raise PtsError(rc, lib().pts_last_error().decode(errors="replace"))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t: torch.Tensor, name: str, cols: int | None = None, dtype=torch.float32) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.device.index != torch.cuda.current_device():
        # the library launches on the current device's current stream
        raise ValueError(f"{name} is on {t.device}, not on the current device cuda:{torch.cuda.current_device()}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError(f"{name} must have shape [n, {cols}], got {tuple(t.shape)}")
    return t


def make_params(C: float = 64.0, kfloor_rel: float = 1e-6, splits: int = 0, offset: float = 0.0) -> Params:
    """pts_params; offset: evaluators return phi - offset and tracing follows the offset surface."""
    return Params(float(C), float(kfloor_rel), int(splits), float(offset))


# ---------------------------------------------------------------------------
# Functions named after the C ABI
# ---------------------------------------------------------------------------

def version() -> int:
    return int(lib().pts_version())


def record_bytes(N: int) -> int:
    out = _SZ(0)
    _check(lib().pts_record_bytes(int(N), ctypes.byref(out)))
    return int(out.value)


def cloud_build(p: torch.Tensor, n: torch.Tensor, a: torch.Tensor, params: Params | None = None,
                rec: torch.Tensor | None = None) -> torch.Tensor:
    """Fit the tori (Algorithm 1 precomputation); returns the record buffer (uint8 tensor)."""
    _dev(p, "p", 3)
    _dev(n, "n", 3)
    _dev(a, "a", 6)
    N = p.shape[0]
    if n.shape[0] != N or a.shape[0] != N:
        raise ValueError("p, n, a must have the same number of rows")
    nb = record_bytes(N)
    if rec is None:
        rec = torch.empty(nb, dtype=torch.uint8, device=p.device)
    _dev(rec, "rec", dtype=torch.uint8)
    prm = params if params is not None else make_params()
    _check(lib().pts_cloud_build(_ptr(p), _ptr(n), _ptr(a), N, ctypes.byref(prm), _ptr(rec), rec.numel(),
                                 _stream()))
    return rec


def cloud_info(rec: torch.Tensor) -> CloudInfo:
    info = CloudInfo()
    _check(lib().pts_cloud_info_get(_ptr(rec), ctypes.byref(info), _stream()))
    return info


def cloud_decode(rec: torch.Tensor, N: int) -> torch.Tensor:
    out = torch.empty((N, 12), dtype=torch.float32, device=rec.device)
    _check(lib().pts_cloud_decode(_ptr(rec), int(N), _ptr(out), _stream()))
    return out


def eval_plan(N: int, Q: int, params: Params | None = None) -> tuple[int, int, int]:
    """(queries per lane, point splits, points per split) of pts_eval for N points, Q queries."""
    q, s, ps = ctypes.c_int(0), ctypes.c_int(0), _I64(0)
    prm = params if params is not None else make_params()
    _check(lib().pts_eval_plan(int(N), int(Q), ctypes.byref(prm), ctypes.byref(q), ctypes.byref(s), ctypes.byref(ps)))
    return q.value, s.value, ps.value


def eval_ws_bytes(N: int, Q: int, params: Params | None = None) -> int:
    out = _SZ(0)
    prm = params if params is not None else make_params()
    _check(lib().pts_eval_ws_bytes(int(N), int(Q), ctypes.byref(prm), ctypes.byref(out)))
    return int(out.value)


def grad_ws_bytes(N: int, Q: int, params: Params | None = None) -> int:
    out = _SZ(0)
    prm = params if params is not None else make_params()
    _check(lib().pts_grad_ws_bytes(int(N), int(Q), ctypes.byref(prm), ctypes.byref(out)))
    return int(out.value)


def eval(rec: torch.Tensor, N: int, x: torch.Tensor, params: Params | None = None, grad: bool = False,
         stats: bool = False, ws: torch.Tensor | None = None, out: torch.Tensor | None = None):
    """phi(x) at queries x [Q,3] (Sec. 4.2); optionally grad phi [Q,3] and (M, W, phi, e_*) [Q,6]."""
    _dev(x, "x", 3)
    Q = x.shape[0]
    prm = params if params is not None else make_params()
    sdf = out if out is not None else torch.empty(Q, dtype=torch.float32, device=x.device)
    g = torch.empty((Q, 3), dtype=torch.float32, device=x.device) if grad else None
    st = torch.empty((Q, 6), dtype=torch.float32, device=x.device) if stats else None
    need = grad_ws_bytes(N, Q, prm) if grad else eval_ws_bytes(N, Q, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
    _check(lib().pts_eval(_ptr(rec), int(N), _ptr(x), Q, _ptr(sdf), _ptr(g), _ptr(st), ctypes.byref(prm), _ptr(ws),
                          ws.numel(), _stream()))
    res = [sdf]
    if grad:
        res.append(g)
    if stats:
        res.append(st)
    return res[0] if len(res) == 1 else tuple(res)


def eval_noalloc(rec: torch.Tensor, N: int, x: torch.Tensor, params: Params | None = None,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """phi(x) at queries x [Q,3] with the library's static device scratch (no allocation by the library)."""
    _dev(x, "x", 3)
    Q = x.shape[0]
    prm = params if params is not None else make_params()
    sdf = out if out is not None else torch.empty(Q, dtype=torch.float32, device=x.device)
    _dev(sdf, "out")
    if sdf.numel() != Q:
        raise ValueError("out must have one value per query")
    _check(lib().pts_eval_noalloc(_ptr(rec), int(N), _ptr(x), Q, _ptr(sdf), ctypes.byref(prm), _stream()))
    return sdf


def eval_bounded_ws_bytes(N: int, Q: int, params: Params | None = None) -> int:
    out = _SZ(0)
    prm = params if params is not None else make_params()
    _check(lib().pts_eval_bounded_ws_bytes(int(N), int(Q), ctypes.byref(prm), ctypes.byref(out)))
    return int(out.value)


def eval_bounded(rec: torch.Tensor, N: int, x: torch.Tensor, eps: float, params: Params | None = None,
                 ws: torch.Tensor | None = None, out: torch.Tensor | None = None, bound: bool = False,
                 kept: bool = False):
    """phi at x [Q,3] with far units skipped while |change| <= eps (proven); optionally the incurred bound [Q]
    and the number of points evaluated per query [Q].  Returns sdf, or (sdf, bound, kept) with None entries."""
    _dev(x, "x", 3)
    Q = x.shape[0]
    prm = params if params is not None else make_params()
    sdf = out if out is not None else torch.empty(Q, dtype=torch.float32, device=x.device)
    bd = torch.empty(Q, dtype=torch.float32, device=x.device) if bound else None
    kp = torch.empty(Q, dtype=torch.int32, device=x.device) if kept else None
    if Q > 0:
        need = eval_bounded_ws_bytes(N, Q, prm)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
        _check(lib().pts_eval_bounded(_ptr(rec), int(N), _ptr(x), Q, float(eps), _ptr(sdf), _ptr(bd), _ptr(kp),
                                      ctypes.byref(prm), _ptr(ws), ws.numel(), _stream()))
    return (sdf, bd, kp) if (bound or kept) else sdf


COMPOSE_OPS = {"offset": 0, "union": 1, "intersect": 2, "subtract": 3}


def compose(a: torch.Tensor, b: torch.Tensor | None, op: str, c: float = 0.0,
            out: torch.Tensor | None = None) -> torch.Tensor:
    """Offsets and Booleans of signed distances, elementwise: a - c, min(a, b), max(a, b), max(a, -b)."""
    _dev(a, "a")
    n = a.numel()
    if op != "offset":
        if b is None:
            raise ValueError(f"{op} needs two operands")
        _dev(b, "b")
        if b.numel() != n:
            raise ValueError("operands must have the same length")
    res = out if out is not None else torch.empty_like(a)
    _check(lib().pts_compose(_ptr(a), _ptr(b), n, COMPOSE_OPS[op], float(c), _ptr(res), _stream()))
    return res


BASELINES = {"sspd": 0, "shc": 1}


def set_areas(rec: torch.Tensor, N: int, area: torch.Tensor | None = None) -> None:
    """Area weights A_i [N] of the baselines (caller's point order); None restores 1."""
    if area is not None:
        _dev(area, "area")
        if area.numel() != N:
            raise ValueError("area must have one value per point")
    _check(lib().pts_set_areas(_ptr(rec), int(N), _ptr(area), _stream()))


def eval_baseline(rec: torch.Tensor, N: int, x: torch.Tensor, kind: str, params: Params | None = None,
                  ws: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Smoothed signed planar distance ('sspd') or signed Hopf-Cole distance ('shc') at x [Q,3]."""
    _dev(x, "x", 3)
    Q = x.shape[0]
    prm = params if params is not None else make_params()
    sdf = out if out is not None else torch.empty(Q, dtype=torch.float32, device=x.device)
    if Q == 0:
        return sdf
    need = eval_ws_bytes(N, Q, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
    _check(lib().pts_eval_baseline(_ptr(rec), int(N), _ptr(x), Q, BASELINES[kind], _ptr(sdf), ctypes.byref(prm),
                                   _ptr(ws), ws.numel(), _stream()))
    return sdf


def grad_x(rec: torch.Tensor, N: int, x: torch.Tensor, stats: torch.Tensor, gout: torch.Tensor | None = None,
           params: Params | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """gout * grad phi(x) [Q,3] from the statistics of a previous eval at the same queries."""
    _dev(x, "x", 3)
    _dev(stats, "stats", 6)
    Q = x.shape[0]
    if gout is not None:
        _dev(gout, "gout")
        if gout.numel() != Q:
            raise ValueError("gout must have one value per query")
    prm = params if params is not None else make_params()
    gx = torch.empty((Q, 3), dtype=torch.float32, device=x.device)
    need = grad_ws_bytes(N, Q, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
    _check(lib().pts_grad_x(_ptr(rec), int(N), _ptr(x), Q, _ptr(gout), _ptr(stats), _ptr(gx), ctypes.byref(prm),
                            _ptr(ws), ws.numel(), _stream()))
    return gx


def eval_far(rec, N: int, x: torch.Tensor, params: Params, ws: torch.Tensor) -> None:
    _check(lib().pts_eval_far(_ptr(rec), int(N), _ptr(x), x.shape[0], ctypes.byref(params), _ptr(ws), ws.numel(),
                              _stream()))


def eval_blend(rec, N: int, x: torch.Tensor, params: Params, ws: torch.Tensor) -> None:
    _check(lib().pts_eval_blend(_ptr(rec), int(N), _ptr(x), x.shape[0], ctypes.byref(params), _ptr(ws),
                                ws.numel(), _stream()))


def eval_combine(N: int, Q: int, sdf: torch.Tensor, params: Params, ws: torch.Tensor) -> None:
    _check(lib().pts_eval_combine(int(N), int(Q), _ptr(sdf), ctypes.byref(params), _ptr(ws), ws.numel(), _stream()))


def laplacian_ws_bytes(N: int, Q: int, params: Params | None = None) -> int:
    out = _SZ(0)
    prm = params if params is not None else make_params()
    _check(lib().pts_laplacian_ws_bytes(int(N), int(Q), ctypes.byref(prm), ctypes.byref(out)))
    return int(out.value)


def laplacian(rec: torch.Tensor, N: int, x: torch.Tensor, stats: torch.Tensor, params: Params | None = None,
              want: str = "lge", ws: torch.Tensor | None = None):
    """(Laplacian [Q], grad phi [Q,3], eikonal residual |grad phi| - 1 [Q]) from the statistics of an eval at x;
    entries not in `want` ('l', 'g', 'e') are None."""
    _dev(x, "x", 3)
    _dev(stats, "stats", 6)
    if not want or set(want) - set("lge"):
        raise ValueError("want must be a non-empty subset of 'lge'")
    Q = x.shape[0]
    prm = params if params is not None else make_params()
    lap = torch.empty(Q, dtype=torch.float32, device=x.device) if "l" in want else None
    grad = torch.empty((Q, 3), dtype=torch.float32, device=x.device) if "g" in want else None
    eik = torch.empty(Q, dtype=torch.float32, device=x.device) if "e" in want else None
    if Q == 0:
        return lap, grad, eik
    need = laplacian_ws_bytes(N, Q, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
    _check(lib().pts_laplacian(_ptr(rec), int(N), _ptr(x), Q, _ptr(stats), _ptr(lap), _ptr(grad), _ptr(eik),
                               ctypes.byref(prm), _ptr(ws), ws.numel(), _stream()))
    return lap, grad, eik


def backward_ws_bytes(N: int, Q: int, params: Params | None = None) -> int:
    out = _SZ(0)
    prm = params if params is not None else make_params()
    _check(lib().pts_backward_ws_bytes(int(N), int(Q), ctypes.byref(prm), ctypes.byref(out)))
    return int(out.value)


def backward_params(rec: torch.Tensor, p: torch.Tensor, n: torch.Tensor, a: torch.Tensor, x: torch.Tensor,
                    stats: torch.Tensor, gout: torch.Tensor | None = None, params: Params | None = None,
                    ws: torch.Tensor | None = None) -> torch.Tensor:
    """dL/da [N,6] for L = sum_q gout_q phi(x_q), from the statistics of an eval at x."""
    _dev(p, "p", 3)
    _dev(n, "n", 3)
    _dev(a, "a", 6)
    _dev(x, "x", 3)
    _dev(stats, "stats", 6)
    N, Q = p.shape[0], x.shape[0]
    if gout is not None:
        _dev(gout, "gout")
        if gout.numel() != Q:
            raise ValueError("gout must have one value per query")
    prm = params if params is not None else make_params()
    ga = torch.empty((N, 6), dtype=torch.float32, device=p.device)
    need = backward_ws_bytes(N, Q, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=p.device)
    _check(lib().pts_backward_params(_ptr(rec), N, _ptr(p), _ptr(n), _ptr(a), _ptr(x), Q, _ptr(gout), _ptr(stats),
                                     _ptr(ga), ctypes.byref(prm), _ptr(ws), ws.numel(), _stream()))
    return ga


def backward_points_ws_bytes(N: int, Q: int, params: Params | None = None) -> int:
    out = _SZ(0)
    prm = params if params is not None else make_params()
    _check(lib().pts_backward_points_ws_bytes(int(N), int(Q), ctypes.byref(prm), ctypes.byref(out)))
    return int(out.value)


def backward_points(rec: torch.Tensor, p: torch.Tensor, n: torch.Tensor, a: torch.Tensor, x: torch.Tensor,
                    stats: torch.Tensor, gout: torch.Tensor | None = None, params: Params | None = None,
                    want: str = "apn", ws: torch.Tensor | None = None):
    """(dL/da [N,6], dL/dp [N,3], dL/dn [N,3]) for L = sum_q gout_q phi(x_q); entries not in `want` are None."""
    _dev(p, "p", 3)
    _dev(n, "n", 3)
    _dev(a, "a", 6)
    _dev(x, "x", 3)
    _dev(stats, "stats", 6)
    N, Q = p.shape[0], x.shape[0]
    if gout is not None:
        _dev(gout, "gout")
        if gout.numel() != Q:
            raise ValueError("gout must have one value per query")
    if not want or set(want) - set("apn"):
        raise ValueError("want must be a non-empty subset of 'apn'")
    prm = params if params is not None else make_params()
    ga = torch.empty((N, 6), dtype=torch.float32, device=p.device) if "a" in want else None
    gp = torch.empty((N, 3), dtype=torch.float32, device=p.device) if "p" in want else None
    gn = torch.empty((N, 3), dtype=torch.float32, device=p.device) if "n" in want else None
    need = backward_points_ws_bytes(N, Q, prm)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=p.device)
    _check(lib().pts_backward_points(_ptr(rec), N, _ptr(p), _ptr(n), _ptr(a), _ptr(x), Q, _ptr(gout), _ptr(stats),
                                     _ptr(ga), _ptr(gp), _ptr(gn), ctypes.byref(prm), _ptr(ws), ws.numel(),
                                     _stream()))
    return ga, gp, gn


def trace(rec: torch.Tensor, N: int, origin: torch.Tensor, direction: torch.Tensor, steps: int, eps: float,
          tmax: float, params: Params | None = None, normals: bool = True, ws: torch.Tensor | None = None,
          eval_eps: float | None = None):
    """Sphere tracing (Sec. 5.3): returns (t [R], hit [R] bool, steps [R] int32, normals [R,3] or None).

    With eval_eps (>= 0) every step evaluates phi with the error-bounded
    evaluation at that eps (pts_trace_bounded)."""
    _dev(origin, "origin", 3)
    _dev(direction, "direction", 3)
    R = origin.shape[0]
    if direction.shape[0] != R:
        raise ValueError("origin and direction must have the same number of rows")
    prm = params if params is not None else make_params()
    t = torch.empty(R, dtype=torch.float32, device=origin.device)
    hit = torch.empty(R, dtype=torch.int32, device=origin.device)
    ns = torch.empty(R, dtype=torch.int32, device=origin.device)
    nrm = torch.empty((R, 3), dtype=torch.float32, device=origin.device) if normals else None
    out = _SZ(0)
    if eval_eps is None:
        _check(lib().pts_trace_ws_bytes(int(N), R, ctypes.byref(prm), ctypes.byref(out)))
    else:
        _check(lib().pts_trace_bounded_ws_bytes(int(N), R, ctypes.byref(prm), ctypes.byref(out)))
    if ws is None or ws.numel() < out.value:
        ws = torch.empty(max(out.value, 256), dtype=torch.uint8, device=origin.device)
    if eval_eps is None:
        _check(lib().pts_trace(_ptr(rec), int(N), _ptr(origin), _ptr(direction), R, int(steps), float(eps),
                               float(tmax), _ptr(t), _ptr(nrm), _ptr(hit), _ptr(ns), ctypes.byref(prm), _ptr(ws),
                               ws.numel(), _stream()))
    else:
        _check(lib().pts_trace_bounded(_ptr(rec), int(N), _ptr(origin), _ptr(direction), R, int(steps), float(eps),
                                       float(tmax), float(eval_eps), _ptr(t), _ptr(nrm), _ptr(hit), _ptr(ns),
                                       ctypes.byref(prm), _ptr(ws), ws.numel(), _stream()))
    return t, hit.bool(), ns, nrm


def radius_prepare(rec: torch.Tensor, N: int, params: Params | None = None) -> None:
    """D, lambda = 1e3/D, R_eval = 2C/lambda of the radius-limited evaluation (Sec. 4.2), into the record."""
    prm = params if params is not None else make_params()
    _check(lib().pts_radius_prepare(_ptr(rec), int(N), ctypes.byref(prm), _stream()))


def radius_info(rec: torch.Tensor) -> RadiusInfo:
    out = RadiusInfo()
    _check(lib().pts_radius_info_get(_ptr(rec), ctypes.byref(out), _stream()))
    return out


def eval_radius_ws_bytes(N: int, Q: int) -> int:
    out = _SZ(0)
    _check(lib().pts_eval_radius_ws_bytes(int(N), int(Q), ctypes.byref(out)))
    return int(out.value)


def eval_radius(rec: torch.Tensor, N: int, x: torch.Tensor, count: bool = False, ws: torch.Tensor | None = None):
    """Radius-limited phi (Sec. 4.2) at x [Q,3]; with count=True also the int32 count of blended points
    (negative for the 32-nearest fallback)."""
    _dev(x, "x", 3)
    Q = x.shape[0]
    sdf = torch.empty(Q, dtype=torch.float32, device=x.device)
    cnt = torch.empty(Q, dtype=torch.int32, device=x.device) if count else None
    need = eval_radius_ws_bytes(N, Q)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
    _check(lib().pts_eval_radius(_ptr(rec), int(N), _ptr(x), Q, _ptr(sdf), _ptr(cnt), _ptr(ws), ws.numel(),
                                 _stream()))
    return (sdf, cnt) if count else sdf


class Cloud:
    """A built point cloud resident in device memory (record buffer + parameters)."""

    def __init__(self, p: torch.Tensor, n: torch.Tensor, a: torch.Tensor, C: float = 64.0,
                 kfloor_rel: float = 1e-6, splits: int = 0):
        self.params = make_params(C, kfloor_rel, splits)
        self.N = int(p.shape[0])
        self.p, self.n, self.a = p, n, a
        self.rec = cloud_build(p, n, a, self.params)
        self._ws = None

    def info(self) -> CloudInfo:
        return cloud_info(self.rec)

    def decode(self) -> torch.Tensor:
        return cloud_decode(self.rec, self.N)

    def __call__(self, x: torch.Tensor, grad: bool = False, stats: bool = False):
        need = (grad_ws_bytes if grad else eval_ws_bytes)(self.N, x.shape[0], self.params)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=x.device)
        return eval(self.rec, self.N, x, self.params, grad=grad, stats=stats, ws=self._ws)
