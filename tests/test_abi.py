"""The C-ABI library loads on a CPU-only host and exports every symbol include/pts.h declares.

Only host-side paths are exercised here (argument checks that return before
any HIP call); compute calls need a GPU and live in the gpu-marked tests.
"""

import ctypes
import os
import re

import pytest

from paper_2607_16946_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pts_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    return binding.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared("pts.h")
    assert "pts_eval" in names and "pts_cloud_build" in names
    for name in names:
        assert hasattr(L, name), name
    # and the binding describes exactly those entry points
    assert set(binding.SIGNATURES) == set(names)


def test_version_and_sizes(L):
    assert binding.version() >= 100
    nb = binding.record_bytes(4096)
    assert nb % 256 == 0 and nb >= 4096 * (16 + 80 + 4)
    assert binding.eval_ws_bytes(4096, 0) == 0
    assert binding.eval_ws_bytes(131072, 128 ** 3) >= 128 ** 3 * 12


def test_host_side_errors(L):
    out = ctypes.c_size_t(0)
    assert L.pts_record_bytes(0, ctypes.byref(out)) == binding.PTS_EINVAL
    assert b"N must be" in L.pts_last_error()
    prm = binding.make_params()
    # Q = 0 is a no-op, before any device work
    assert L.pts_eval(None, 10, None, 0, None, None, None, ctypes.byref(prm), None, 0, None) == binding.PTS_OK
    assert L.pts_eval(None, 0, None, 5, None, None, None, ctypes.byref(prm), None, 0, None) == binding.PTS_EINVAL
    assert L.pts_eval(None, 10, None, 5, None, None, None, ctypes.byref(prm), None, 0, None) == binding.PTS_EINVAL
    bad = binding.make_params(C=100.0)
    assert L.pts_eval_ws_bytes(10, 10, ctypes.byref(bad), ctypes.byref(out)) == binding.PTS_EINVAL
    bad = binding.make_params(splits=3)
    assert L.pts_eval_ws_bytes(10, 10, ctypes.byref(bad), ctypes.byref(out)) == binding.PTS_EINVAL
    assert L.pts_cloud_build(None, None, None, 10, None, None, 0, None) == binding.PTS_EINVAL
    # compositions: unknown op, a two-operand op without b, n < 0
    assert L.pts_compose(None, None, 4, 9, 0.0, None, None) == binding.PTS_EINVAL
    assert L.pts_compose(ctypes.c_void_p(16), None, 4, 1, 0.0, ctypes.c_void_p(16), None) == binding.PTS_EINVAL
    assert L.pts_compose(None, None, 0, 1, 0.0, None, None) == binding.PTS_OK
    # a non-finite offset is refused before any device work
    bad = binding.make_params(offset=float("nan"))
    assert L.pts_eval_ws_bytes(10, 10, ctypes.byref(bad), ctypes.byref(out)) == binding.PTS_EINVAL
    # the point backward needs at least one output, and its workspace covers every combination
    assert L.pts_backward_points(None, 10, None, None, None, None, 5, None, None, None, None, None,
                                 ctypes.byref(prm), None, 0, None) == binding.PTS_EINVAL
    assert b"no output" in L.pts_last_error()
    wa, wp = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.pts_backward_ws_bytes(5000, 3000, ctypes.byref(prm), ctypes.byref(wa)) == binding.PTS_OK
    assert L.pts_backward_points_ws_bytes(5000, 3000, ctypes.byref(prm), ctypes.byref(wp)) == binding.PTS_OK
    assert wp.value >= wa.value * 12 // 8 + 3000 * (4 + 4 + 48)


def test_bounded_trace_host_checks(L):
    # argument checks before any device work, and a workspace that covers the
    # bounded evaluation at every number of rays still marching (its point
    # splits grow as the active set shrinks)
    prm = binding.make_params()
    args = (None, 1000, None, None, 5, 8, 1e-3, 1.0)
    tail = (None, None, None, None, ctypes.byref(prm), None, 0, None)
    assert L.pts_trace_bounded(*args, -1.0, *tail) == binding.PTS_EINVAL
    assert b"eval_eps" in L.pts_last_error()
    assert L.pts_trace_bounded(*args, float("inf"), *tail) == binding.PTS_EINVAL
    assert L.pts_trace_bounded(None, 1000, None, None, 0, 8, 1e-3, 1.0, 0.0, *tail) == binding.PTS_OK
    out, q = ctypes.c_size_t(0), ctypes.c_size_t(0)
    for N, R in ((4096, 5000), (131072, 70000), (1 << 20, 1 << 20)):
        assert L.pts_trace_bounded_ws_bytes(N, R, ctypes.byref(prm), ctypes.byref(out)) == binding.PTS_OK
        for Q in sorted({1, 63, 64, 65, 4095, 4096, 8191, 65536, 65535 * 2, R // 3, R - 1, R} - {0}):
            if Q > R:
                continue
            assert L.pts_eval_bounded_ws_bytes(N, Q, ctypes.byref(prm), ctypes.byref(q)) == binding.PTS_OK
            assert out.value >= q.value, (N, R, Q)


def test_parameter_ranges(L):
    """C in (0, 75] (the weights' FP32 range with the shift min(C, 64)); kfloor_rel >= 1e-12."""
    out = ctypes.c_size_t(0)
    for C, ok in ((75.0, True), (64.0, True), (0.5, True), (75.5, False), (87.0, False), (-1.0, False)):
        prm = binding.make_params(C=C)
        rc = L.pts_eval_ws_bytes(10, 10, ctypes.byref(prm), ctypes.byref(out))
        assert (rc == binding.PTS_OK) == ok, C
    for kf, ok in ((1e-12, True), (1e-6, True), (1e-13, False), (float("inf"), False)):
        prm = binding.make_params(kfloor_rel=kf)
        rc = L.pts_eval_ws_bytes(10, 10, ctypes.byref(prm), ctypes.byref(out))
        assert (rc == binding.PTS_OK) == ok, kf
    cfg = binding.ServerCfg()
    cfg.mock = 1
    cfg.C = 80.0
    srv = ctypes.c_void_p()
    assert L.pts_server_create(ctypes.byref(cfg), ctypes.byref(srv)) == binding.PTS_EINVAL
    cfg.C = 0.0
    cfg.kfloor_rel = 1e-13
    assert L.pts_server_create(ctypes.byref(cfg), ctypes.byref(srv)) == binding.PTS_EINVAL


def test_noalloc_refuses_a_workspace_beyond_its_static_scratch(L):
    # checked on the host before any device call: 2^22 queries with 8 splits need 512 MiB > 64 MiB
    prm = binding.make_params()
    fake = ctypes.c_void_p(256)
    rc = L.pts_eval_noalloc(fake, 1 << 17, fake, 1 << 22, fake, ctypes.byref(prm), None)
    assert rc == binding.PTS_EINVAL
    assert b"static scratch" in L.pts_last_error()
    assert L.pts_eval_noalloc(None, 10, None, 0, None, ctypes.byref(prm), None) == binding.PTS_OK
    assert L.pts_eval_noalloc(None, 10, None, 5, None, ctypes.byref(prm), None) == binding.PTS_EINVAL


def test_probe_library_exports():
    path = os.path.join(ROOT, "paper_2607_16946_amd", "libpts_probe.so")
    P = ctypes.CDLL(path)
    P.ptsprobe_instr_per_lane.restype = ctypes.c_longlong
    assert P.ptsprobe_instr_per_lane(0, 10) == 10 * 4 * 8
    assert P.ptsprobe_instr_per_lane(5, 10) == 10 * 4 * 8 * 5


def test_plan_covers_every_point():
    rng = __import__("numpy").random.default_rng(0)
    Ns = [1, 2, 511, 512, 513, 4096, 5000, 8192, 20000, 131072, 262144, 1 << 20] + list(rng.integers(1, 3_000_000, 40))
    Qs = [1, 7, 1000, 1728, 4096, 70001, 128 ** 3, 1 << 20]
    for N in Ns:
        for Q in Qs:
            for S in (0, 1, 2, 8, 32, 64):
                qpl, splits, per = binding.eval_plan(int(N), Q, binding.make_params(splits=S))
                assert qpl in (1, 2, 4)
                assert per % 64 == 0 and per > 0
                assert splits >= 1 and splits * per >= N, (N, Q, S, splits, per)
                assert (splits - 1) * per < N, (N, Q, S, splits, per)     # no empty split
                assert splits <= (S if S else 1024)


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes structures have the sizes and field offsets gcc gives the C structs."""
    structs = {"pts_params": binding.Params, "pts_cloud_info": binding.CloudInfo,
               "pts_server_cfg": binding.ServerCfg, "pts_request": binding.Request,
               "pts_server_stats": binding.ServerStats, "pts_radius_info": binding.RadiusInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pts.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
