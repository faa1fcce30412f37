#!/usr/bin/env python3
"""Throughput of the pointwise SDF hot path on one MI355X.

Workload (one "step"): the large photogrammetry-like configuration -- a
2^20-point cloud on the union of 32 random ellipsoids / ring tori with density
varying 10x across the surface, sigma = 0.005 position noise, 3% outliers
uniform in the bounding box with random normals, and analytic coefficients,
queried at 2^20 points uniform in its bounding box padded by 10% per side.  A
step runs the whole path through the C ABI: torus fitting (pts_cloud_build),
the farthest-point sweep, the blend sweep and the split combine
(pts_eval_far / _blend / _combine).  Inputs are resident in device memory
before timing starts.

Prints one JSON line (rank 0): value = query x point SDF evaluations per
second (pairs/s), with a `roofline` object for the dominant kernel (the blend
sweep, timed with HIP events on the stream it runs on) and a `cpu_baseline`
object (the FP64 oracle on a bounded sample, on this host's cores).  Beside
it: the same workload's 1024^2 x 64-step sphere trace, the mid workload
(131,072 points, 128^3 lattice), the radius-limited, error-bounded and
baseline evaluators, the differentiation workload, serving, and every
configuration beside the oracle.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The serving leg's server overlaps consecutive packed launches on two HIP
# streams, which only overlap on the device if HIP maps them to different
# hardware queues.  With HIP's default of 4 queues per process that depends on
# how many streams the process created before the server (measured: one
# earlier stream put both launch streams on one queue, device busy 0.9 instead
# of 1.7 of wall time and p50 latency 3.5 instead of 2.0 ms at 90% load); with
# 8 it does not.  Must be set before HIP initialises; raised to 8 unless the
# environment already allows more.
# `--hw-queues K` sets it to K instead (the serving leg at HIP's default of 4
# runs in a child process started that way).
def _hw_queues_arg():
    for i, a in enumerate(sys.argv):
        if a == "--hw-queues" and i + 1 < len(sys.argv):
            return sys.argv[i + 1]
        if a.startswith("--hw-queues="):
            return a.split("=", 1)[1]
    return None


if _hw_queues_arg() is not None:
    os.environ["GPU_MAX_HW_QUEUES"] = str(int(_hw_queues_arg()))
else:
    try:
        _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
    except ValueError:
        _hwq = 4
    if _hwq < 8:
        os.environ["GPU_MAX_HW_QUEUES"] = "8"

METRIC = "query×point SDF evals/sec (FP32, % of VALU peak); p50/p99 latency in serving mode"

# Algorithmic work per (query, point) pair, counted from the definition
# (Eqs. BasicFormulaShifted, RelationshipBetweenLambdaAndRadius,
# SingleTorusSDF): farthest-point sweep 5 plain + 2 FMA; blend sweep 13 plain +
# 11 FMA + 4 transcendental (3 sqrt, 1 exp).  FLOPs count an FMA as 2.
BLEND_PLAIN, BLEND_FMA, BLEND_TRANS = 13, 11, 4
BLEND_FLOP = BLEND_PLAIN + 2 * BLEND_FMA + BLEND_TRANS      # 39
FAR_FLOP = 5 + 2 * 2                                         # 9

# MI355X VALU unit counts at the 2.4 GHz peak engine clock (256 CUs):
#  - FP32 add/mul/FMA: 128 lanes/clk/CU (two VALU issue ports per SIMD fed by
#    different waves; the published 157.3 TFLOP/s FP32 vector peak);
#  - transcendentals (sqrt, exp2, rcp): 32 lanes/clk/CU (a quarter of that);
#  - the two share issue cycles (measured: in mixes their costs add).
CUS, CLOCK_HZ = 256, 2.4e9
ARITH_LANES_PER_CLK, TRANS_LANES_PER_CLK = 128, 32
PUBLISHED_FP32_TFLOPS = 157.3
# CU-cycles per blend pair at that peak, and the resulting pairs/s and FLOP/s
BLEND_CYCLES = (BLEND_PLAIN + BLEND_FMA) / ARITH_LANES_PER_CLK + BLEND_TRANS / TRANS_LANES_PER_CLK
PEAK_PAIRS = CUS * CLOCK_HZ / BLEND_CYCLES                   # 1.97e12 pairs/s
PEAK_TFLOPS = BLEND_FLOP * PEAK_PAIRS / 1e12                 # 76.7 TFLOP/s
TRAFFIC_FILES = {w: os.path.join(ROOT, "profiles", f"k_blend_{w}_traffic.json") for w in ("large", "mid")}


def measured_traffic(workload: str):
    """HBM bytes per k_blend launch on a workload from the committed counter
    summary, if it was taken on the current kernel source (else None)."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILES[workload]))
    except (OSError, ValueError, KeyError):
        return None
    src = os.path.join(ROOT, "paper_2607_16946_amd", "csrc", "pts_eval.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("pts_eval_sha256") != h:
        return None
    return {"bytes_per_launch": rec.get("bytes_per_launch"), "over_algorithmic": rec.get("over_algorithmic")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROBES = ((0, "fma_vop3_sgpr", 8192), (1, "exp", 2048), (2, "sqrt", 2048), (3, "rcp", 2048), (4, "max3", 8192),
          (5, "exp_then_4fma", 1024), (6, "fmac_vop2", 8192), (7, "fma_vop3", 8192), (8, "add_vop2", 8192),
          (9, "mul_vop2", 8192), (10, "exp_par_3fmac", 4096), (11, "sqrt_par_3fmac", 4096),
          (12, "max_vop2", 8192), (13, "exp_par_7fmac", 4096), (14, "exp_par_14fmac", 2048), (15, "sub_vop2", 8192))


def probe_issue_rates():
    """Sustained lane-instructions/s of the VALU forms the kernels use, and the shader clock."""
    import torch
    path = os.path.join(ROOT, "paper_2607_16946_amd", "libpts_probe.so")
    P = ctypes.CDLL(path)
    P.ptsprobe_run.restype = ctypes.c_int
    P.ptsprobe_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_float)]
    P.ptsprobe_instr_per_lane.restype = ctypes.c_longlong
    P.ptsprobe_instr_per_lane.argtypes = [ctypes.c_int, ctypes.c_int]
    blocks = CUS * 8
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    clk = torch.zeros(2, dtype=torch.int64, device="cuda")
    rates, clocks = {}, {}
    for op, name, iters in PROBES:
        best = None
        for _ in range(3):
            ms = ctypes.c_float(0)
            rc = P.ptsprobe_run(op, blocks, iters, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(clk.data_ptr()),
                                ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"probe {name} failed: {rc}")
            best = ms.value if best is None else min(best, ms.value)
        n = P.ptsprobe_instr_per_lane(op, iters) * blocks * 256
        rates[name] = n / (best * 1e-3)
        ticks = clk.cpu().tolist()
        if ticks[1] > 0:
            clocks[name] = ticks[0] / (ticks[1] / 100e6)
    return {"lane_instr_per_s": rates, "shader_clock_hz": clocks}


def cpu_baseline(cl, x, sample: int):
    """The FP64 oracle as it stands, on a seeded sample of the workload's queries:
    all host threads (up to 16), then one thread on a sixteenth of the sample."""
    import numpy as np
    import oracle
    threads = min(16, os.cpu_count() or 1)
    idx = np.random.default_rng(12345).choice(x.shape[0], size=min(sample, x.shape[0]), replace=False)
    xs = x[np.sort(idx)]
    t0 = time.perf_counter()
    tor = oracle.fit(cl.p, cl.n, cl.a)
    t1 = time.perf_counter()
    oracle.eval_sdf(cl.p, tor, xs, nthreads=threads)
    t2 = time.perf_counter()
    pairs = xs.shape[0] * cl.N
    x1 = xs[:max(1, xs.shape[0] // 16)]
    t3 = time.perf_counter()
    oracle.eval_sdf(cl.p, tor, x1, nthreads=1)
    t4 = time.perf_counter()
    return {"value": pairs / (t2 - t1), "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{xs.shape[0]} seeded queries of the workload's {x.shape[0]} x all {cl.N} points "
                      f"({pairs:.3g} pairs), FP64, after a {t1 - t0:.2f} s torus fit",
            "seconds": t2 - t1,
            "one_core": {"value": x1.shape[0] * cl.N / (t4 - t3), "queries": x1.shape[0], "seconds": t4 - t3}}


def configs_bench(threads: int):
    """Each configuration's plain evaluation on the GPU beside the FP64 oracle:
    GPU pairs/s (HIP events, median of 5 after a warm-up), the oracle's pairs/s
    on the timed sets (all 4096 queries of the tiny cloud, a seeded 8192-query
    subset of the others; all host threads, then one thread on a sixteenth of
    the set), and max |phi_gpu - phi_oracle| / D over the oracle's queries."""
    import numpy as np
    import torch
    import oracle
    from paper_2607_16946_amd import binding, synth
    cases = [("1 tiny", lambda: synth.tiny()), ("2 mid", lambda: synth.mid()),
             ("3 diff", lambda: synth.diff_workload()[:2]), ("5 large", lambda: synth.large())]
    out = {}
    for name, make in cases:
        cl, x = make()
        N, Q = cl.N, x.shape[0]
        p, n, a, xd = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a, x))
        prm = binding.make_params()
        rec = binding.cloud_build(p, n, a, prm)
        ws = torch.empty(max(binding.eval_ws_bytes(N, Q, prm), 256), dtype=torch.uint8, device="cuda")
        sdf = torch.empty(Q, dtype=torch.float32, device="cuda")
        ms = _timed(lambda: binding.eval(rec, N, xd, prm, ws=ws, out=sdf), 5 if N * Q > 1e9 else 50, warm=3)
        phi = sdf.cpu().numpy().astype(np.float64)
        idx = np.arange(Q) if Q <= 4096 else np.sort(np.random.default_rng(8192).choice(Q, 8192, replace=False))
        t0 = time.perf_counter()
        tor = oracle.fit(cl.p, cl.n, cl.a)
        t1 = time.perf_counter()
        ref = oracle.eval_sdf(cl.p, tor, x[idx], nthreads=threads)
        t2 = time.perf_counter()
        one = idx[:max(1, len(idx) // 16)]
        oracle.eval_sdf(cl.p, tor, x[one], nthreads=1)
        t3 = time.perf_counter()
        D = max(oracle.bbox_diag(cl.p), 1.0)
        err = np.abs(phi[idx] - ref)
        out[name] = {"N": N, "Q": Q, "gpu_ms": ms, "gpu_pairs_per_s": float(N) * Q / (ms * 1e-3),
                     "oracle_queries": int(len(idx)), "oracle_pairs_per_s": len(idx) * N / (t2 - t1),
                     "oracle_threads": threads, "oracle_one_thread_pairs_per_s": len(one) * N / (t3 - t2),
                     "oracle_fit_s": t1 - t0, "max_abs_err_over_D": float(err.max() / D),
                     "p99_abs_err_over_D": float(np.quantile(err, 0.99) / D)}
        log(f"config {name}: GPU {out[name]['gpu_pairs_per_s']:.3g} pairs/s; oracle "
            f"{out[name]['oracle_pairs_per_s']:.3g} ({threads} threads), {out[name]['oracle_one_thread_pairs_per_s']:.3g} "
            f"(1 thread); max |err|/D {out[name]['max_abs_err_over_D']:.2e}")
        del rec, ws, sdf, xd, p, n, a
        torch.cuda.empty_cache()
    return out


def _timed(fn, reps: int, warm: int = 1) -> float:
    """Median milliseconds of fn() over reps runs, bracketed by events on the current stream."""
    import numpy as np
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(s)
        fn()
        e1.record(s)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def diff_bench(reps: int):
    """Differentiation workload: one ellipsoid, N = 32768, Q = 2^20 (half within
    0.05 of the surface, half uniform in the padded bbox), loss = sum phi^2 over
    the near-surface half.  Times the plain forward, the forward with the
    statistics backward needs, the fused forward+gradient, d/dquery,
    d/dcoefficients, d/d(coefficients, points, normals) together, and the
    Laplacian sweep (with the gradient and eikonal residual), each as pairs/s
    beside the plain forward."""
    import torch
    from paper_2607_16946_amd import binding, synth
    cl, x, mask = synth.diff_workload()
    N, Q = cl.N, x.shape[0]
    p, n, a, xd = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a, x))
    md = torch.from_numpy(mask).cuda()
    prm = binding.make_params()
    rec = binding.cloud_build(p, n, a, prm)
    ws_e = torch.empty(binding.eval_ws_bytes(N, Q, prm), dtype=torch.uint8, device="cuda")
    ws_g = torch.empty(binding.grad_ws_bytes(N, Q, prm), dtype=torch.uint8, device="cuda")
    ws_b = torch.empty(binding.backward_ws_bytes(N, Q, prm), dtype=torch.uint8, device="cuda")
    ws_p = torch.empty(binding.backward_points_ws_bytes(N, Q, prm), dtype=torch.uint8, device="cuda")
    ws_l = torch.empty(binding.laplacian_ws_bytes(N, Q, prm), dtype=torch.uint8, device="cuda")
    sdf = torch.empty(Q, dtype=torch.float32, device="cuda")
    ms = {"forward": _timed(lambda: binding.eval(rec, N, xd, prm, ws=ws_e, out=sdf), reps)}
    ms["forward_stats"] = _timed(lambda: binding.eval(rec, N, xd, prm, stats=True, ws=ws_g), reps)
    ms["forward_grad"] = _timed(lambda: binding.eval(rec, N, xd, prm, grad=True, ws=ws_g), reps)
    phi, st = binding.eval(rec, N, xd, prm, stats=True, ws=ws_g)
    gout = torch.where(md, 2.0 * phi, torch.zeros_like(phi))
    ms["grad_x"] = _timed(lambda: binding.grad_x(rec, N, xd, st, gout, prm, ws_g), reps)
    ms["grad_a"] = _timed(lambda: binding.backward_params(rec, p, n, a, xd, st, gout, prm, ws_b), reps)
    ms["grad_apn"] = _timed(lambda: binding.backward_points(rec, p, n, a, xd, st, gout, prm, "apn", ws_p), reps)
    ms["laplacian"] = _timed(lambda: binding.laplacian(rec, N, xd, st, prm, "lge", ws_l), reps)
    ms["build"] = _timed(lambda: binding.cloud_build(p, n, a, prm, rec), reps)
    pairs = float(N) * Q
    out = {"workload": f"ellipsoid, N={N}, Q={Q} (half near-surface), loss = sum phi^2 over the near half",
           "N": N, "Q": Q, "ms": ms, "pairs_per_s": {k: pairs / (v * 1e-3) for k, v in ms.items() if k != "build"},
           "vs_forward": {k: ms["forward"] / v for k, v in ms.items() if k != "build"},
           "train_step_ms": ms["forward_stats"] + ms["grad_x"] + ms["grad_a"]}
    log(f"diff: forward {ms['forward']:.2f} ms, +stats {ms['forward_stats']:.2f}, fused grad "
        f"{ms['forward_grad']:.2f}, grad_x {ms['grad_x']:.2f}, grad_a {ms['grad_a']:.2f}, grad_apn "
        f"{ms['grad_apn']:.2f}, laplacian {ms['laplacian']:.2f} ms")
    return out


def baseline_bench(cl, x, reps: int = 3):
    """The two baselines of Sec. 5.2 (smoothed signed planar distance, signed
    Hopf-Cole distance; A_i = 1) on the same workload and skeleton as the
    blend: whole-evaluation throughput of each beside the blend's.  Then the
    paper's accuracy measure, mean |phi - phi_true| over a 64^3 grid (the bbox
    padded 10%), for the three methods on clouds with a closed-form SDF: the
    unit sphere (4096 points) and a ring torus R = 0.6, r = 0.25 (4096 and
    1024 points), analytic normals and coefficients."""
    import numpy as np
    import torch
    from paper_2607_16946_amd import binding, synth
    N, Q = cl.N, x.shape[0]
    p, n, a, xd = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a, x))
    prm = binding.make_params()
    rec = binding.cloud_build(p, n, a, prm)
    ws = torch.empty(binding.eval_ws_bytes(N, Q, prm), dtype=torch.uint8, device="cuda")
    sdf = torch.empty(Q, dtype=torch.float32, device="cuda")
    ms = {"torus_blend": _timed(lambda: binding.eval(rec, N, xd, prm, ws=ws, out=sdf), reps)}
    for kind in ("sspd", "shc"):
        ms[kind] = _timed(lambda: binding.eval_baseline(rec, N, xd, kind, prm, ws, sdf), reps)
    pairs = float(N) * Q
    thr = {"N": N, "Q": Q, "ms": ms, "pairs_per_s": {k: pairs / (v * 1e-3) for k, v in ms.items()}}

    def truth_sphere(q):
        return np.linalg.norm(q, axis=1) - 1.0

    def truth_torus(prim):
        def f(q):
            y = prim.local(q)
            return np.hypot(np.hypot(y[:, 0], y[:, 1]) - prim.R, y[:, 2]) - prim.r
        return f

    shapes = [("unit sphere, 4096 points", synth.sphere_cloud(4096), truth_sphere)]
    for m in (4096, 1024):
        tc, prim = synth.torus_cloud(m)
        shapes.append((f"ring torus R=0.6 r=0.25, {m} points", tc, truth_torus(prim)))
    acc = {}
    for name, sc, truth in shapes:
        lo, hi = synth.padded_bbox(sc.p, 0.1)
        g = synth.lattice(lo, hi, 64)
        true = truth(g.astype(np.float64))
        c = binding.Cloud(torch.from_numpy(sc.p).cuda(), torch.from_numpy(sc.n).cuda(), torch.from_numpy(sc.a).cuda())
        gd = torch.from_numpy(g).cuda()
        est = {"torus_blend": c(gd)}
        for kind in ("sspd", "shc"):
            est[kind] = binding.eval_baseline(c.rec, c.N, gd, kind, c.params)
        acc[name] = {k: float(np.mean(np.abs(v.cpu().numpy().astype(np.float64) - true))) for k, v in est.items()}
        log(f"baselines: accuracy on {name}: " + ", ".join(f"{k} {v:.3e}" for k, v in acc[name].items()))
    log(f"baselines: mid workload ms: " + ", ".join(f"{k} {v:.2f}" for k, v in ms.items()))
    return {"throughput": thr, "accuracy_mean_abs_error_64cubed": acc}


def bounded_bench(cl, x, reps: int = 3):
    """Error-bounded evaluation on the same workload: far point units skipped
    while a proven bound on the change of phi stays within eps (absolute,
    given as a fraction of the bbox diagonal D).  Reports the time, the
    fraction of pairs actually evaluated, the effective rate N Q / time and
    the evaluated-pair rate, beside the plain evaluation."""
    import numpy as np
    import torch
    from paper_2607_16946_amd import binding
    N, Q = cl.N, x.shape[0]
    p, n, a, xd = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a, x))
    prm = binding.make_params()
    rec = binding.cloud_build(p, n, a, prm)
    D = float(binding.cloud_info(rec).diag)
    ws = torch.empty(binding.eval_bounded_ws_bytes(N, Q, prm), dtype=torch.uint8, device="cuda")
    sdf = torch.empty(Q, dtype=torch.float32, device="cuda")
    pairs = float(N) * Q
    out = {"N": N, "Q": Q, "diag": D, "runs": []}
    for rel in (0.0, 1e-6, 1e-5, 1e-4):
        ms = _timed(lambda: binding.eval_bounded(rec, N, xd, rel * D, prm, ws, sdf), reps)
        _, bd, kept = binding.eval_bounded(rec, N, xd, rel * D, prm, ws, sdf, bound=True, kept=True)
        kf = kept.double()
        frac = float(kf.mean().item()) / N
        r = {"eps_over_D": rel, "ms": ms, "evaluated_frac": frac, "effective_pairs_per_s": pairs / (ms * 1e-3),
             "evaluated_pairs_per_s": frac * pairs / (ms * 1e-3), "max_bound_over_D": float(bd.max().item()) / D,
             "kept_max_over_mean": float(kf.max().item() / max(kf.mean().item(), 1.0))}
        out["runs"].append(r)
        log(f"bounded: eps {rel:g} D: {ms:.2f} ms, {100 * frac:.1f}% of pairs evaluated (max/mean per query "
            f"{r['kept_max_over_mean']:.2f}), effective {r['effective_pairs_per_s']:.3g} pairs/s "
            f"(evaluated {r['evaluated_pairs_per_s']:.3g})")
    return out


def radius_bench(name: str, cl, x, reps: int = 3):
    """Radius-limited evaluation (Sec. 4.2, constant lambda = 1e3/D, R_eval =
    2C/lambda, 32-nearest fallback): preparation (the mean 64-nearest distance
    D over all points) and evaluation at every query, HIP-event timed."""
    import numpy as np
    import torch
    from paper_2607_16946_amd import binding
    p, n, a, xd = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a, x))
    prm = binding.make_params()
    rec = binding.cloud_build(p, n, a, prm)
    ms_prep = _timed(lambda: binding.radius_prepare(rec, cl.N, prm), reps)
    info = binding.radius_info(rec)
    sdf = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
    ws = torch.empty(max(binding.eval_radius_ws_bytes(cl.N, x.shape[0]), 256), dtype=torch.uint8, device="cuda")
    ms_eval = _timed(lambda: binding.eval_radius(rec, cl.N, xd, ws=ws), reps)
    _, cnt = binding.eval_radius(rec, cl.N, xd, count=True, ws=ws)
    cnt = cnt.cpu().numpy()
    out = {"workload": name, "N": cl.N, "Q": int(x.shape[0]), "D": info.D, "lambda": float(info.lam),
           "R_eval": float(info.reval), "prepare_ms": ms_prep, "eval_ms": ms_eval,
           "queries_per_s": x.shape[0] / (ms_eval * 1e-3),
           "frac_within_R_eval": float(np.mean(cnt > 0)), "mean_points_blended": float(np.mean(np.abs(cnt)))}
    log(f"radius ({name}): prepare {ms_prep:.2f} ms, eval {ms_eval:.2f} ms ({out['queries_per_s']:.4g} queries/s), "
        f"{100 * out['frac_within_R_eval']:.1f}% within R_eval, {out['mean_points_blended']:.1f} points blended")
    del sdf
    return out


def serving_bench(n_requests: int, n_warmup: int, loads, n_clouds: int = 64, budget_gib: int = 64,
                  mock: bool = False, quantum: float = 0.0):
    """Serving workload: resident clouds, Poisson arrivals of query / trace requests.

    64 clouds, cloud j from the sphere generator with N log-uniform in
    [1024, 262144]; 90% query requests (Q log-uniform in [1, 65536], x uniform in
    [-1.5, 1.5]^3) and 10% trace requests (256^2 rays, 48 steps, camera on a
    radius-3 sphere aimed at the origin, 45 degree field of view, normals).
    Capacity is measured closed-loop (a burst of requests, all submitted at
    once); then Poisson arrivals at each fraction of it.  Latency is the
    server's own (submit -> result written to host memory)."""
    import numpy as np
    from paper_2607_16946_amd import synth
    from paper_2607_16946_amd.server import Server

    t_setup = time.perf_counter()
    clouds = [synth.serving_cloud(j) for j in range(n_clouds)]
    S = Server(budget_bytes=budget_gib << 30, max_inflight=64, mock=mock, mock_pairs_per_s=1e12,
               quantum_pairs=quantum)
    quantum = quantum if quantum > 0 else 4e9  # 0: the server's default quantum_pairs
    ids = [S.add_cloud(c.p, c.n, c.a) for c in clouds]
    Ns = np.array([c.N for c in clouds], dtype=np.float64)
    diag = [float(np.linalg.norm(c.p.max(0) - c.p.min(0))) for c in clouds]
    cams = []
    for k in range(8):
        o, d = synth.camera_rays(256, radius=3.0, fov_deg=45.0, seed=100 + k)
        d = d.astype(np.float64)
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        cams.append((np.ascontiguousarray(o, np.float32), np.ascontiguousarray(d, np.float32)))
    log(f"serving: {n_clouds} clouds resident (N {int(Ns.min())}..{int(Ns.max())}, sum {int(Ns.sum())}); "
        f"setup {time.perf_counter() - t_setup:.1f} s")
    rng = np.random.Generator(np.random.PCG64(synth.SERVE_SEED_BASE + 777))

    def draw():
        j = int(rng.integers(n_clouds))
        if rng.random() < 0.1:
            return ("trace", j, int(rng.integers(len(cams))))
        q = int(round(math.exp(rng.uniform(0.0, math.log(65536)))))
        return ("eval", j, rng.uniform(-1.5, 1.5, size=(q, 3)).astype(np.float32))

    def submit(r):
        kind, j, arg = r
        if kind == "eval":
            return S.submit_eval(ids[j], arg)
        o, d = cams[arg]
        return S.submit_trace(ids[j], o, d, steps=48, eps=1e-4 * diag[j], tmax=6.0, normals=True)

    def run_open(reqs, rate):
        """Submit reqs at Poisson times of the given rate; wait for all."""
        gaps = rng.exponential(1.0 / rate, size=len(reqs))
        t0 = time.perf_counter()
        due = t0
        tickets, lag = [], 0.0
        for r, g in zip(reqs, gaps):
            due += g
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            lag = max(lag, time.perf_counter() - due)
            tickets.append(submit(r))
        for t in tickets:
            S.wait(t)
        return time.perf_counter() - t0, lag

    # closed-loop capacity
    burst = [draw() for _ in range(min(400, max(n_requests, 100)))]
    S.reset_stats()
    t0 = time.perf_counter()
    ts = [submit(r) for r in burst]
    for t in ts:
        S.wait(t)
    wall = time.perf_counter() - t0
    st = S.stats()
    cap = len(burst) / wall
    out = {"workload": f"{n_clouds} resident clouds (sphere generator, N log-uniform 1024..262144); 90% query "
                       f"requests Q log-uniform 1..65536, 10% 256x256 sphere traces of 48 steps with normals",
           "budget_gib": budget_gib, "clouds": n_clouds, "points_resident": int(Ns.sum()),
           "gpu_max_hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"), "quantum_pairs": quantum,
           "capacity_req_s": cap, "capacity_pairs_s": st["pairs"] / wall, "capacity_requests": len(burst),
           "capacity_launches": st["launches"], "capacity_busy_frac": st["busy_s"] / wall, "loads": []}
    log(f"serving: capacity {cap:.1f} req/s, {st['pairs'] / wall:.3g} pairs/s over {len(burst)} requests "
        f"({st['launches']} launches, device busy {st['busy_s'] / wall:.2f} of wall)")
    for load in loads:
        rate = load * cap
        run_open([draw() for _ in range(n_warmup)], rate)
        S.reset_stats()
        reqs = [draw() for _ in range(n_requests)]
        wall, lag = run_open(reqs, rate)
        st = S.stats()
        row = {"load": load, "offered_req_s": rate, "achieved_req_s": len(reqs) / wall, "requests": len(reqs),
               "n_trace": sum(r[0] == "trace" for r in reqs), "wall_s": wall, "pairs_s": st["pairs"] / wall,
               "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "max_ms": st["max_ms"],
               "p50_query_ms": st["p50_eval_ms"], "p99_query_ms": st["p99_eval_ms"],
               "p50_trace_ms": st["p50_trace_ms"], "p99_trace_ms": st["p99_trace_ms"],
               "launches": st["launches"], "overlapped_launches": st["overlapped_launches"],
               "max_batch_requests": st["max_batch_requests"], "device_busy_frac": st["busy_s"] / wall,
               "max_submit_lag_ms": lag * 1e3}
        out["loads"].append(row)
        log(f"serving: load {load:.2f}: {row['achieved_req_s']:.1f} req/s, p50 {row['p50_ms']:.2f} ms, "
            f"p99 {row['p99_ms']:.2f} ms (query p50/p99 {row['p50_query_ms']:.2f}/{row['p99_query_ms']:.2f}, "
            f"trace {row['p50_trace_ms']:.1f}/{row['p99_trace_ms']:.1f})")
    S.close()
    return out


def step_bench(cl, x, steps: int, warmup: int, label: str, splits: int = 0):
    """One step = the whole hot path through the C ABI on resident inputs: torus
    fitting (pts_cloud_build), the farthest-point sweep, the blend sweep and the
    split combine (pts_eval_far / _blend / _combine).  Returns wall ms per step
    (synchronised on both sides of the timed steps) and each stage's mean time
    from HIP events recorded on the stream the kernels run on."""
    import numpy as np
    import torch
    from paper_2607_16946_amd import binding
    N, Q = cl.N, x.shape[0]
    p, n, a = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a))
    xd = torch.from_numpy(x).cuda()
    prm = binding.make_params(splits=splits)
    rec = torch.empty(binding.record_bytes(N), dtype=torch.uint8, device="cuda")
    ws = torch.empty(max(binding.eval_ws_bytes(N, Q, prm), 256), dtype=torch.uint8, device="cuda")
    sdf = torch.empty(Q, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        binding.cloud_build(p, n, a, prm, rec)
        if ev is not None:
            ev[1].record(stream)
        binding.eval_far(rec, N, xd, prm, ws)
        if ev is not None:
            ev[2].record(stream)
        binding.eval_blend(rec, N, xd, prm, ws)
        if ev is not None:
            ev[3].record(stream)
        binding.eval_combine(N, Q, sdf, prm, ws)
        if ev is not None:
            ev[4].record(stream)

    for i in range(warmup):
        step()
        log(f"bench: {label}: warmup step {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    stage = {k: float(np.mean([e[j].elapsed_time(e[j + 1]) for e in evs]))
             for j, k in enumerate(("build", "far", "blend", "combine"))}
    log(f"bench: {label}: {steps} steps, {ms_step:.3f} ms/step; stages (ms) {stage}")
    del rec, ws, sdf, xd, p, n, a
    torch.cuda.empty_cache()
    return ms_step, stage


def roofline_of(stage, pairs: float, traffic_key: str):
    """Roofline object of the blend sweep (the dominant kernel) from its event-timed launch."""
    achieved_tflops = BLEND_FLOP * pairs / (stage["blend"] * 1e-3) / 1e12
    traffic = measured_traffic(traffic_key)
    return {
        "bound": "alu", "unit": "TFLOP/s", "kernel": "k_blend (blend sweep)",
        "achieved": achieved_tflops, "peak": PEAK_TFLOPS, "frac": achieved_tflops / PEAK_TFLOPS,
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "traffic_over_algorithmic": traffic["over_algorithmic"] if traffic else None,
        "flop_per_pair": BLEND_FLOP, "pairs_per_launch": pairs, "launch_ms": stage["blend"],
        "peak_basis": f"issue-slot ceiling of the blend's instruction mix: {CUS} CU x {CLOCK_HZ / 1e9} GHz / "
                      f"({BLEND_PLAIN + BLEND_FMA} add/mul/FMA at {ARITH_LANES_PER_CLK} lanes/clk + {BLEND_TRANS} "
                      f"sqrt/exp2 at {TRANS_LANES_PER_CLK} lanes/clk per pair) = {PEAK_PAIRS:.3e} pairs/s x "
                      f"{BLEND_FLOP} FLOP",
        "published_fp32_peak": PUBLISHED_FP32_TFLOPS,
        "frac_of_published_fp32": achieved_tflops / PUBLISHED_FP32_TFLOPS,
        "far_sweep": {"ms": stage["far"], "flop_per_pair": FAR_FLOP,
                      "tflops": FAR_FLOP * pairs / (stage["far"] * 1e-3) / 1e12},
    }


def small_bench(reps: int = 100):
    """Latency of small evaluations (pts_eval, phi only): the tiny cloud (4096
    points on the unit sphere) and a 262,144-point sphere cloud, at 1 to 65,536
    uniform queries; median of `reps` HIP-event-timed calls after 5 warm-ups."""
    import numpy as np
    import torch
    from paper_2607_16946_amd import binding, synth
    out = {}
    prm = binding.make_params()
    for name, cl in (("tiny 4096", synth.tiny()[0]), ("sphere 262144", synth.sphere_cloud(262144, 77))):
        c = binding.Cloud(*(torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a)))
        for Q in (1, 64, 1024, 4096, 65536):
            x = torch.from_numpy(np.random.default_rng(Q).uniform(-1.5, 1.5, size=(Q, 3)).astype(np.float32)).cuda()
            ws = torch.empty(max(binding.eval_ws_bytes(c.N, Q, prm), 256), dtype=torch.uint8, device="cuda")
            sdf = torch.empty(Q, dtype=torch.float32, device="cuda")
            ms = _timed(lambda: binding.eval(c.rec, c.N, x, prm, ws=ws, out=sdf), reps, warm=5)
            out[f"{name}, Q={Q}"] = {"ms": ms, "plan": list(binding.eval_plan(c.N, Q, prm)),
                                     "pairs_per_s": float(c.N) * Q / (ms * 1e-3)}
            log(f"small: {name} points, {Q} queries: {ms * 1e3:.1f} us, plan {binding.eval_plan(c.N, Q, prm)}")
    return out


def trace_bench(cl, res: int = 1024, steps: int = 64):
    """The large workload's sphere trace: a res x res pinhole camera at 1.5 D from
    the bbox centre (45 degree field of view), `steps` evaluations per ray,
    eps = 1e-4 D, tmax = 3 D, normals at the hits (pts_trace)."""
    import numpy as np
    import torch
    from paper_2607_16946_amd import binding, synth
    N = cl.N
    p, n, a = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a))
    prm = binding.make_params()
    rec = binding.cloud_build(p, n, a, prm)
    lo, hi = cl.p.min(0), cl.p.max(0)
    D = float(np.linalg.norm(hi.astype(np.float64) - lo))
    ctr = 0.5 * (lo + hi)
    o, d = synth.camera_rays(res, radius=1.5 * D, fov_deg=45.0, seed=5, target=tuple(ctr))
    d = d.astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    od, dd = torch.from_numpy(o.astype(np.float32)).cuda(), torch.from_numpy(d.astype(np.float32)).cuda()
    R = od.shape[0]
    binding.trace(rec, N, od[:4096], dd[:4096], steps=4, eps=1e-4 * D, tmax=3.0 * D, params=prm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    t, hit, ns, nrm = binding.trace(rec, N, od, dd, steps=steps, eps=1e-4 * D, tmax=3.0 * D, params=prm)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t1
    steps_sum = float(torch.clamp(ns, max=steps).sum())
    out = {"rays": R, "steps": steps, "seconds": sec, "hits": int(hit.sum()), "ray_steps": steps_sum,
           "pairs_per_s": steps_sum * N / sec,
           "workload": f"{res}x{res} camera at 1.5 D, 45 deg, {steps} steps, eps 1e-4 D, tmax 3 D, normals"}
    log(f"trace: {R} rays x {steps} steps in {sec:.2f} s, {out['hits']} hits, {steps_sum:.4g} ray-steps, "
        f"{out['pairs_per_s']:.4g} pairs/s")
    # the same march with each step's phi from the error-bounded evaluation
    # (pts_trace_bounded), 1e-6 D per step against the 1e-4 D hit threshold
    ee = 1e-6 * D
    binding.trace(rec, N, od[:4096], dd[:4096], steps=4, eps=1e-4 * D, tmax=3.0 * D, params=prm, eval_eps=ee)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tb, hb, nsb, nrb = binding.trace(rec, N, od, dd, steps=steps, eps=1e-4 * D, tmax=3.0 * D, params=prm,
                                     eval_eps=ee)
    torch.cuda.synchronize()
    secb = time.perf_counter() - t1
    both = hit & hb
    dt = float((tb[both] - t[both]).abs().max()) if bool(both.any()) else 0.0
    steps_b = float(torch.clamp(nsb, max=steps).sum())
    out["bounded"] = {"eval_eps_over_D": 1e-6, "seconds": secb, "speedup": sec / secb, "hits": int(hb.sum()),
                      "ray_steps": steps_b, "effective_pairs_per_s": steps_b * N / secb,
                      "hit_disagreements": int((hit != hb).sum()), "max_abs_dt_over_D": dt / D,
                      "max_normal_diff": float((nrb[both] - nrm[both]).abs().max()) if bool(both.any()) else 0.0}
    log(f"trace (bounded phi, eval_eps 1e-6 D): {secb:.2f} s ({sec / secb:.2f}x), {out['bounded']['hits']} hits, "
        f"{out['bounded']['hit_disagreements']} rays differ in hit, max |dt| {dt / D:.2e} D")
    return out


def serving_child(hw_queues: int, n_requests: int, n_warmup: int, loads: str, quantum: float = 0.0):
    """The serving leg in a child process started with GPU_MAX_HW_QUEUES = hw_queues
    (it must be set before HIP initialises, so not in this process)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--serving-only", "--hw-queues", str(hw_queues),
           "--serve-requests", str(n_requests), "--serve-warmup", str(n_warmup), "--serve-loads", loads,
           "--serve-quantum", str(quantum)]
    log(f"serving: child process with GPU_MAX_HW_QUEUES={hw_queues} ...")
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    for line in r.stderr.splitlines():
        if line.startswith("serving:"):
            log(f"[{hw_queues} queues] {line}")
    if r.returncode != 0:
        return {"error": f"child exited with {r.returncode}", "stderr_tail": r.stderr[-2000:]}
    return json.loads(r.stdout.strip().splitlines()[-1])["serving"]


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=8192,
                    help="oracle sample (queries of the large workload); about 7 s on 16 host threads")
    ap.add_argument("--no-mid", action="store_true", help="skip the mid workload's step")
    ap.add_argument("--no-trace", action="store_true", help="skip the large workload's 1024^2 x 64-step trace")
    ap.add_argument("--trace-only", action="store_true", help="only the large workload's traces (exact and bounded)")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation workload")
    ap.add_argument("--no-baselines", action="store_true", help="skip the two baselines of the accuracy comparison")
    ap.add_argument("--no-radius", action="store_true", help="skip the radius-limited evaluation")
    ap.add_argument("--no-bounded", action="store_true", help="skip the error-bounded evaluation")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the per-configuration GPU-vs-oracle table")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-mode measurement")
    ap.add_argument("--serving-only", action="store_true", help="only the serving-mode measurement")
    ap.add_argument("--diff-only", action="store_true", help="only the differentiation workload")
    ap.add_argument("--bounded-only", action="store_true", help="only the error-bounded evaluation")
    ap.add_argument("--step-only", choices=("large", "mid"), help="only the timed steps of one workload")
    ap.add_argument("--radius-only", choices=("large", "mid"), help="only the radius-limited evaluation of one workload")
    ap.add_argument("--splits", type=int, default=0, help="pts_params.splits of --step-only (0 = automatic)")
    ap.add_argument("--small-only", action="store_true", help="only the latency of small evaluations")
    ap.add_argument("--baselines-only", action="store_true", help="only the two baselines (mid workload)")
    ap.add_argument("--no-small", action="store_true", help="skip the latency of small evaluations")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured requests per load level")
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-loads", default="0.5,0.9", help="arrival rates as fractions of capacity")
    ap.add_argument("--serve-quantum", type=float, default=0.0,
                    help="pairs per packed launch of the server (0 = its default, 4e9)")
    ap.add_argument("--hw-queues", type=int, default=None,
                    help="GPU_MAX_HW_QUEUES for this process (default: raised to 8)")
    ap.add_argument("--no-serving-default-queues", action="store_true",
                    help="skip the serving leg at HIP's default of 4 hardware queues (a child process)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one plain device copy of MIB MiB (calibrates the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(args.copy_calibration * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; multi-GPU figures are not produced "
                                   "(queries shard across GPUs with no exchange; see the design notes)"}))
        sys.exit(2)

    import torch
    from paper_2607_16946_amd import synth

    torch.cuda.set_device(0)
    log(f"bench: device {torch.cuda.get_device_name(0)}")
    loads = [float(v) for v in args.serve_loads.split(",") if v]
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(args.serve_requests, args.serve_warmup, loads,
                                                   quantum=args.serve_quantum)}))
        return
    if args.diff_only:
        print(json.dumps({"diff": diff_bench(max(3, args.steps))}))
        return
    if args.bounded_only:
        cl, x = synth.mid()
        print(json.dumps({"bounded": bounded_bench(cl, x)}))
        return
    if args.baselines_only:
        cl, x = synth.mid()
        print(json.dumps({"baselines": baseline_bench(cl, x)}))
        return
    if args.small_only:
        print(json.dumps({"small": small_bench()}))
        return
    if args.trace_only:
        cl, _ = synth.large()
        print(json.dumps({"trace": trace_bench(cl)}))
        return
    if args.radius_only:
        cl, x = synth.large() if args.radius_only == "large" else synth.mid()
        print(json.dumps({"radius_limited": radius_bench(args.radius_only, cl, x)}))
        return
    if args.step_only:
        cl, x = synth.large() if args.step_only == "large" else synth.mid()
        ms, stage = step_bench(cl, x, args.steps, args.warmup, args.step_only, args.splits)
        print(json.dumps({"workload": args.step_only, "ms_per_step": ms, "stages_ms": stage,
                          "pairs_per_s": float(cl.N) * x.shape[0] / (ms * 1e-3)}))
        return

    t0 = time.perf_counter()
    cl, x = synth.large()
    N, Q = cl.N, x.shape[0]
    log(f"bench: large workload N={N} Q={Q} pairs/step={N * Q:.4g} (generated in {time.perf_counter() - t0:.1f} s)")
    ms_step, stage = step_bench(cl, x, args.steps, args.warmup, "large")
    pairs = float(N) * Q
    value = pairs / (ms_step * 1e-3)
    roofline = roofline_of(stage, pairs, "large")
    probe = None
    if not args.no_probe:
        try:
            probe = probe_issue_rates()
            for k, v in probe["lane_instr_per_s"].items():
                log(f"bench: probe {k:16s} {v:.4g} lane-instr/s  clock {probe['shader_clock_hz'].get(k, 0):.4g}")
        except Exception as e:
            log(f"bench: probe failed: {e}")
    if probe:
        roofline["probe"] = probe
    out = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"large photogrammetry-like: {N} points on 32 random ellipsoids/ring tori, density "
                               f"varying 10x, sigma 0.005 noise, 3% outliers with random normals; {Q} queries "
                               f"uniform in the bbox padded 10%", "N": N, "Q": Q,
                   "C": 64.0, "parallelism": "single GPU"},
        "stages_ms": stage,
        "roofline": roofline,
    }
    if not args.no_trace:
        out["trace"] = trace_bench(cl)
    if not args.no_radius:
        out["radius_limited_large"] = radius_bench("large", cl, x)
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(cl, x, args.cpu_sample)
        log(f"bench: oracle {out['cpu_baseline']['value']:.3g} pairs/s on {out['cpu_baseline']['cores']} threads")
    del cl, x
    mid_cl, mid_x = synth.mid()
    if not args.no_mid:
        ms_mid, st_mid = step_bench(mid_cl, mid_x, 5, 1, "mid")
        pm = float(mid_cl.N) * mid_x.shape[0]
        out["mid"] = {"workload": f"mid: {mid_cl.N} points on 8 random ellipsoids/ring tori, sigma 0.002 noise; "
                                  f"128^3 lattice over the bbox padded 10%", "N": mid_cl.N, "Q": int(mid_x.shape[0]),
                      "ms_per_step": ms_mid, "pairs_per_s": pm / (ms_mid * 1e-3), "stages_ms": st_mid,
                      "roofline": roofline_of(st_mid, pm, "mid")}
    if not args.no_radius:
        out["radius_limited_mid"] = radius_bench("mid", mid_cl, mid_x)
    if not args.no_baselines:
        out["baselines"] = baseline_bench(mid_cl, mid_x)
    if not args.no_bounded:
        out["bounded"] = bounded_bench(mid_cl, mid_x)
    del mid_cl, mid_x
    if not args.no_small:
        out["small"] = small_bench()
    if not args.no_diff:
        out["diff"] = diff_bench(5)
    if not args.no_serving:
        # a server runs in a process of its own: after the other legs, this
        # process's streams can leave the server's two launch streams on one
        # hardware queue (device busy 1.17 of wall against 1.71 in a fresh
        # process, same request stream)
        out["serving"] = serving_child(8, args.serve_requests, args.serve_warmup, args.serve_loads,
                                       args.serve_quantum)
        if not args.no_serving_default_queues:
            out["serving_4_hw_queues"] = serving_child(4, args.serve_requests, args.serve_warmup, args.serve_loads,
                                                       args.serve_quantum)
    if not args.no_configs:
        out["configs"] = configs_bench(min(16, os.cpu_count() or 1))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
