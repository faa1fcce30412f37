#!/usr/bin/env python3
"""Throughput of the pointwise SDF hot path on one MI355X.

Workload (one "step"): the mid-size plain-method configuration -- a
131,072-point cloud on the union of 8 random ellipsoids / ring tori with
sigma = 0.002 position noise and analytic coefficients, queried on the 128^3
lattice over its bounding box padded by 10% per side.  A step runs the whole
path through the C ABI: torus fitting (pts_cloud_build), the farthest-point
sweep, the blend sweep and the split combine (pts_eval_far / _blend /
_combine).  Inputs are resident in device memory before timing starts.

Prints one JSON line (rank 0): value = query x point SDF evaluations per
second (pairs/s), with a `roofline` object for the dominant kernel (the blend
sweep, timed with HIP events on the stream it runs on) and a `cpu_baseline`
object (the FP64 oracle on a bounded sample, on this host's cores).
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "query×point SDF evals/sec (FP32, % of VALU peak); p50/p99 latency in serving mode"

# Algorithmic work per (query, point) pair, counted from the definition
# (Eqs. BasicFormulaShifted, RelationshipBetweenLambdaAndRadius,
# SingleTorusSDF): farthest-point sweep 5 plain + 2 FMA; blend sweep 13 plain +
# 11 FMA + 4 transcendental (3 sqrt, 1 exp).  FLOPs count an FMA as 2.
BLEND_PLAIN, BLEND_FMA, BLEND_TRANS = 13, 11, 4
BLEND_FLOP = BLEND_PLAIN + 2 * BLEND_FMA + BLEND_TRANS      # 39
FAR_FLOP = 5 + 2 * 2                                         # 9

# MI355X: 256 CUs x 4 SIMD x 16 lanes, 2.4 GHz peak engine clock.
CUS, LANES_PER_CU, CLOCK_HZ = 256, 64, 2.4e9
LANE_SLOTS = CUS * LANES_PER_CU * CLOCK_HZ                   # 3.93e13 VALU lane-instr/s
PUBLISHED_FP32_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def probe_issue_costs():
    """Issue cost of v_exp_f32 / v_sqrt_f32 / v_rcp_f32 relative to v_fma_f32, and the shader clock."""
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
    rates, clock = {}, None
    for op, name, iters in ((0, "fma", 8192), (1, "exp", 2048), (2, "sqrt", 2048), (3, "rcp", 2048),
                            (5, "exp+4fma", 1024), (6, "sqrt+4fma", 1024)):
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
        if op == 0:
            ticks = clk.cpu().tolist()
            if ticks[1] > 0:
                clock = ticks[0] / (ticks[1] / 100e6)
    fma = rates["fma"]
    tau = {k: fma / rates[k] for k in ("exp", "sqrt", "rcp")}
    # mixes: slots of (1 trans + 4 fma) relative to 5 fma
    tau["exp_in_mix"] = 5 * fma / rates["exp+4fma"] - 4
    tau["sqrt_in_mix"] = 5 * fma / rates["sqrt+4fma"] - 4
    return {"fma_lane_instr_per_s": fma, "tau": tau, "shader_clock_hz": clock, "rates": rates}


def cpu_baseline(cl, x, sample: int):
    import numpy as np
    import oracle
    threads = min(16, os.cpu_count() or 1)
    oracle.threads(threads)
    idx = np.random.default_rng(12345).choice(x.shape[0], size=min(sample, x.shape[0]), replace=False)
    xs = x[np.sort(idx)]
    t0 = time.perf_counter()
    tor = oracle.fit(cl.p, cl.n, cl.a)
    t1 = time.perf_counter()
    oracle.eval_sdf(cl.p, tor, xs, nthreads=threads)
    t2 = time.perf_counter()
    pairs = xs.shape[0] * cl.N
    return {"value": pairs / (t2 - t1), "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{xs.shape[0]} seeded queries of the {x.shape[0]}-query lattice x all {cl.N} points "
                      f"({pairs:.3g} pairs), FP64, after a {t1 - t0:.2f} s torus fit",
            "seconds": t2 - t1}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=128, help="query lattice resolution (default 128)")
    ap.add_argument("--points", type=int, default=131072)
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU figures are not produced "
                                   "(queries shard across GPUs with no exchange; see the design notes)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2607_16946_amd import binding, synth

    torch.cuda.set_device(0)
    log(f"bench: device {torch.cuda.get_device_name(0)}")
    cl, x = synth.mid(N=args.points, grid=args.grid)
    N, Q = cl.N, x.shape[0]
    log(f"bench: workload N={N} Q={Q} pairs/step={N * Q:.4g}")
    p, n, a = (torch.from_numpy(v).cuda() for v in (cl.p, cl.n, cl.a))
    xd = torch.from_numpy(x).cuda()
    prm = binding.make_params()
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

    for i in range(args.warmup):
        step()
        log(f"bench: warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    stage = {k: float(np.mean([e[j].elapsed_time(e[j + 1]) for e in evs]))
             for j, k in enumerate(("build", "far", "blend", "combine"))}
    log(f"bench: {args.steps} steps, {ms_step:.3f} ms/step; stages (ms) {stage}")
    pairs = float(N) * Q
    value = pairs / (ms_step * 1e-3)

    probe = None
    if not args.no_probe:
        try:
            probe = probe_issue_costs()
            log(f"bench: probe tau {probe['tau']} clock {probe['shader_clock_hz']}")
        except Exception as e:  # the roofline falls back to the documented quarter rate
            log(f"bench: probe failed: {e}")
    tau_sqrt = probe["tau"]["sqrt"] if probe else 4.0
    tau_exp = probe["tau"]["exp"] if probe else 4.0
    # minimum VALU issue slots per blend pair for the algorithm's op mix
    slots = BLEND_PLAIN + BLEND_FMA + 3 * tau_sqrt + tau_exp
    peak_tflops = BLEND_FLOP * LANE_SLOTS / slots / 1e12
    achieved_tflops = BLEND_FLOP * pairs / (stage["blend"] * 1e-3) / 1e12
    roofline = {
        "bound": "alu", "unit": "TFLOP/s", "kernel": "k_blend (blend sweep)",
        "achieved": achieved_tflops, "peak": peak_tflops, "frac": achieved_tflops / peak_tflops,
        "traffic": None,
        "flop_per_pair": BLEND_FLOP, "pairs_per_launch": pairs, "launch_ms": stage["blend"],
        "peak_basis": f"{CUS} CU x {LANES_PER_CU} lanes x {CLOCK_HZ / 1e9} GHz / ({BLEND_PLAIN}+{BLEND_FMA} "
                      f"plain/FMA + 3x{tau_sqrt:.2f} sqrt + {tau_exp:.2f} exp issue slots per pair), "
                      "no packed FP32",
        "frac_of_published_fp32": achieved_tflops / PUBLISHED_FP32_TFLOPS,
    }
    if probe:
        roofline["probe"] = {"tau": probe["tau"], "shader_clock_hz": probe["shader_clock_hz"],
                             "fma_lane_instr_per_s": probe["fma_lane_instr_per_s"]}
    out = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"mid: {N} points on 8 random ellipsoids/ring tori, sigma 0.002 noise; "
                               f"{args.grid}^3 lattice over the bbox padded 10%", "N": N, "Q": Q,
                   "C": 64.0, "parallelism": "single GPU"},
        "stages_ms": stage,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(cl, x, args.cpu_sample)
        log(f"bench: oracle {out['cpu_baseline']['value']:.3g} pairs/s on {out['cpu_baseline']['cores']} threads")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
