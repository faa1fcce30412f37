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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_blend_mid_traffic.json")


def measured_traffic():
    """HBM bytes per k_blend launch from the committed counter summary, if it
    was taken on the current kernel source (else None)."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_2607_16946_amd", "csrc", "pts_eval.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return rec.get("bytes_per_launch") if rec.get("pts_eval_sha256") == h else None


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
            probe = probe_issue_rates()
            for k, v in probe["lane_instr_per_s"].items():
                log(f"bench: probe {k:16s} {v:.4g} lane-instr/s  clock {probe['shader_clock_hz'].get(k, 0):.4g}")
        except Exception as e:
            log(f"bench: probe failed: {e}")
    achieved_tflops = BLEND_FLOP * pairs / (stage["blend"] * 1e-3) / 1e12
    roofline = {
        "bound": "alu", "unit": "TFLOP/s", "kernel": "k_blend (blend sweep)",
        "achieved": achieved_tflops, "peak": PEAK_TFLOPS, "frac": achieved_tflops / PEAK_TFLOPS,
        "traffic": measured_traffic(),
        "flop_per_pair": BLEND_FLOP, "pairs_per_launch": pairs, "launch_ms": stage["blend"],
        "peak_basis": f"{CUS} CU x {CLOCK_HZ / 1e9} GHz / ({BLEND_PLAIN + BLEND_FMA} add/mul/FMA at "
                      f"{ARITH_LANES_PER_CLK} lanes/clk + {BLEND_TRANS} sqrt/exp2 at {TRANS_LANES_PER_CLK} lanes/clk "
                      f"per pair) = {PEAK_PAIRS:.3e} pairs/s x {BLEND_FLOP} FLOP",
        "frac_of_published_fp32": achieved_tflops / PUBLISHED_FP32_TFLOPS,
        "far_sweep": {"ms": stage["far"], "flop_per_pair": FAR_FLOP,
                      "tflops": FAR_FLOP * pairs / (stage["far"] * 1e-3) / 1e12},
    }
    if probe:
        roofline["probe"] = probe
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
