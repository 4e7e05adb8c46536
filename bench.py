#!/usr/bin/env python3
"""Throughput of the ensemble mapper on one MI355X.

Metric: orbit map-steps per second with the tangent map (one map step = one
application of the 6th-order map -- 9 kicks, 10 drifts -- to one orbit and its
tangent vector), with the fraction of the FP64 vector-ALU peak reached by the
propagation kernel, beside the CPU oracle timed on this host.

Default workload (c2): eps = 1e-3, a 1024 x 1024 slice of (px, py) in
[0, 2 pi)^2 with x = y = z = pz = 0, T = 1e5 steps of h = 0.01 * 2 pi, tangent
start seed 0; one bench step = initial conditions + propagation + per-orbit
indicators + the chi image, the class map and the chaotic count.

Prints ONE JSON line.  Single GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
KERNEL_SOURCES = ["paper_1107_4107_amd/csrc/aw_fwd.hip", "paper_1107_4107_amd/csrc/aw_device.hpp",
                  "paper_1107_4107_amd/csrc/aw_sincos_coef.h", "paper_1107_4107_amd/csrc/aw_internal.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(ens, target_s: float, threads: int):
    """The oracle on a bounded sample of the same workload: a strided set of
    orbits of the slice, each run for the full T steps."""
    import numpy as np

    import oracle
    N = ens.nx * ens.ny
    h = ens.h

    def run(m):
        idx = np.linspace(0, N - 1, m).astype(np.int64)
        ic = oracle.ic_grid2(tuple(ens.axis), tuple(ens.lo), tuple(ens.hi), ens.nx, ens.ny, list(ens.base), idx=idx)
        w0 = oracle.w0(ens.seed_tangent, idx=idx)
        t0 = time.perf_counter()
        oracle.ensemble(ens.map_form, ens.eps, h, ens.n_steps, ic, w0, nthreads=threads)
        return time.perf_counter() - t0

    m0 = max(threads, 16)
    t0 = run(m0)
    rate0 = m0 * ens.n_steps / t0
    m = int(max(m0, min(N, rate0 * target_s / ens.n_steps)))
    m = max(threads, (m // threads) * threads)
    t = run(m)
    return {"value": m * ens.n_steps / t, "unit": "map-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} orbits (evenly strided over the {ens.nx}x{ens.ny} slice) x {ens.n_steps} steps, "
                      f"{t:.1f} s on {threads} host threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--opl", type=int, default=1)
    ap.add_argument("--unroll", type=int, default=1)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the ensemble path has no multi-GPU mode in this build "
              "(orbits are independent; see the sharding notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1107_4107_amd as aw
    from paper_1107_4107_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    ens = wl.c2() if args.workload == "c2" else wl.c1()
    desc = {"c2": "eps=1e-3 1024x1024 (px,py) slice, T=1e5, S6 + tangent, chi image + class map",
            "c1": "eps=1e-2 64x64 (px,py) slice, T=1e3, S6 + tangent, chi image"}[args.workload]
    N, T = ens.nx * ens.ny, ens.n_steps
    spec = wl.chi_image(ens.nx)
    tuning = aw.Tuning(block=args.block, orbits_per_lane=args.opl, unroll=args.unroll)

    def step():
        return aw.indicator_image(ens, spec, want_counts=True, want_class=True, tuning=tuning)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    aw.timing_read()
    aw.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        img, cnt, cls = step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done ({time.perf_counter() - t0:.2f} s)")
    elapsed = time.perf_counter() - t0
    aw.timing_enable(False)
    kern_ms, launches = aw.timing_read()
    n_chaotic = int(cnt.cpu().numpy().view("uint32")[0])

    fma, mul, add = aw.step_op_counts(ens.map_form, True)
    flop_per_step = 2 * fma + mul + add
    kms = kern_ms / max(launches, 1)
    achieved = flop_per_step * N * T / (kms * 1e-3) / 1e12
    value = N * T * args.steps / elapsed

    cpu = None
    if not args.no_cpu_baseline:
        threads = host_threads()
        log(f"cpu baseline on {threads} threads ...")
        cpu = cpu_baseline(ens, args.cpu_seconds, threads)

    rec = {
        "metric": "orbit map-steps/sec (with tangent map)",
        "value": value,
        "unit": "map-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "eps": ens.eps, "grid": [ens.nx, ens.ny],
                   "n_orbits": N, "n_steps": T, "h": ens.h, "map": ens.map_form, "tangent": True,
                   "tuning": {"block": args.block, "orbits_per_lane": args.opl, "unroll": args.unroll}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic_for(args.workload),
                     "kernel": "k_fwd<6,true,1,1> (propagation)", "kernel_ms": kms,
                     "flop_per_map_step": flop_per_step, "fp64_ops_per_map_step": {"fma": fma, "mul": mul, "add": add}},
        "cpu_baseline": cpu,
        "chaotic_fraction": n_chaotic / N,
    }
    if cpu:
        rec["speedup_vs_oracle"] = value / cpu["value"]
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
