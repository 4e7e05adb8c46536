#!/usr/bin/env python3
"""Throughput of the ensemble mapper on one MI355X.

Metric: orbit map-steps per second with the tangent map (one map step = one
application of the 6th-order map -- 9 kicks, 10 drifts -- to one orbit and its
tangent vector), with the fraction of the FP64 vector-ALU peak reached by the
propagation kernel, beside the CPU oracle timed on this host.

Default workload (c2): eps = 1e-3, a 1024 x 1024 slice of (px, py) in
[0, 2 pi)^2 with x = y = z = pz = 0, T = 1e5 steps of h = 0.01 * 2 pi, tangent
start seed 0; one bench step = initial conditions + propagation + per-orbit
indicators + the chi image, the class map and the chaotic count.  The default
line also carries sub-records timed after the steps: one 1e5-step chunk of
the 1e7-orbit ensemble (c5_chunk), the c4 gradients against their forward
passes (c4_gradients), and the c3 batch at a tenth of its horizons against
its separate launches (c3_batch_t0.1); then the oracle on all host threads
and on one.

Other workloads (measurement records, not the default line):
  c1  the 64 x 64, T = 1e3 slice at eps = 1e-2 (latency-bound);
  c3  64 ensembles (eps sweep, mixed grids and horizons): one persistent
      launch captured in a HIP graph against the sum of 64 separate launches;
  c4  gradient of J on the 512 x 512, T = 1e4 slice with checkpoints every
      100 steps: adjoint time against the forward pass; also the gradient of
      the tangent growth L (second-order adjoint) on the same slice, and both
      in one segment (every step state stored by the forward pass) where HBM
      holds them;
  c5  1e7 orbits uniform on [0, 2 pi)^6, eps = 5e-3, T = 1e6, run in chunks
      of 1e5 steps with the state carried in HBM, then the momentum-drift image
      and the direction density on the sphere (512 x 512 each);
  nsweep  map-steps/s against the ensemble size N = 1e3 .. 1e7 at T = 1e4
      (the c5 distribution): where the device fills;
  peak    the achievable FP64 rate of independent FMA chains and the shader
      clock the SIMDs sustain under that load (the probe library);
  forms   the integrators side by side on one slice (eps = 1e-2, 512 x 512,
      pz0 = 1, T = 1e4): map-steps/s and the energy error |dE| at h and 2h;
  energy  the energy error of S6 at the paper's h on the configurations' eps
      and at the paper's energies E = 400 and E = 15.

Prints ONE JSON line.  Single GPU only.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
# Best rate of independent v_fma_f64 chains measured on this GPU model with
# `bench.py --workload peak` (8 waves per SIMD, 2.384 GHz sustained).
FP64_ACHIEVABLE_TFLOPS = 76.92
KICKS_PER_STEP = {"stdmap": 1, "s2": 1, "s4": 3, "s6": 9, "y6": 7}
KERNEL_SOURCES = ["paper_1107_4107_amd/csrc/aw_fwd.hip", "paper_1107_4107_amd/csrc/aw_device.hpp",
                  "paper_1107_4107_amd/csrc/aw_sincos_coef.h", "paper_1107_4107_amd/csrc/aw_sincos_tab.h",
                  "paper_1107_4107_amd/csrc/aw_internal.hpp"]
METRIC = "orbit map-steps/sec (with tangent map)"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the propagation kernel's sources with comments and whitespace
    taken out, so that a counter record stays keyed across edits that cannot
    change the code."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
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


def valu_for(workload: str):
    """VALU wave-instructions per map step from the committed counter record,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.json")
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_source_hash") != kernel_hash():
        return None
    return rec.get("valu_insts_per_map_step")


def host_info() -> str:
    """CPU model, logical CPUs and SMT state of the host the oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    smt = "unknown"
    try:
        smt = "on" if open("/sys/devices/system/cpu/smt/active").read().strip() == "1" else "off"
    except OSError:
        pass
    return f"{model}; {os.cpu_count()} logical CPUs; SMT {smt}"


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


_ORACLE_BUILD = None


def oracle_native():
    """The oracle built for this host (gcc -O3 -march=native, contraction off:
    bitwise the results of the portable build), loaded for the timing."""
    global _ORACLE_BUILD
    import atexit
    import shutil
    import tempfile

    import oracle
    if _ORACLE_BUILD is None:
        tmp = tempfile.mkdtemp(prefix="aw_oracle_")
        atexit.register(shutil.rmtree, tmp, True)
        path = os.path.join(tmp, "liboracle_native.so")
        oracle.build(force=True, variant="native", out=path)
        oracle.use_build(path)
        _ORACLE_BUILD = "gcc " + " ".join(oracle.CFLAGS + oracle.VARIANT_FLAGS["native"])
    return _ORACLE_BUILD


def cpu_baseline(ens, target_s: float, threads: int):
    """The oracle as it stands on a bounded sample of the same workload: an
    evenly strided set of its orbits, each run for the full T steps."""
    import numpy as np

    import oracle
    build = oracle_native()
    N = ens.size

    def sample(m):
        idx = np.linspace(0, N - 1, m).astype(np.int64)
        if ens.ic_kind == "grid2":
            ic = oracle.ic_grid2(tuple(ens.axis), tuple(ens.lo), tuple(ens.hi), ens.nx, ens.ny, list(ens.base),
                                 idx=idx)
        else:
            ic = oracle.ic_box(ens.box_lo, ens.box_hi, ens.seed_ic, idx=idx)
        return ic, oracle.w0(ens.seed_tangent, idx=idx)

    def run(m):
        ic, w0 = sample(m)
        t0 = time.perf_counter()
        oracle.ensemble(ens.map_form, ens.eps, ens.h, ens.n_steps, ic, w0, nthreads=threads)
        return time.perf_counter() - t0

    m0 = threads
    t0 = run(m0)
    rate0 = m0 * ens.n_steps / t0
    m = int(max(m0, min(N, rate0 * target_s / ens.n_steps)))
    m = max(threads, (m // threads) * threads)
    t = run(m)
    where = f"{ens.nx}x{ens.ny} slice" if ens.ic_kind == "grid2" else f"{N} orbits"
    return {"value": m * ens.n_steps / t, "unit": "map-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} orbits (evenly strided over the {where}) x {ens.n_steps} steps each, "
                      f"{t:.1f} s on {threads} host thread{'s' if threads > 1 else ''}", "host": host_info(),
            "build": build}


def roofline(aw, ens, kernel_ms, workload, steps_per_launch=None):
    """FP64 roofline of the propagation kernel: algorithmic flops of one
    launch (flop per map step x orbits x steps the launch runs) over its
    average duration."""
    fma, mul, add = aw.step_op_counts(ens.map_form, ens.tangent)
    flop = 2 * fma + mul + add
    steps = ens.n_steps if steps_per_launch is None else steps_per_launch
    achieved = flop * ens.size * steps / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic_for(workload),
            "frac_of_achievable_peak": achieved / FP64_ACHIEVABLE_TFLOPS,
            "force_evals_per_s": KICKS_PER_STEP[ens.map_form] * ens.size * steps / (kernel_ms * 1e-3),
            "kernel": f"k_fwd<{ {'s6': 6, 's4': 4, 's2': 2, 'stdmap': 1}[ens.map_form]},"
                      f"{'true' if ens.tangent else 'false'}> (propagation)",
            "kernel_ms": kernel_ms, "flop_per_map_step": flop,
            "fp64_ops_per_map_step": {"fma": fma, "mul": mul, "add": add},
            "valu_issue": valu_issue(ens, kernel_ms, workload, steps)}


def valu_issue(ens, kernel_ms, workload, steps):
    """The instruction-issue view of the same launch: every wave64 VALU
    instruction occupies its SIMD for 4 cycles, so the chip issues at most
    1024 SIMDs x 2.4 GHz / 4 wave-instructions per second."""
    per_step = valu_for(workload)
    if per_step is None:
        return None
    achieved = per_step / 64.0 * ens.size * steps / (kernel_ms * 1e-3)
    peak = 1024 * 2.4e9 / 4
    flop = sum(k * v for k, v in zip((2, 1, 1), _ops(ens)))
    return {"valu_insts_per_map_step": per_step, "achieved": achieved, "peak": peak,
            "unit": "wave-instructions/s", "frac": achieved / peak,
            "note": f"the kernel is bound by VALU issue: {per_step:.0f} wave-instructions per map step carry "
                    f"{flop} FP64 flops ({flop / per_step:.2f} per instruction), which caps the FP64 fraction "
                    f"at {flop / per_step / 2:.0%} of the FMA peak even at full issue"}


def _ops(ens):
    import paper_1107_4107_amd as aw
    return aw.step_op_counts(ens.map_form, ens.tangent)


def base_record(value, steps, warmup, ms_per_step, dtype="f64"):
    return {"metric": METRIC, "value": value, "unit": "map-steps/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic"}


# ---------------------------------------------------------------------------
def run_slice(args, aw, wl, torch):
    ens = wl.c2() if args.workload == "c2" else wl.c1()
    desc = {"c2": "eps=1e-3 1024x1024 (px,py) slice, T=1e5, S6 + tangent, chi image + class map",
            "c1": "eps=1e-2 64x64 (px,py) slice, T=1e3, S6 + tangent, chi image"}[args.workload]
    N, T = ens.size, ens.n_steps
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
    rec = base_record(N * T * args.steps / elapsed, args.steps, args.warmup, elapsed / args.steps * 1e3)
    rec["config"] = {"workload": f"{args.workload}: {desc}", "eps": ens.eps, "grid": [ens.nx, ens.ny],
                     "n_orbits": N, "n_steps": T, "h": ens.h, "map": ens.map_form, "tangent": True,
                     "tuning": {"block": args.block or "auto", "orbits_per_lane": args.opl, "unroll": args.unroll}}
    rec["roofline"] = roofline(aw, ens, kern_ms / max(launches, 1), args.workload)
    rec["chaotic_fraction"] = n_chaotic / N
    return rec, ens


def run_c5_chunk(aw, wl, torch, chunk: int = 100_000):
    """One chunk of the largest configuration: the 1e7-orbit ensemble uniform
    on [0, 2 pi)^6 (eps = 5e-3) advanced by 1e5 of its 1e6 steps from the
    initial conditions, the state left in HBM as the chunked run carries it."""
    e = wl.c5()
    N = e.size
    carry = torch.empty((aw.NCARRY, N), dtype=torch.float64, device="cuda")
    aw.map_ensemble_steps(e, carry, 0, 1000)          # warm-up (loads the kernel)
    torch.cuda.synchronize()
    aw.timing_read()
    aw.timing_enable(True)
    t0 = time.perf_counter()
    aw.map_ensemble_steps(e, carry, 0, chunk)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    aw.timing_enable(False)
    kern_ms, launches = aw.timing_read()
    del carry
    log(f"c5 chunk: {N} orbits x {chunk} steps in {elapsed:.2f} s")
    return {"workload": f"c5 chunk: {N} orbits uniform on [0,2pi)^6 (seed 2), eps=5e-3, steps 0..{chunk} of 1e6, "
                        f"S6 + tangent, state carried in HBM", "value": N * chunk / elapsed, "unit": "map-steps/s",
            "ms": elapsed * 1e3, "n_orbits": N, "n_steps": chunk,
            "roofline": roofline(aw, e, kern_ms / max(launches, 1), "c5", steps_per_launch=chunk)}


def sub_record(fn):
    """A sub-record of the default line; a failure is recorded, not raised."""
    try:
        return fn()
    except Exception as exc:  # noqa: BLE001 -- the main line must still print
        log(f"sub-record failed: {exc!r}")
        return {"error": repr(exc)}


def c4_summary(args, aw, wl, torch):
    """The gradients of the 512x512, T = 1e4 slice against their forward passes."""
    sub = argparse.Namespace(**{**vars(args), "no_one_segment": True})
    r, _ = run_adjoint(sub, aw, wl, torch)
    keys = ("forward_s", "forward_tangent_s", "gradient_s", "gradient_over_forward", "reversible_gradient_s",
            "reversible_gradient_over_forward", "ftle_gradient_s", "ftle_gradient_over_forward_tangent",
            "reversible_ftle_gradient_s", "reversible_ftle_gradient_over_forward_tangent")
    return {"workload": r["config"]["workload"], **{k: r[k] for k in keys}}


def c3_summary(args, aw, wl, torch):
    """The 64-ensemble batch at a tenth of its horizons: one graph launch
    against the separate launches."""
    sub = argparse.Namespace(**{**vars(args), "t_scale": 0.1})
    r, _ = run_batched(sub, aw, wl, torch)
    keys = ("batched_s", "separate_s", "separate_own_tuning_s", "batched_over_separate_throughput",
            "batched_over_separate_same_shape", "batched_equals_separate_bitwise")
    return {"workload": r["config"]["workload"], "value": r["value"], "unit": r["unit"], **{k: r[k] for k in keys}}


def run_batched(args, aw, wl, torch):
    """One graph launch of the 64-ensemble batch vs 64 separate launches."""
    from paper_1107_4107_amd.autotune import autotune
    ens = wl.c3(t_scale=args.t_scale)
    total = sum(e.size * e.n_steps for e in ens)
    log(f"c3: {len(ens)} ensembles, {sum(e.size for e in ens)} orbits, {total:.4g} map-steps")
    tun = autotune(ens, verbose=True)
    log(f"autotuned: {tun}")
    # chi image of every ensemble on its own grid (W = H = 0) and its chaotic count
    spec = aw.ImageSpec(kind="ic_grid", field=aw.OUT_CHI, W=0, H=0)
    imgs = [torch.empty((e.ny, e.nx), dtype=torch.float64, device="cuda") for e in ens]
    cnts = [torch.empty((1,), dtype=torch.int32, device="cuda") for e in ens]
    graph = aw.Graph(ens, spec, imgs, cnts, tuning=tun)
    small = [dataclasses.replace(e, n_steps=10) for e in ens]
    aw.map_ensembles(small, tuning=tun)   # warm-up of the kernels on tiny horizons
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graph.launch()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    log(f"batched (one graph launch): {tb:.2f} s")
    sep = []
    t0 = time.perf_counter()
    for e in ens:
        sep.append(aw.indicator_image(e, spec, want_counts=True, tuning=tun))
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    log(f"separate (64 launches, the batch's launch shape): {ts:.2f} s")
    # The separate launches again, each with the shape tuned for it alone.
    own = [autotune([e]) for e in ens]
    aw.map_ensembles([small[0]], tuning=own[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sep_own = [aw.indicator_image(e, spec, want_counts=True, tuning=t) for e, t in zip(ens, own)]
    torch.cuda.synchronize()
    ts_own = time.perf_counter() - t0
    log(f"separate (64 launches, each with its own tuned shape): {ts_own:.2f} s")
    same = all(torch.equal(a, b[0]) and torch.equal(c, b[1]) for a, c, b in zip(imgs, cnts, sep))
    same = same and all(torch.equal(a, b[0]) for a, b in zip(imgs, sep_own))
    graph.close()
    rec = base_record(total / tb, 1, 0, tb * 1e3)
    rec["config"] = {"workload": f"c3: 64 ensembles, eps 1e-4..1e-1 log-spaced, grids 128^2..1024^2 and T "
                                 f"1e4/3e4/1e5 drawn with seed 1 (horizons x{args.t_scale}), one persistent launch",
                     "n_orbits": sum(e.size for e in ens), "map_steps": total,
                     "tuning": dataclasses.asdict(tun)}
    rec["batched_s"] = tb
    rec["separate_s"] = ts
    rec["separate_own_tuning_s"] = ts_own
    rec["batched_over_separate_throughput"] = ts_own / tb
    rec["batched_over_separate_same_shape"] = ts / tb
    rec["batched_equals_separate_bitwise"] = bool(same)
    return rec, None


def run_adjoint(args, aw, wl, torch):
    s = wl.c4()
    N, T = s.size, s.n_steps
    ic, _ = aw.generate_ic(s)
    fwd = aw.Ensemble(eps=s.eps, n_steps=T, ic_kind="explicit", n_orbits=N, tangent=False)
    fwd_t = dataclasses.replace(fwd, tangent=True)
    ws = torch.empty((aw.grad_workspace_bytes(fwd, wl.C4_CKPT),), dtype=torch.uint8, device="cuda")

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        return ts[len(ts) // 2]

    t_fwd = timed(lambda: aw.map_ensemble(fwd, ic, want_class=False))
    t_fwd_tan = timed(lambda: aw.map_ensemble(fwd_t, ic, want_class=False))
    t_grad = timed(lambda: aw.indicator_grad(fwd, ic, ckpt_every=wl.C4_CKPT, workspace=ws))
    t_grad_rev = timed(lambda: aw.indicator_grad(fwd, ic, ckpt_every=wl.C4_CKPT, workspace=ws, reversible=True))
    log(f"forward {t_fwd:.3f} s, forward+tangent {t_fwd_tan:.3f} s, gradient {t_grad:.3f} s, "
        f"reversible gradient {t_grad_rev:.3f} s")
    del ws
    # Gradient of the tangent growth L (second-order adjoint) on the same slice.
    _, w0 = aw.generate_ic(fwd_t, ic)
    ws2 = torch.empty((aw.ftle_grad_workspace_bytes(fwd_t, wl.C4_CKPT),), dtype=torch.uint8, device="cuda")
    t_fgrad = timed(lambda: aw.ftle_grad(fwd_t, ic, w0, ckpt_every=wl.C4_CKPT, workspace=ws2))
    t_fgrad_rev = timed(lambda: aw.ftle_grad(fwd_t, ic, w0, ckpt_every=wl.C4_CKPT, workspace=ws2, reversible=True))
    log(f"FTLE gradient {t_fgrad:.3f} s, reversible {t_fgrad_rev:.3f} s")
    g_ck = aw.ftle_grad(fwd_t, ic, w0, ckpt_every=wl.C4_CKPT, workspace=ws2)
    del ws2
    # One segment: the forward pass stores every step state and the reverse
    # sweep reads them back without recomputing, where HBM holds them
    # (6 doubles per orbit-step for J, 12 for L: 126 GB and 252 GB here).
    free = torch.cuda.mem_get_info()[0]
    one = {}
    for name, ens, nbytes, call in (
            ("gradient", fwd, aw.grad_workspace_bytes(fwd, T),
             lambda w: aw.indicator_grad(fwd, ic, ckpt_every=T, workspace=w)),
            ("ftle_gradient", fwd_t, aw.ftle_grad_workspace_bytes(fwd_t, T),
             lambda w: aw.ftle_grad(fwd_t, ic, w0, ckpt_every=T, workspace=w))):
        if args.no_one_segment or nbytes + (4 << 30) > free:
            one[name] = None
            log(f"{name} in one segment skipped: {nbytes / 1e9:.1f} GB of workspace, {free / 1e9:.1f} GB free"
                + (" (--no-one-segment)" if args.no_one_segment else ""))
            continue
        w = torch.empty((nbytes,), dtype=torch.uint8, device="cuda")
        t1 = timed(lambda: call(w))
        if name == "gradient":
            same = all(torch.equal(a, b) for a, b in zip(call(w), aw.indicator_grad(fwd, ic, ckpt_every=wl.C4_CKPT)))
        else:
            same = all(torch.equal(a, b) for a, b in zip(call(w), g_ck))
        del w
        torch.cuda.empty_cache()
        one[name] = (t1, nbytes, bool(same))
        log(f"{name} in one segment {t1:.3f} s ({nbytes / 1e9:.1f} GB of workspace), equal to the checkpointed "
            f"one bit for bit: {same}")
    del g_ck
    rec = base_record(N * T / t_grad, 3, 1, t_grad * 1e3)
    rec["metric"] = "orbit map-steps/sec through the adjoint (forward + checkpoints + reverse)"
    rec["config"] = {"workload": "c4: eps=1e-2 512x512 (px,py) slice, T=1e4, checkpoint every 100 steps, "
                                 "gradient of J w.r.t. (x,p) and eps", "n_orbits": N, "n_steps": T}
    rec["forward_s"] = t_fwd
    rec["forward_tangent_s"] = t_fwd_tan
    rec["gradient_s"] = t_grad
    rec["gradient_over_forward"] = t_grad / t_fwd
    rec["gradient_over_forward_tangent"] = t_grad / t_fwd_tan
    rec["reversible_gradient_s"] = t_grad_rev
    rec["reversible_gradient_over_forward"] = t_grad_rev / t_fwd
    rec["ftle_gradient_s"] = t_fgrad
    rec["ftle_gradient_over_forward_tangent"] = t_fgrad / t_fwd_tan
    rec["reversible_ftle_gradient_s"] = t_fgrad_rev
    rec["reversible_ftle_gradient_over_forward_tangent"] = t_fgrad_rev / t_fwd_tan
    for name, base in (("gradient", t_fwd), ("ftle_gradient", t_fwd_tan)):
        r = one[name]
        rec[f"one_segment_{name}"] = None if r is None else {
            "s": r[0], "over_forward": r[0] / base, "workspace_bytes": r[1], "equals_checkpointed_bitwise": r[2]}
    return rec, None


def run_large(args, aw, wl, torch):
    """1e7 orbits, T = 1e6 (scaled by --t-scale), chunks of 1e5 steps."""
    import numpy as np
    T = max(1, int(round(1_000_000 * args.t_scale)))
    e = wl.c5(n_orbits=args.n_orbits, T=T)
    N = e.size
    chunk = min(T, 100_000)
    carry = torch.empty((aw.NCARRY, N), dtype=torch.float64, device="cuda")
    out = torch.empty((aw.NOUT, N), dtype=torch.float64, device="cuda")
    cls = torch.empty((N,), dtype=torch.uint8, device="cuda")
    aw.timing_read()
    aw.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    while k < T:
        k1 = min(T, k + chunk)
        aw.map_ensemble_steps(e, carry, k, k1, orbit_out=out if k1 == T else None, cls=cls if k1 == T else None)
        torch.cuda.synchronize()
        log(f"steps {k1}/{T} done ({time.perf_counter() - t0:.1f} s)")
        k = k1
    aw.timing_enable(False)
    kern_ms, launches = aw.timing_read()
    p0 = torch.empty((2, N), dtype=torch.float64, device="cuda")
    ic, _ = aw.generate_ic(e)
    spec = wl.c5_p0_image()
    cnt, sums, drop = aw.histogram2d(ic[3].contiguous(), ic[4].contiguous(), out[aw.OUT_DP2].contiguous(),
                                     spec.lo, spec.hi, spec.W, spec.H)
    phi, mu = aw.vdir_keys(out[aw.OUT_VX:aw.OUT_VZ + 1].contiguous())
    vcnt, _, vdrop = aw.histogram2d(phi, mu, None, (-np.pi, -1.0), (np.pi, 1.0), 512, 512, closed_upper=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c = cnt.cpu().numpy().view(np.uint32)
    rec = base_record(N * T / elapsed, 1, 0, elapsed * 1e3)
    rec["config"] = {"workload": f"c5: {N} orbits uniform on [0,2pi)^6 (seed 2), eps=5e-3, T={T}, S6 + tangent, "
                                 f"chunks of {chunk} steps, |P-P0|^2 image keyed on (px0,py0) 512x512 + V-direction "
                                 f"density 512x512", "n_orbits": N, "n_steps": T}
    rec["roofline"] = roofline(aw, e, kern_ms / max(launches, 1), "c5", steps_per_launch=chunk)
    rec["roofline"]["note"] = f"average over the {launches} chunk launches of {chunk} steps each"
    rec["hist_p0_count_sum"] = int(c.sum())
    rec["hist_p0_dropped"] = int(drop.cpu()[0])
    rec["hist_vdir_dropped"] = int(vdrop.cpu()[0])
    rec["chaotic_fraction"] = float(cls.float().mean())
    # sampled parity of the full-horizon run against the oracle
    if not args.no_cpu_baseline:
        import oracle
        idx = np.sort(np.random.default_rng(2).choice(N, 32, replace=False))
        ic_o = oracle.ic_box(e.box_lo, e.box_hi, e.seed_ic, idx=idx)
        t1 = time.perf_counter()
        out_o = oracle.ensemble("s6", e.eps, e.h, T, ic_o, oracle.w0(e.seed_tangent, idx=idx), nthreads=host_threads())
        log(f"oracle sample of 32 orbits: {time.perf_counter() - t1:.1f} s")
        g = out.cpu().numpy()[:, idx]
        reg = out_o[2] < 1.5
        err = np.abs(g[0] - out_o[0]) / np.maximum(1, np.abs(out_o[0]))
        rec["sample_parity"] = {"orbits": 32, "regular": int(reg.sum()),
                                "max_rel_err_L_regular": float(np.max(err[reg])),
                                "median_rel_err_L_regular": float(np.median(err[reg])),
                                "per_orbit": [{"n": int(idx[k]), "chi_oracle": float(out_o[2, k]),
                                               "rel_err_L": float(err[k]),
                                               "rel_err_dP2": float(abs(g[6, k] - out_o[6, k]) /
                                                                    max(1e-9, abs(out_o[6, k])))}
                                              for k in range(32)],
                                "class_disagreements": int(np.sum((g[2] > 2) != (out_o[2] > 2)))}
        # How well FP64 determines these indicators at this horizon: the oracle
        # against itself with every initial momentum moved by one ulp.
        ic_p = ic_o.copy()
        ic_p[3:] = np.nextafter(ic_p[3:], np.inf)
        out_p = oracle.ensemble("s6", e.eps, e.h, T, ic_p, oracle.w0(e.seed_tangent, idx=idx),
                                nthreads=host_threads())
        sL = np.abs(out_p[0] - out_o[0]) / np.maximum(1, np.abs(out_o[0]))
        sP = np.abs(out_p[6] - out_o[6]) / np.maximum(1e-9, np.abs(out_o[6]))
        rec["sample_parity"]["oracle_one_ulp_sensitivity"] = {
            "perturbation": "initial momenta moved by one ulp (oracle vs oracle)",
            "max_rel_L_regular": float(np.max(sL[reg])), "median_rel_L_regular": float(np.median(sL[reg])),
            "max_rel_dP2": float(np.max(sP)), "median_rel_dP2": float(np.median(sP))}
        # A regular orbit beyond the 1e-6 bar must lie within 4 times its own
        # one-ulp spread: the largest change of the oracle's L when any one of
        # the six initial coordinates moves by one ulp either way (12 runs).
        beyond = []
        for k in np.flatnonzero(reg & (err > 1e-6)):
            moved = np.repeat(ic_o[:, k:k + 1], 12, axis=1)
            for a in range(6):
                moved[a, 2 * a] = np.nextafter(ic_o[a, k], -np.inf)
                moved[a, 2 * a + 1] = np.nextafter(ic_o[a, k], np.inf)
            w0k = np.repeat(oracle.w0(e.seed_tangent, idx=idx[k:k + 1]), 12, axis=1)
            out_m = oracle.ensemble("s6", e.eps, e.h, T, moved, w0k, nthreads=host_threads())
            spread = float(np.max(np.abs(out_m[0] - out_o[0, k])) / max(1.0, abs(out_o[0, k])))
            beyond.append({"n": int(idx[k]), "rel_err_L": float(err[k]), "one_ulp_spread_L": spread,
                           "within_4x_spread": bool(err[k] <= 4 * spread)})
            log(f"orbit {idx[k]}: |GPU - oracle| {err[k]:.3g}, oracle one-ulp spread {spread:.3g}")
        rec["sample_parity"]["regular_beyond_1e-6"] = beyond
        rec["sample_parity"]["regular_within_1e-6_or_4x_own_spread"] = all(b["within_4x_spread"] for b in beyond)
    return rec, e


def run_sphere(args, aw, wl, torch):
    """The paper's Fig. 2 experiment (section "Main results"): eps = 1,
    E = 400, N = 1e8 orbits with the direction of P uniform on the momentum
    sphere and X uniform on the torus, propagated for Delta t = 50 T (5000
    steps; --t-scale 2 gives the paper's other window, 100 T), reduced to the
    density F of the direction of V (1024 x 512).  The paper propagates the
    state only, so the tangent is off here (the metric of
    this record is map-steps/s without the tangent).  fig3: E = 15, a zoom
    window with the stay-in-area selection."""
    if args.workload == "fig2":
        e = wl.fig2(n_orbits=args.n_orbits if args.n_orbits != 10_000_000 else 100_000_000)
        spec = wl.sphere_image(1024, 512)
    else:
        e = wl.fig3_zoom(n_orbits=args.n_orbits if args.n_orbits != 10_000_000 else 20_000_000)
        spec = wl.sphere_image(512, 512, e.window)
    e = dataclasses.replace(e, n_steps=max(1, int(round(e.n_steps * args.t_scale))))   # 2: Delta t = 100 T
    N, T = e.size, e.n_steps
    small = dataclasses.replace(e, n_steps=10, n_orbits=min(N, 1_000_000))
    aw.indicator_image(small, spec)
    torch.cuda.synchronize()
    aw.timing_read()
    aw.timing_enable(True)
    t0 = time.perf_counter()
    img, cnt, _ = aw.indicator_image(e, spec)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    aw.timing_enable(False)
    kern_ms, launches = aw.timing_read()
    log(f"{args.workload}: {N} orbits x {T} steps in {elapsed:.2f} s")
    import numpy as np
    c = cnt.cpu().numpy().view(np.uint32)
    F = img.cpu().numpy()
    rec = base_record(N * T / elapsed, 1, 1, elapsed * 1e3)
    rec["metric"] = "orbit map-steps/sec (state only, as in the paper's experiment)"
    rec["config"] = {"workload": f"{args.workload}: E={e.energy}, eps=1, N={N}, T={T} (Delta t = {T / 100:g} T), "
                                 f"window={list(e.window)}, stay_in_window={e.stay_in_window}, "
                                 f"F image {spec.W}x{spec.H}", "n_orbits": N, "n_steps": T}
    rec["roofline"] = roofline(aw, e, kern_ms / max(launches, 1), args.workload)
    rec["wall_s"] = elapsed
    rec["paper_wall_s"] = 45 * 60.0
    rec["paper_hardware"] = "NVIDIA Tesla M2050, FP64 (section Main results: 45 minutes per experiment)"
    rec["binned"] = int(c.sum())
    rec["median_density_over_uniform"] = float(np.median(F) * 4 * np.pi) if args.workload == "fig2" else None
    return rec, None


def run_diffusion(args, aw, wl, torch):
    """Fig. 4 (section "Main results"): N = 3.2e4 orbits injected at
    W = (sqrt E, sqrt E, 0), E = 15, F accumulated over consecutive windows of
    Delta t = 50 T (5000 steps).  The paper runs 1e9 steps per orbit (24 h on a
    Tesla M2050); this record runs --windows windows and reports the rate, the
    time the full horizon would take at that rate, and how far the cloud has
    spread.  At one lane per orbit the ensemble fills only 500 waves; by
    default the library runs it two lanes per orbit (1000 waves), and
    --lanes-per-orbit 1 times the one-lane kernel (blocks of 64 lanes, to
    spread it over as many CUs as possible)."""
    import numpy as np
    n_win = args.windows
    e = wl.fig4_cloud()
    N = e.n_orbits
    w = math.pi / 4
    spec = aw.ImageSpec(kind="hist_vdir", W=512, H=512, lo=(w - 0.5, -0.5), hi=(w + 0.5, 0.5))
    carry = torch.empty((aw.NCARRY, N), dtype=torch.float64, device="cuda")
    counts = torch.zeros((512, 512), dtype=torch.int32, device="cuda")
    tun = aw.Tuning(block=64, lanes_per_orbit=args.lanes_per_orbit)
    aw.window_density(e, carry, 0, 1, 10, spec, torch.zeros_like(counts), tuning=tun)   # loads the kernel
    aw.timing_read()
    aw.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    spread = []
    while done < n_win:
        k = min(50, n_win - done)
        aw.window_density(e, carry, done * wl.DT50, k, wl.DT50, spec, counts, tuning=tun)
        torch.cuda.synchronize()
        done += k
        P = carry[3:6].cpu().numpy()
        d = np.arctan2(P[1], P[0]) - w
        spread.append(float(np.std(d)))
        log(f"windows {done}/{n_win} ({time.perf_counter() - t0:.1f} s), spread of phi(P) {spread[-1]:.4f}")
    elapsed = time.perf_counter() - t0
    aw.timing_enable(False)
    kern_ms, launches = aw.timing_read()
    steps = n_win * wl.DT50
    rate = N * steps / elapsed
    rec = base_record(rate, 1, 0, elapsed * 1e3)
    rec["metric"] = "orbit map-steps/sec (state only, as in the paper's experiment)"
    rec["config"] = {"workload": f"fig4: E=15, eps=1, N={N} cloud at W=(sqrt E, sqrt E, 0), sigma_v=0.01, "
                                 f"{n_win} windows of 50 T (5000 steps), F zoom 512x512 around W",
                     "n_orbits": N, "n_steps": steps, "lanes_per_orbit": args.lanes_per_orbit or "auto"}
    rec["roofline"] = roofline(aw, e, kern_ms / max(launches, 1), "fig4", steps_per_launch=wl.DT50)
    rec["wall_s"] = elapsed
    rec["projected_s_for_1e9_steps"] = N * 1e9 / rate
    rec["paper_wall_s"] = 24 * 3600.0
    rec["paper_hardware"] = "NVIDIA Tesla M2050, FP64 (section Main results: 24 hours for 1e9 steps per orbit)"
    rec["binned_total"] = int(counts.cpu().numpy().view(np.uint32).sum())
    rec["phi_spread_by_50_windows"] = spread
    return rec, None


def run_nsweep(args, aw, wl, torch):
    """Throughput against N at T = 1e4 (orbits uniform on the 6-torus, eps =
    5e-3, S6 + tangent): one wave per SIMD is 65 536 orbits."""
    sizes = [1_000, 4_000, 16_000, 32_000, 65_536, 131_072, 262_144, 524_288, 1_048_576, 3_000_000, 10_000_000]
    T = 10_000
    fma, mul, add = aw.step_op_counts("s6", True)
    flop = 2 * fma + mul + add
    rows = []
    tot_steps, tot_s = 0, 0.0
    for n in sizes:
        e = wl.c5(n_orbits=n, T=T)
        aw.map_ensemble(dataclasses.replace(e, n_steps=10), want_class=False)
        torch.cuda.synchronize()
        aw.timing_read()
        aw.timing_enable(True)
        t0 = time.perf_counter()
        aw.map_ensemble(e, want_class=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        aw.timing_enable(False)
        kms, _ = aw.timing_read()
        rate = n * T / wall
        rows.append({"n_orbits": n, "waves_per_simd": n / 64 / 1024, "wall_s": wall, "kernel_ms": kms,
                     "map_steps_per_s": rate, "kernel_tflops": flop * n * T / (kms * 1e-3) / 1e12,
                     "frac_of_peak": flop * n * T / (kms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS})
        tot_steps += n * T
        tot_s += wall
        log(f"N={n}: {rate:.4g} map-steps/s, {rows[-1]['frac_of_peak'] * 100:.1f}% of peak")
    rec = base_record(tot_steps / tot_s, 1, 1, tot_s * 1e3)
    rec["config"] = {"workload": "N sweep: 1e3..1e7 orbits uniform on [0,2pi)^6 (seed 2), eps=5e-3, T=1e4, "
                                 "S6 + tangent, one launch per N", "n_steps": T}
    rec["sweep"] = rows
    return rec, None


def run_peak(args, aw, wl, torch):
    """Independent-chain FP64 FMA probe: the rate the SIMDs reach on pure
    v_fma_f64 issue, and the shader clock under that load."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1107_4107_amd", "libaw_probe.so"))
    lib.awp_fma_peak.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    lib.awp_fma_peak.restype = ctypes.c_int
    torch.cuda.synchronize()
    rows = []
    for w in (1, 2, 4, 8):
        out = (ctypes.c_double * 5)()
        rc = lib.awp_fma_peak(w, 2_000_000 // w, out)
        if rc != 0:
            raise RuntimeError(f"FMA probe failed with code {rc}")
        rows.append({"waves_per_simd": w, "ms": out[0], "tflops": out[1], "shader_clock_ghz": out[2] / 1e9,
                     "wall_clock_mhz": out[3] / 1e6, "waves": int(out[4]),
                     "tflops_at_2p4ghz_equiv": out[1] * 2.4e9 / out[2] if out[2] > 0 else None})
        log(f"probe {w} waves/SIMD: {out[1]:.2f} TFLOP/s at {out[2] / 1e9:.3f} GHz")
    best = max(rows, key=lambda r: r["tflops"])
    rec = base_record(best["tflops"], 1, 1, best["ms"])
    rec.update({"metric": "FP64 FLOP/s of independent FMA chains (achievable vector peak)", "unit": "TFLOP/s"})
    rec["config"] = {"workload": "FMA probe: 8 independent v_fma_f64 chains per lane, 1..8 waves per SIMD"}
    rec["probe"] = rows
    rec["published_peak_tflops"] = FP64_PEAK_TFLOPS
    return rec, None


def run_forms(args, aw, wl, torch):
    """Integrators compared on the eps = 1e-2, 512 x 512 (px, py) slice with
    pz0 = 1, T = 1e4: throughput, and the energy error |dE| (median and 99th
    percentile over the slice) at the paper's h and at 2h, with T halved at 2h
    so that both cover the same time."""
    import numpy as np
    rows = []
    for form in ("stdmap", "s2", "s4", "s6", "y6"):
        for hs in (1.0, 2.0):
            T = int(10_000 / hs)
            e = dataclasses.replace(wl.slice_ensemble(1e-2, 512, T, map_form=form, pz0=1.0), h=aw.H_PAPER * hs)
            aw.map_ensemble(dataclasses.replace(e, n_steps=10), want_class=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = aw.map_ensemble(e, want_class=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            dE = np.abs(r.orbit_out[aw.OUT_DE].cpu().numpy())
            fma, mul, add = aw.step_op_counts(form, True)
            rows.append({"form": form, "h_over_paper_h": hs, "n_steps": T, "map_steps_per_s": e.size * T / wall,
                         "kicks_per_step": {"stdmap": 1, "s2": 1, "s4": 3, "s6": 9, "y6": 7}[form],
                         "flop_per_step": 2 * fma + mul + add, "wall_s": wall,
                         "dE_median": float(np.median(dE)), "dE_p99": float(np.quantile(dE, 0.99))})
            log(f"{form} h x{hs:g}: {rows[-1]['map_steps_per_s']:.4g} steps/s, |dE| median "
                f"{rows[-1]['dE_median']:.3e}, p99 {rows[-1]['dE_p99']:.3e}")
    tot = sum(r["n_steps"] * 512 * 512 for r in rows)
    rec = base_record(tot / sum(r["wall_s"] for r in rows), 1, 1, sum(r["wall_s"] for r in rows) * 1e3)
    rec["config"] = {"workload": "integrator comparison: eps=1e-2, 512x512 (px,py) slice with pz0=1, "
                                 "t = 1e4 h, tangent on, at h and 2h"}
    rec["forms"] = rows
    return rec, None


def run_energy(args, aw, wl, torch):
    """The energy error |dE| = |H(X_T, P_T) - H(X_0, P_0)| of S6 at the
    paper's h on each configuration's eps and on the paper's two energies
    (E = 400 on the whole sphere, Fig. 2; E = 15, Figs. 3-4), and at E = 15
    also S6 at h/2 and Y6 at h: median, 99th percentile and maximum over the
    ensemble, and the share under the paper's 1e-8 (section "Computational
    method").  The paper's integrator is not the one built here, so this is
    reported, not a gate."""
    import numpy as np
    cases = [("c2 eps=1e-3, 512^2 slice", wl.slice_ensemble(1e-3, 512, 10_000)),
             ("c4 eps=1e-2, 512^2 slice", wl.slice_ensemble(1e-2, 512, 10_000)),
             ("c5 eps=5e-3, 1e6 box orbits", wl.c5(n_orbits=1_000_000, T=10_000)),
             ("Fig. 2: E=400, eps=1, whole sphere, 1e6 orbits", wl.fig2(n_orbits=1_000_000)),
             ("Figs. 3-4: E=15, eps=1, whole sphere, 1e6 orbits", wl.sphere_ensemble(15.0, 1_000_000, wl.DT50)),
             ("Fig. 4 cloud: E=15, eps=1, 3.2e4 orbits at W", wl.fig4_cloud(n_orbits=32_000, T=wl.DT50)),
             ("Figs. 3-4 at h/2 (same time span)",
              dataclasses.replace(wl.sphere_ensemble(15.0, 1_000_000, 2 * wl.DT50), h=aw.H_PAPER / 2)),
             ("Figs. 3-4 with Y6 at h", dataclasses.replace(wl.sphere_ensemble(15.0, 1_000_000, wl.DT50),
                                                            map_form="y6"))]
    rows = []
    t_all, steps_all = 0.0, 0
    for name, e in cases:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = aw.map_ensemble(e, want_class=False)
        torch.cuda.synchronize()
        t_all += time.perf_counter() - t0
        steps_all += e.size * e.n_steps
        dE = np.abs(r.orbit_out[aw.OUT_DE].cpu().numpy())
        dE = dE[np.isfinite(dE)]
        rows.append({"case": name, "n_orbits": int(e.size), "n_steps": int(e.n_steps), "eps": e.eps,
                     "dE_median": float(np.median(dE)), "dE_p99": float(np.quantile(dE, 0.99)),
                     "dE_max": float(dE.max()), "share_below_1e-8": float(np.mean(dE < 1e-8))})
        log(f"{name}: |dE| median {rows[-1]['dE_median']:.3e}, p99 {rows[-1]['dE_p99']:.3e}, "
            f"max {rows[-1]['dE_max']:.3e}, {100 * rows[-1]['share_below_1e-8']:.2f}% under 1e-8")
    rec = base_record(steps_all / t_all, 1, 1, t_all * 1e3)
    rec["config"] = {"workload": "energy error of S6 at h = 0.01 T on the configurations' eps and at E = 15, 400; "
                                 "at E = 15 also S6 at h/2 and Y6"}
    rec["energy"] = rows
    return rec, None


def run_sweep(args, aw, wl, torch):
    """Chaotic fraction (chi > 2) against eps on the literal slice and on the
    pz0 = 1 companion (256 x 256, T = 3e4, 16 eps values), each slice as one
    batched launch; the slope of log(fraction) against log(eps) is compared
    with the sqrt(eps) web-volume scaling of the model section."""
    import numpy as np
    rec = None
    out = {}
    t_all = 0.0
    for pz0 in (0.0, 1.0):
        ens = wl.eps_sweep(pz0=pz0)
        spec = aw.ImageSpec(kind="ic_grid", field=aw.OUT_CHI, W=0, H=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        imgs, cnts, _ = aw.indicator_images(ens, spec, want_counts=True)
        torch.cuda.synchronize()
        t_all += time.perf_counter() - t0
        eps = np.array([e.eps for e in ens])
        frac = np.array([int(c.cpu().numpy().view(np.uint32)[0]) for c in cnts]) / (ens[0].nx * ens[0].ny)
        ok = frac > 0
        slope = float(np.polyfit(np.log(eps[ok]), np.log(frac[ok]), 1)[0]) if ok.sum() >= 3 else None
        out[f"pz0={pz0:g}"] = {"eps": eps.tolist(), "chaotic_fraction": frac.tolist(),
                               "loglog_slope": slope}
        log(f"pz0={pz0}: fractions {np.array2string(frac, precision=4)} slope {slope}")
    steps = 2 * sum(e.size * e.n_steps for e in wl.eps_sweep())
    rec = base_record(steps / t_all, 1, 0, t_all * 1e3)
    rec["config"] = {"workload": "eps sweep: 16 eps log-spaced 1e-4..1e-1, 256x256 (px,py) slice, T=3e4, "
                                 "S6 + tangent, literal slice and pz0=1 companion, one batched launch each",
                     "map_steps": steps}
    rec["sweep"] = out
    rec["paper_claim"] = "web volume ~ sqrt(eps) (model section): log-log slope 0.5"
    return rec, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "fig2", "fig3", "fig4", "sweep",
                                                             "nsweep", "peak", "forms", "energy"])
    ap.add_argument("--windows", type=int, default=200, help="fig4: number of 50 T windows")
    ap.add_argument("--t-scale", type=float, default=1.0,
                    help="c3/c5/fig2/fig3: scale the horizons (fig2, fig3: 2 gives Delta t = 100 T)")
    ap.add_argument("--n-orbits", type=int, default=10_000_000, help="c5: ensemble size")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-1core", action="store_true",
                    help="leave out the oracle on one host thread (cpu_baseline_1core)")
    ap.add_argument("--no-c5-chunk", action="store_true",
                    help="c2: leave out the sub-record of one 1e5-step chunk of the 1e7-orbit ensemble")
    ap.add_argument("--no-sub-records", action="store_true",
                    help="c2: leave out the sub-records of the c4 gradients and of the c3 batch at horizons x0.1")
    ap.add_argument("--block", type=int, default=0, help="lanes per block; 0 = the library's automatic choice")
    ap.add_argument("--opl", type=int, default=1)
    ap.add_argument("--unroll", type=int, default=1)
    ap.add_argument("--lanes-per-orbit", type=int, default=0, choices=[0, 1, 2],
                    help="fig4: lanes per orbit of the window launches (0 = the library's choice)")
    ap.add_argument("--no-one-segment", action="store_true",
                    help="c4: leave out the one-segment gradients (126 GB and 252 GB of workspace)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the ensemble path has no multi-GPU mode (orbits are "
              "independent, so ensembles shard by orbit ranges; nothing is run across GPUs here).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1107_4107_amd as aw
    from paper_1107_4107_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_mib} MiB done")
        del src, dst
    runner = {"c1": run_slice, "c2": run_slice, "c3": run_batched, "c4": run_adjoint, "c5": run_large,
              "fig2": run_sphere, "fig3": run_sphere, "fig4": run_diffusion, "sweep": run_sweep,
              "nsweep": run_nsweep, "peak": run_peak, "forms": run_forms,
              "energy": run_energy}
    rec, ens = runner[args.workload](args, aw, wl, torch)
    if args.workload == "c2" and not args.no_c5_chunk:
        rec["c5_chunk"] = run_c5_chunk(aw, wl, torch)
    if args.workload == "c2" and not args.no_sub_records:
        rec["c4_gradients"] = sub_record(lambda: c4_summary(args, aw, wl, torch))
        rec["c3_batch_t0.1"] = sub_record(lambda: c3_summary(args, aw, wl, torch))
    rec.setdefault("cpu_baseline", None)
    if ens is not None and not args.no_cpu_baseline and args.workload in ("c1", "c2", "c5"):
        threads = host_threads()
        log(f"cpu baseline on {threads} threads ...")
        rec["cpu_baseline"] = cpu_baseline(ens, args.cpu_seconds, threads)
        rec["speedup_vs_oracle"] = rec["value"] / rec["cpu_baseline"]["value"]
        if not args.no_cpu_1core:
            log("cpu baseline on 1 thread ...")
            rec["cpu_baseline_1core"] = cpu_baseline(ens, args.cpu_seconds, 1)
            rec["speedup_vs_oracle_1core"] = rec["value"] / rec["cpu_baseline_1core"]["value"]
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
