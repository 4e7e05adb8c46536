"""The measurement and tuning tools on the GPU.

bench.py must print one JSON line with the fields its contract names (the
metric, the timing, the roofline of the dominant kernel and the oracle's CPU
rate), self-consistent; the autotuner must return one of its candidates,
cache it, and return the cached choice on the next call."""
import json
import os
import subprocess
import sys

import pytest

from gpu_util import gpu, need_gpu, print_case

pytestmark = gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def aw():
    need_gpu()
    import paper_1107_4107_amd as m
    return m


def test_bench_prints_its_contract_line(aw):
    print_case("bench contract")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "c1", "--steps", "2",
                        "--warmup", "1", "--cpu-seconds", "1"], capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 1, lines[:3]   # one JSON line on stdout, progress on stderr
    rec = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["steps"] == 2 and rec["warmup"] == 1
    assert rec["higher_is_better"] is True and rec["vs_baseline"] is None
    assert rec["dtype"] == "f64" and rec["unit"] == "map-steps/s"
    cfg = rec["config"]
    assert isinstance(cfg["workload"], str)
    steps = cfg["n_orbits"] * cfg["n_steps"]
    assert rec["value"] == pytest.approx(steps / (rec["ms_per_step"] * 1e-3), rel=1e-9)
    rf = rec["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["peak"] == 78.6 and rf["unit"] == "TFLOP/s"
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-12)
    # achieved = algorithmic flops per launch / the kernel's own duration
    assert rf["achieved"] == pytest.approx(rf["flop_per_map_step"] * steps / (rf["kernel_ms"] * 1e-3) / 1e12, rel=1e-9)
    cb = rec["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and isinstance(cb["sample"], str)


def test_autotuner_picks_caches_and_reuses(aw, tmp_path):
    print_case("autotune")
    from paper_1107_4107_amd import autotune, workloads as wl
    e = wl.slice_ensemble(1e-2, 64, 300)
    cache = str(tmp_path / "tune.json")
    cands = ((64, 1, 1), (256, 1, 1), (512, 2, 1))
    t = autotune.autotune([e], probe_steps=50, cache=cache, candidates=cands)
    assert (t.block, t.orbits_per_lane, t.unroll) in cands
    data = json.load(open(cache))
    assert len(data) == 1
    rec = next(iter(data.values()))
    assert set(rec["probe_ms"]) == {f"{b},{o},{u}" for b, o, u in cands}
    assert all(ms > 0 for ms in rec["probe_ms"].values())
    again = autotune.autotune([e], probe_steps=50, cache=cache, candidates=((128, 1, 1),))
    assert (again.block, again.orbits_per_lane, again.unroll) == (t.block, t.orbits_per_lane, t.unroll)
    # a batch runs as one persistent launch: tuned over its own candidates
    # (blocks up to 256, no unroll) and cached under its own key
    tb = autotune.autotune([e, wl.slice_ensemble(2e-2, 32, 300)], probe_steps=50, cache=cache)
    assert (tb.block, tb.orbits_per_lane, tb.unroll) in autotune.BATCH_CANDIDATES
    data = json.load(open(cache))
    keys = [k for k in data if "|batch|" in k]
    assert len(data) == 2 and len(keys) == 1
    assert set(data[keys[0]]["probe_ms"]) == {f"{b},{o},{u}" for b, o, u in autotune.BATCH_CANDIDATES}
