"""Autotuner of the propagation launch shape.

Times short probes of an ensemble (the same descriptor with a reduced number
of steps) under every candidate (block, orbits per lane, unroll) with the
library's HIP-event kernel timing, keeps the fastest, and caches the choice in
a JSON file keyed by device, library build, single launch or batch, map form,
tangent flag and ensemble-size bucket.  A batch runs as one persistent launch,
which takes blocks of at most 256 lanes and does not unroll, so a batch is
tuned over block and orbits per lane only.  Results are bitwise independent
of the choice, so tuning never changes numbers, only speed.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
import os
import sys
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import Ensemble, Tuning, _abi, map_ensembles, timing_enable, timing_read

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "arnoldweb_tuning.json")
CANDIDATES: Tuple[Tuple[int, int, int], ...] = tuple(
    (b, o, u) for b in (64, 128, 256, 512) for o in (1, 2) for u in (1, 2))
# The persistent launch of a batch: blocks above 256 lanes run as 256, and the
# step loop is not unrolled.
BATCH_CANDIDATES: Tuple[Tuple[int, int, int], ...] = tuple((b, o, 1) for b in (64, 128, 256) for o in (1, 2))

_LIB_ID = None


def _lib_id() -> str:
    """Identity of the library build: size and a hash of libaw.so."""
    global _LIB_ID
    if _LIB_ID is None:
        with open(_abi.LIB_PATH, "rb") as f:
            data = f.read()
        _LIB_ID = f"{len(data)}:{hashlib.sha1(data).hexdigest()[:12]}"
    return _LIB_ID


def _key(ens: Ensemble, n_total: int, batch: bool) -> str:
    name = torch.cuda.get_device_name(torch.cuda.current_device()).replace("|", "/")
    bucket = 1 << max(0, int(math.log2(max(1, n_total))))
    return (f"{name}|lib={_lib_id()}|{'batch' if batch else 'single'}|form={ens.map_form}|"
            f"tangent={int(ens.tangent)}|N~{bucket}")


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except Exception:
        return {}


def _save(path: str, data: Dict[str, dict]) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def probe_time(ens_list: Sequence[Ensemble], tuning: Tuning, reps: int = 3) -> float:
    """Median kernel milliseconds of the propagation for a launch shape."""
    map_ensembles(list(ens_list), want_class=False, tuning=tuning)  # warm-up
    torch.cuda.synchronize()
    timing_read()
    times = []
    for _ in range(reps):
        timing_enable(True)
        map_ensembles(list(ens_list), want_class=False, tuning=tuning)
        torch.cuda.synchronize()
        timing_enable(False)
        ms, n = timing_read()
        times.append(ms / max(n, 1))
    times.sort()
    return times[len(times) // 2]


def autotune(ens_list: Sequence[Ensemble], probe_steps: int = 200, cache: Optional[str] = DEFAULT_CACHE,
             force: bool = False, candidates=None, verbose: bool = False) -> Tuning:
    """Pick the fastest launch shape for one ensemble or a batch of them."""
    ens_list = list(ens_list)
    batch = len(ens_list) > 1
    if candidates is None:
        candidates = BATCH_CANDIDATES if batch else CANDIDATES
    n_total = sum(e.size for e in ens_list)
    key = _key(ens_list[0], n_total, batch)
    data = _load(cache) if cache else {}
    if not force and key in data:
        return Tuning(**data[key]["tuning"])
    probes = [dataclasses.replace(e, n_steps=min(e.n_steps, probe_steps)) for e in ens_list]
    results: List[Tuple[float, Tuple[int, int, int]]] = []
    for b, o, u in candidates:
        t = Tuning(block=b, orbits_per_lane=o, unroll=u)
        ms = probe_time(probes, t)
        results.append((ms, (b, o, u)))
        if verbose:
            print(f"autotune {key}: block={b} opl={o} unroll={u}: {ms:.3f} ms", file=sys.stderr, flush=True)
    results.sort()
    b, o, u = results[0][1]
    best = Tuning(block=b, orbits_per_lane=o, unroll=u)
    if cache:
        data[key] = {"tuning": dataclasses.asdict(best),
                     "probe_ms": {f"{c[0]},{c[1]},{c[2]}": ms for ms, c in results},
                     "probe_steps": probe_steps}
        _save(cache, data)
    return best
