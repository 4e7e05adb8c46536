"""Builds libaw.so (the HIP library, gfx950) and libaw_probe.so (the FP64
peak and clock probe the benchmark uses) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libaw.so")
SOURCES = ["aw_api.hip", "aw_fwd.hip", "aw_hist.hip", "aw_adj.hip", "aw_ftle_adj.hip"]
PROBE_LIB = os.path.join(HERE, "libaw_probe.so")
PROBE_SOURCES = ["aw_probe.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # Packed FP32 instructions are kept out of the code objects.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return path


def command(out: str = LIB, extra=(), sources=SOURCES) -> list:
    srcs = [os.path.join(CSRC, s) for s in sources]
    return [hipcc(), *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, *srcs, "-o", out]


def _run(cmd, verbose: bool, what: str) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {what}")


def _compile(lib: str, sources, verbose: bool) -> str:
    """Compile each source to an object in parallel, then link the library."""
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="aw_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in sources]
        cmds = [[hipcc(), *flags, "-c", "-I", INCLUDE, "-I", CSRC, os.path.join(CSRC, s), "-o", o]
                for s, o in zip(sources, objs)]
        workers = max(1, min(len(cmds), (os.cpu_count() or 1)))
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(lambda c: _run(c, verbose, os.path.basename(c[-3])), cmds))
        tmp = lib + ".tmp"
        _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose,
             os.path.basename(lib))
        os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libaw.so and the probe into
    libaw_probe.so (always recompiles)."""
    _compile(PROBE_LIB, PROBE_SOURCES, verbose)
    return _compile(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
