"""Writes the oracle's expected values for the full-size parity tests.

Every number stored here comes from the CPU oracle (``oracle/``) run on the
same seeded synthetic inputs the GPU tests run; nothing is read from the HIP
library.  The inputs are restated below from their definitions (grid slices,
counter-based draws), so this script imports only the oracle and numpy.

Workloads (all M = 3, FP64, the sixth-order map S6, h = 0.01 * 2 pi -- section
"Computational method"; the model is eqs. 1-2):

  c2sub  eps = 1e-3, the 1024 x 1024 slice (px, py) in [0, 2 pi)^2 (left
         edges), x = y = z = pz = 0, T = 1e5, tangent start seed 0: L, chi,
         dP2 and J of every point of the stride-4 256 x 256 sub-grid.
  c2full the same slice, every point: the regular/chaotic class (chi > 2) of
         all 1 048 576 points as packed bits, with chi and L of every point
         whose chi lies in [1.4, 3.0] (so that every class disagreement can be
         placed against the band [1.5, 2.5]).
  c4     eps = 1e-2, the 512 x 512 slice, T = 1e4: 256 orbits drawn with
         numpy's default_rng(3) among those with oracle chi < 1.5; their J,
         the forward-mode dJ/d(x, y, z, px, py, pz, eps) and central finite
         differences of the oracle's J with an absolute step of 1e-6.
  c5     orbits 0..4095 of the 1e7-orbit ensemble uniform on [0, 2 pi)^6
         (SplitMix64 seed 2, counter 16 n + k), eps = 5e-3, T = 1e6: all nine
         per-orbit rows.
  c5spread  the same orbits' one-ulp spread: for every orbit and row, the
         largest change of the oracle's value when one initial coordinate
         moves by one ulp either way (12 runs per orbit; how far binary64
         fixes each value at this horizon).
  sweep  the pz0 = 1 companion slice of the 256 x 256 grid, T = 3e4, 16 eps
         values 10^(-4 + 3k/15), on its stride-2 128 x 128 sub-grid: packed
         class bits per eps, chi of every point in [1.4, 3.0], and the
         oracle's chaotic fractions and their log-log slope against eps.

Usage: python tests/golden/make_goldens.py [--only c4,c5,c5spread,sweep,c2sub,c2full]
       [--threads N] [--work DIR]
Chunks of the long runs are kept under --work so that an interrupted run
resumes where it stopped.  The oracle takes about 1e6 map steps per second
per core: on 7 cores c4 ~7 min, c5 ~10 min, c5spread ~2 h, sweep ~20 min,
c2sub ~16 min, c2full ~4 h.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402

H = 0.01 * 2.0 * np.pi
TWO_PI = 2.0 * np.pi
BAND_STORE = (1.4, 3.0)


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def slice_run(eps, n, T, pz0, idx, threads):
    ic = oracle.ic_grid2((3, 4), (0.0, 0.0), (TWO_PI, TWO_PI), n, n, [0, 0, 0, 0, 0, pz0], idx=idx)
    return oracle.ensemble("s6", eps, H, T, ic, oracle.w0(0, idx=idx), nthreads=threads)


def chunked(name, n_total, chunk, fn, work):
    """Run fn(idx) over [0, n_total) in chunks, caching each chunk's result."""
    parts = []
    for c0 in range(0, n_total, chunk):
        path = os.path.join(work, f"{name}_{c0:09d}.npy")
        if os.path.exists(path):
            parts.append(np.load(path))
            continue
        t0 = time.time()
        idx = np.arange(c0, min(n_total, c0 + chunk))
        out = fn(idx)
        np.save(path, out)
        parts.append(out)
        log(f"{name}: orbits {c0}..{idx[-1]} done in {time.time() - t0:.0f} s")
    return np.concatenate(parts, axis=1)


def band_entries(chi, L):
    sel = np.flatnonzero((chi >= BAND_STORE[0]) & (chi <= BAND_STORE[1]))
    return sel.astype(np.int64), chi[sel], L[sel]


def c2_subgrid(n=1024, stride=4):
    j, i = np.meshgrid(np.arange(0, n, stride), np.arange(0, n, stride), indexing="ij")
    return (j * n + i).ravel().astype(np.int64)


def make_c2sub(threads, work):
    n, T, eps = 1024, 100_000, 1e-3
    sub = c2_subgrid(n)
    out = chunked("c2sub", sub.size, 8192, lambda k: slice_run(eps, n, T, 0.0, sub[k], threads), work)
    np.savez_compressed(os.path.join(HERE, "c2_slice_1024_T1e5_stride4.npz"), eps=eps, n=n, T=T, stride=4,
                        idx=sub, L=out[0], chi=out[2], dP2=out[6], J=out[7])
    log(f"c2sub: chaotic fraction {np.mean(out[2] > 2.0):.6f} on {sub.size} points")


def make_c2full(threads, work):
    n, T, eps = 1024, 100_000, 1e-3
    out = chunked("c2", n * n, 65536, lambda idx: slice_run(eps, n, T, 0.0, idx, threads), work)
    chi, L = out[2], out[0]
    bi, bchi, bL = band_entries(chi, L)
    np.savez_compressed(os.path.join(HERE, "c2_slice_1024_T1e5_classes.npz"), eps=eps, n=n, T=T,
                        class_bits=np.packbits(chi > 2.0, bitorder="little"),
                        band_idx=bi, band_chi=bchi, band_L=bL)
    log(f"c2full: chaotic fraction {np.mean(chi > 2.0):.6f}, {bi.size} points in the stored band")


def make_c4(threads, work):
    n, T, eps = 512, 10_000, 1e-2
    out = chunked("c4", n * n, 65536, lambda idx: slice_run(eps, n, T, 0.0, idx, threads), work)
    reg = np.flatnonzero(out[2] < 1.5)
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(reg, size=256, replace=False))
    ic = oracle.ic_grid2((3, 4), (0.0, 0.0), (TWO_PI, TWO_PI), n, n, [0] * 6, idx=idx)
    J, dJ = oracle.J_grad_ensemble("s6", eps, H, T, ic, nthreads=threads)
    # Central differences of the oracle's own J, absolute step 1e-6 per
    # coordinate and on eps.
    step = 1e-6
    fd = np.empty((7, idx.size))
    w = oracle.w0(0, idx=idx)
    for a in range(7):
        Jpm = []
        for sgn in (1.0, -1.0):
            c = ic.copy()
            e = eps
            if a < 6:
                c[a] = c[a] + sgn * step
            else:
                e = eps + sgn * step
            Jpm.append(oracle.ensemble("s6", e, H, T, c, w, nthreads=threads)[7])
        fd[a] = (Jpm[0] - Jpm[1]) / (2.0 * step)
    np.savez_compressed(os.path.join(HERE, "c4_grad_512_T1e4.npz"), eps=eps, n=n, T=T, fd_step=step,
                        n_regular=reg.size, idx=idx.astype(np.int64), J=J, dJ=dJ, fd=fd)
    log(f"c4: {reg.size} regular orbits of {n * n}; 256 picked")


def make_c5(threads, work):
    T, eps, M = 1_000_000, 5e-3, 4096

    def run(idx):
        ic = oracle.ic_box([0.0] * 6, [TWO_PI] * 6, 2, idx=idx)
        return oracle.ensemble("s6", eps, H, T, ic, oracle.w0(0, idx=idx), nthreads=threads)

    out = chunked("c5", M, 512, run, work)
    np.savez_compressed(os.path.join(HERE, "c5_box_orbits0-4095_T1e6.npz"), eps=eps, T=T, seed_ic=2,
                        out=out)
    log(f"c5: {np.sum(out[2] < 1.5)} of {M} orbits regular (chi < 1.5)")


def one_ulp_spread(ic, w0, eps, T, threads):
    """For every orbit (column of ic[6, n]): the largest change of each of the
    oracle's nine output rows when one of its six initial coordinates moves by
    one ulp down or up (12 runs per orbit).  Returns spread[9, n] (absolute)."""
    n = ic.shape[1]
    base = oracle.ensemble("s6", eps, H, T, ic, w0, nthreads=threads)
    moved = np.repeat(ic, 12, axis=1)
    for k in range(n):
        for a in range(6):
            moved[a, 12 * k + 2 * a] = np.nextafter(ic[a, k], -np.inf)
            moved[a, 12 * k + 2 * a + 1] = np.nextafter(ic[a, k], np.inf)
    out = oracle.ensemble("s6", eps, H, T, moved, np.repeat(w0, 12, axis=1), nthreads=threads)
    return np.max(np.abs(out.reshape(9, n, 12) - base[:, :, None]), axis=2)


def make_c5spread(threads, work):
    T, eps, M = 1_000_000, 5e-3, 4096

    def run(idx):
        ic = oracle.ic_box([0.0] * 6, [TWO_PI] * 6, 2, idx=idx)
        return one_ulp_spread(ic, oracle.w0(0, idx=idx), eps, T, threads)

    spread = chunked("c5spread", M, 64, run, work)
    np.savez_compressed(os.path.join(HERE, "c5_box_orbits0-4095_T1e6_one_ulp_spread.npz"), eps=eps, T=T,
                        seed_ic=2, spread=spread)
    log(f"c5spread: median one-ulp spread of L {np.median(spread[0]):.3e}")


def make_sweep(threads, work):
    n, T, pz0, stride = 256, 30_000, 1.0, 2
    eps = np.array([10.0 ** (-4.0 + 3.0 * k / 15.0) for k in range(16)])
    sub = c2_subgrid(n, stride)
    bits, frac, band = [], [], []
    for k, e in enumerate(eps):
        out = chunked(f"sweep{k:02d}", sub.size, 8192,
                      lambda m, e=e: slice_run(e, n, T, pz0, sub[m], threads), work)
        chi = out[2]
        bits.append(np.packbits(chi > 2.0, bitorder="little"))
        frac.append(np.mean(chi > 2.0))
        bi, bchi, _ = band_entries(chi, out[0])
        band.append(np.stack([bi.astype(np.float64), bchi]))
    ok = np.array(frac) > 0
    slope = float(np.polyfit(np.log(eps[ok]), np.log(np.array(frac)[ok]), 1)[0])
    band_k = np.concatenate([np.full(b.shape[1], k) for k, b in enumerate(band)]).astype(np.int64)
    band_all = np.concatenate(band, axis=1)
    # band_idx indexes the sub-grid (idx[band_idx] is the orbit of the 256 x 256 grid)
    np.savez_compressed(os.path.join(HERE, "sweep_pz1_256_T3e4_stride2.npz"), eps=eps, n=n, T=T, pz0=pz0,
                        stride=stride, idx=sub, class_bits=np.stack(bits), fraction=np.array(frac),
                        loglog_slope=slope, band_eps=band_k, band_idx=band_all[0].astype(np.int64),
                        band_chi=band_all[1])
    log(f"sweep: fractions {np.round(frac, 5)}, slope {slope:.4f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="c4,c5,sweep,c2sub")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--work", default=os.path.join(ROOT, "_work", "golden_chunks"))
    a = ap.parse_args()
    os.makedirs(a.work, exist_ok=True)
    jobs = {"c2sub": make_c2sub, "c2full": make_c2full, "c4": make_c4, "c5": make_c5, "c5spread": make_c5spread,
            "sweep": make_sweep}
    for name in a.only.split(","):
        t0 = time.time()
        jobs[name](a.threads, a.work)
        log(f"{name} written in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
