"""Shared helpers of the GPU parity tests."""
import numpy as np
import pytest

H = 0.01 * 2.0 * np.pi

gpu = pytest.mark.gpu


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def np_(t):
    return t.detach().cpu().numpy()


def assert_close(a, b, rel, floor=1.0, what=""):
    """|a - b| <= rel * max(floor, |b|) element by element."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tol = rel * np.maximum(floor, np.abs(b))
    bad = ~(np.abs(a - b) <= tol)
    if bad.any():
        i = np.flatnonzero(bad.ravel())[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {a.size} differ beyond rel {rel}; e.g. idx {i}: "
                             f"{a.ravel()[i]} vs {b.ravel()[i]}")


def class_agreement(chi_gpu, chi_orc, thr=2.0, band=(1.5, 2.5), min_frac=0.995):
    """Regular/chaotic classes agree on >= min_frac of the points and every
    disagreement has the oracle's chi inside the band around the threshold."""
    cg = chi_gpu > thr
    co = chi_orc > thr
    dis = cg != co
    frac = 1.0 - dis.mean()
    assert frac >= min_frac, f"class agreement {frac:.5f} < {min_frac}"
    out_band = dis & ~((chi_orc >= band[0]) & (chi_orc <= band[1]))
    assert not out_band.any(), f"{out_band.sum()} disagreements outside the band: chi_orc={chi_orc[out_band][:5]}"
    return frac


def print_case(*args):
    print("CASE", *args, flush=True)


def one_ulp_outputs(form, eps, T, ic, w0):
    """The oracle's outputs for every orbit (column of ic[6, n]) with one of its
    six initial coordinates moved by one ulp down or up: out[9, n, 12]."""
    import oracle
    n = ic.shape[1]
    moved = np.repeat(ic, 12, axis=1)
    for k in range(n):
        for a in range(6):
            moved[a, 12 * k + 2 * a] = np.nextafter(ic[a, k], -np.inf)
            moved[a, 12 * k + 2 * a + 1] = np.nextafter(ic[a, k], np.inf)
    out = oracle.ensemble(form, eps, H, T, moved, np.repeat(w0, 12, axis=1))
    return out.reshape(out.shape[0], n, 12)


def check_regular_rows(got, ref, rows, ic, w0, eps, T, form="s6", rel=1e-6, floors=None, factor=4.0,
                       max_frac=1e-3, what=""):
    """Per-orbit rows of regular orbits against the oracle: |a - b| <= rel *
    max(floor, |b|), with a floor per row (a number, or one per orbit).  An orbit that misses the bar must lie within `factor`
    times its own one-ulp spread (the largest change of the oracle's value when
    any one initial coordinate moves by one ulp either way: FP64 does not fix
    the value more closely than that), and such orbits must be rare (at most
    max_frac of the orbits, or one).  Returns (worst error within the bar,
    list of (orbit column, row, error, spread) of the orbits beyond it)."""
    floors = floors or {}
    worst, beyond = 0.0, []
    miss = {}
    for r in rows:
        scale = np.maximum(floors.get(r, 1.0), np.abs(ref[r]))
        err = np.abs(got[r] - ref[r]) / scale
        ok = err <= rel
        if ok.any():
            worst = max(worst, float(err[ok].max()))
        miss[r] = (np.flatnonzero(~ok), err, scale)
    cols = np.unique(np.concatenate([m[0] for m in miss.values()])) if miss else np.array([], dtype=int)
    # the count first: the one-ulp runs below cost 12 oracle runs per orbit
    assert cols.size <= max(1, int(max_frac * ref.shape[1])), \
        f"{what}: {cols.size} orbits beyond the bar, e.g. " + \
        ", ".join(f"row {r}: {np.sort(m[1][m[0]])[-3:]}" for r, m in miss.items() if m[0].size)
    if cols.size:
        print(f"{what}: {cols.size} orbits beyond {rel}; their one-ulp spreads ...", flush=True)
        spread_out = one_ulp_outputs(form, eps, T, ic[:, cols], w0[:, cols])
        pos = {c: k for k, c in enumerate(cols)}
        for r, (bad, err, scale) in miss.items():
            for c in bad:
                s = float(np.max(np.abs(spread_out[r, pos[c]] - ref[r, c])) / scale[c])
                beyond.append((int(c), r, float(err[c]), s))
                assert err[c] <= factor * s, f"{what} row {r} orbit {c}: error {err[c]:.3e} beyond {factor} x " \
                                             f"its one-ulp spread {s:.3e}"
    return worst, beyond


def check_rows_with_spread(got, ref, spread, rows, floors=None, rel=1e-6, factor=4.0, what=""):
    """As check_regular_rows, with every orbit's one-ulp spread given
    (spread[row, orbit], absolute, from the oracle): each value within rel of
    the oracle's, or within `factor` times its own spread.  Returns
    {row: (orbits beyond rel, largest error / spread among them)}."""
    floors = floors or {}
    report = {}
    for r in rows:
        scale = np.maximum(floors.get(r, 1.0), np.abs(ref[r]))
        err = np.abs(got[r] - ref[r]) / scale
        s = spread[r] / scale
        beyond = err > rel
        bad = beyond & ~(err <= factor * s)
        assert not bad.any(), f"{what} row {r}: {bad.sum()} orbits beyond {rel} and beyond {factor} x their one-ulp " \
                              f"spread, e.g. errors {err[bad][:4]} spreads {s[bad][:4]}"
        ratio = float(np.max(err[beyond] / s[beyond])) if beyond.any() else 0.0
        report[r] = (int(beyond.sum()), ratio)
    return report
