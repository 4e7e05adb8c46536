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
