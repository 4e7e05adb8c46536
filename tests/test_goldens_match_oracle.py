"""The stored parity sets under tests/golden/ are the current oracle's values:
a few of their orbits are run again here, on the CPU, from the same inputs,
and must come out bit for bit (the oracle is deterministic and its build
variants agree bitwise).  A change to the oracle's arithmetic shows up here
first, and the stored values must then be written again with
tests/golden/make_goldens.py."""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
H = 0.01 * 2.0 * np.pi
TWO_PI = 2.0 * np.pi


def _golden(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"missing {path}")
    return np.load(path)


def test_c2_subgrid_values(orc):
    g = _golden("c2_slice_1024_T1e5_stride4.npz")
    k = np.array([0, 777, 20_001, 65_535])
    idx = g["idx"][k]
    ic = orc.ic_grid2((3, 4), (0.0, 0.0), (TWO_PI, TWO_PI), 1024, 1024, [0] * 6, idx=idx)
    out = orc.ensemble("s6", float(g["eps"]), H, int(g["T"]), ic, orc.w0(0, idx=idx))
    for row, name in ((0, "L"), (2, "chi"), (6, "dP2"), (7, "J")):
        np.testing.assert_array_equal(out[row], g[name][k], err_msg=name)


def test_c2_classes_agree_with_the_subgrid(orc):
    full = _golden("c2_slice_1024_T1e5_classes.npz")
    sub = _golden("c2_slice_1024_T1e5_stride4.npz")
    bits = np.unpackbits(full["class_bits"], bitorder="little")[:1024 * 1024].astype(bool)
    np.testing.assert_array_equal(bits[sub["idx"]], sub["chi"] > 2.0)
    # the stored band entries are the points with chi in [1.4, 3.0]
    assert np.all((full["band_chi"] >= 1.4) & (full["band_chi"] <= 3.0))
    on_sub = np.isin(full["band_idx"], sub["idx"])
    pos = np.searchsorted(sub["idx"], full["band_idx"][on_sub])
    np.testing.assert_array_equal(full["band_chi"][on_sub], sub["chi"][pos])


def test_c5_values_and_spread(orc):
    g = _golden("c5_box_orbits0-4095_T1e6.npz")
    sp = _golden("c5_box_orbits0-4095_T1e6_one_ulp_spread.npz")["spread"]
    idx = np.array([3, 4094])
    ic = orc.ic_box([0.0] * 6, [TWO_PI] * 6, int(g["seed_ic"]), idx=idx)
    w0 = orc.w0(0, idx=idx)
    eps, T = float(g["eps"]), int(g["T"])
    out = orc.ensemble("s6", eps, H, T, ic, w0)
    np.testing.assert_array_equal(out, g["out"][:, idx])
    # one orbit's spread: the 12 one-ulp moves of its initial coordinates
    n = 3
    moved = np.repeat(ic[:, :1], 12, axis=1)
    for a in range(6):
        moved[a, 2 * a] = np.nextafter(ic[a, 0], -np.inf)
        moved[a, 2 * a + 1] = np.nextafter(ic[a, 0], np.inf)
    om = orc.ensemble("s6", eps, H, T, moved, np.repeat(w0[:, :1], 12, axis=1))
    np.testing.assert_array_equal(np.max(np.abs(om - out[:, :1]), axis=1), sp[:, n])


def test_c4_values(orc):
    g = _golden("c4_grad_512_T1e4.npz")
    k = np.array([0, 255])
    idx = g["idx"][k]
    ic = orc.ic_grid2((3, 4), (0.0, 0.0), (TWO_PI, TWO_PI), 512, 512, [0] * 6, idx=idx)
    J, dJ = orc.J_grad_ensemble("s6", float(g["eps"]), H, int(g["T"]), ic)
    np.testing.assert_array_equal(J, g["J"][k])
    np.testing.assert_array_equal(dJ, g["dJ"][:, k])
    out = orc.ensemble("s6", float(g["eps"]), H, int(g["T"]), ic, orc.w0(0, idx=idx))
    assert np.all(out[2] < 1.5)          # drawn among the regular orbits


def test_sweep_values(orc):
    g = _golden("sweep_pz1_256_T3e4_stride2.npz")
    k = np.array([0, 5000, 16_383])
    idx = g["idx"][k]
    for e in (0, 15):
        ic = orc.ic_grid2((3, 4), (0.0, 0.0), (TWO_PI, TWO_PI), 256, 256, [0, 0, 0, 0, 0, float(g["pz0"])], idx=idx)
        chi = orc.ensemble("s6", float(g["eps"][e]), H, int(g["T"]), ic, orc.w0(0, idx=idx))[2]
        bits = np.unpackbits(g["class_bits"][e], bitorder="little")[:g["idx"].size].astype(bool)
        np.testing.assert_array_equal(chi > 2.0, bits[k])
