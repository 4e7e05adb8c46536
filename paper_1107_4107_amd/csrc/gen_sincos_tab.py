"""Writes aw_sincos_tab.h: constants of the table-driven FP64 sin/cos of the
propagation and adjoint kernels.

The device routine reduces x modulo pi/2048: q = nearest integer to
2048 x/pi (by adding 1.5 * 2^52, whose low mantissa word then holds q in two's
complement), r = x - q pi/2048 by a two-part Cody-Waite step with fused
multiply-adds, so |r| <= pi/4096 (plus the rounding of q).  With
k = q mod 4096 and (S_k, C_k) = (sin, cos)(k pi/2048) read from a 4096-entry
table held in LDS,
    sin x = S_k cos r + C_k sin r,   cos x = C_k cos r - S_k sin r,
    sin r = r + r^3 c,               cos r = 1 + r^2 Q(r^2),
with c a single coefficient and Q of two: near-minimax fits in u = r^2 on
[0, (pi/4096 + 1e-8)^2] at 60 digits (mpmath Chebyshev interpolation).  The
table carries the signs of every quadrant, so no parity correction follows.
Its byte offset 16 k is the low word of t shifted left by 4 and cut to 16
bits.  pi/2048 is split as PI_A/2048 + PI_B/2048 (exact scalings of the
two-part pi).

The whole device sequence is replayed here in double precision with each
fused multiply-add rounded once (exactly, through mpmath), against mpmath's
sin and cos, over arguments up to 1e6 in magnitude and around the table's
interval edges; the errors are written into the header.  So is the error of
the kicks' z terms, cos^2 z = (1 + cos 2z)/2 and cos z sin z = sin(2z)/2, which
the device takes from the same table at the doubled angle: same reduction,
node 2q, and polynomials for sin(2r)/2 and cos(2r)/2 (device_zterms).

Run:  python gen_sincos_tab.py > aw_sincos_tab.h
"""
import random
import struct
import sys

import mpmath as mp

mp.mp.dps = 60
N_TAB = 4096
RMAX = mp.pi / 4096 + mp.mpf("1e-8")
MAGIC = 1.5 * 2.0 ** 52


def fit(g, n):
    poly, err = mp.chebyfit(g, [mp.mpf(0), RMAX ** 2], n, error=True)
    return [float(c) for c in poly[::-1]], err  # ascending powers of u


def g_sin(u):
    if u == 0:
        return mp.mpf(-1) / 6
    r = mp.sqrt(u)
    return (mp.sin(r) - r) / (u * r)


def g_cos(u):
    if u == 0:
        return mp.mpf(-1) / 2
    return (mp.cos(mp.sqrt(u)) - 1) / u


def fma(a, b, c):
    """a * b + c rounded once to double."""
    return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))


def lo32(t):
    return struct.unpack("<Q", struct.pack("<d", t))[0] & 0xFFFFFFFF


def device_sincos(x, tab, ps0, pc, inv, pa, pb):
    t = fma(x, inv, MAGIC)
    q = t - MAGIC
    r = fma(-q, pa, x)
    r = fma(-q, pb, r)
    k = ((lo32(t) << 4) & 0xFFFF) >> 4
    S, C = tab[2 * k], tab[2 * k + 1]
    u = r * r
    sr = fma(r * u, ps0, r)
    c = fma(pc[1], u, pc[0])
    cr = fma(u, c, 1.0)
    return fma(S, cr, C * sr), fma(C, cr, -(S * sr))


def device_zterms(z, tab, zs0, zc, inv, pa, pb):
    """The kicks' z terms (cos z sin z, cos^2 z) as the device computes them
    from the table at the doubled angle: the reduction of z is sincos_tab's
    (q, r), 2z = 2q pi/2048 + 2r picks node 2q mod 4096 (the same low word of
    t, shifted by 5 instead of 4), and two short polynomials in u = r^2 give
    sin(2r)/2 and cos(2r)/2.  Returns (cos z sin z, cos^2 z)."""
    t = fma(z, inv, MAGIC)
    q = t - MAGIC
    r = fma(-q, pa, z)
    r = fma(-q, pb, r)
    k = ((lo32(t) << 5) & 0xFFFF) >> 4
    S, C = tab[2 * k], tab[2 * k + 1]
    u = r * r
    sh = fma(r * u, zs0, r)
    ph = fma(zc[1], u, zc[0])
    ch = fma(u, ph, 0.5)
    return fma(S, ch, C * sh), fma(C, ch, fma(-S, sh, 0.5))


def g_zsin(u):
    if u == 0:
        return mp.mpf(-2) / 3
    r = mp.sqrt(u)
    return (mp.sin(2 * r) / 2 - r) / (u * r)


def g_zcos(u):
    if u == 0:
        return mp.mpf(-1)
    return (mp.cos(2 * mp.sqrt(u)) / 2 - mp.mpf(1) / 2) / u


def z_constants():
    """Coefficients of sin(2r)/2 = r + r^3 a and cos(2r)/2 = 1/2 + r^2 B(r^2)
    on the same reduced range, with their fit errors: (zs, zc, errzs, errzc)."""
    zs, errzs = fit(g_zsin, 1)
    zc, errzc = fit(g_zcos, 2)
    return zs, zc, errzs, errzc


def constants():
    """The table, the coefficients and the reduction constants, with the fit
    errors: (tab, ps, pc, inv, pa, pb, errs, errc)."""
    ps, errs = fit(g_sin, 1)
    pc, errc = fit(g_cos, 2)
    tab = []
    for k in range(N_TAB):
        a = k * mp.pi / 2048
        tab += [float(mp.sin(a)), float(mp.cos(a))]
    pi_a = float(mp.pi)
    pi_b = float(mp.pi - pi_a)
    pa, pb = pi_a / 2048.0, pi_b / 2048.0      # exact: division by a power of two
    inv = float(2048 / mp.pi)
    return tab, ps, pc, inv, pa, pb, errs, errc


def main():
    tab, ps, pc, inv, pa, pb, errs, errc = constants()
    rnd = random.Random(5)
    xs = [rnd.uniform(-7.0, 7.0) for _ in range(4000)]
    xs += [rnd.uniform(-1e6, 1e6) for _ in range(2000)]
    xs += [float((k + 0.5) * mp.pi / 2048) * (1 + s * 1e-15) for k in range(-4200, 4200, 7) for s in (-1, 1)]
    es = ec = 0.0
    for x in xs:
        s, c = device_sincos(x, tab, ps[0], pc, inv, pa, pb)
        es = max(es, abs(s - float(mp.sin(mp.mpf(x)))))
        ec = max(ec, abs(c - float(mp.cos(mp.mpf(x)))))
    # The kicks' z terms from the doubled angle, over the same arguments and
    # around the edges of the doubled angle's intervals.
    zsc, zcc, errzs, errzc = z_constants()
    zs = xs[:6000] + [float((k + 0.5) * mp.pi / 4096) * (1 + s * 1e-15) for k in range(-4200, 4200, 7) for s in (-1, 1)]
    ez2 = ezs = 0.0
    for z in zs:
        zsz, z2 = device_zterms(z, tab, zsc[0], zcc, inv, pa, pb)
        cz, sz = mp.cos(mp.mpf(z)), mp.sin(mp.mpf(z))
        ez2 = max(ez2, abs(z2 - float(cz * cz)))
        ezs = max(ezs, abs(zsz - float(cz * sz)))
    out = sys.stdout
    out.write("/* Generated by gen_sincos_tab.py -- do not edit. */\n#pragma once\n")
    out.write(f"/* sin r = r + r^3 c: 1 coefficient, fit error {mp.nstr(errs, 3)}; "
              f"cos r = 1 + r^2 Q(r^2): 2 coefficients, fit error {mp.nstr(errc, 3)}; |r| <= pi/4096 */\n")
    out.write(f"/* device sequence replayed with single-rounding FMAs over {len(xs)} arguments up to 1e6: "
              f"max abs error sin {es:.3e}, cos {ec:.3e} */\n")
    out.write(f"/* kick z terms from the doubled angle: sin(2r)/2 = r + r^3 a, fit error {mp.nstr(errzs, 3)}; "
              f"cos(2r)/2 = 1/2 + r^2 B(r^2), fit error {mp.nstr(errzc, 3)}; replayed over {len(zs)} arguments "
              f"up to 1e6: max abs error cos^2 z {ez2:.3e}, cos z sin z {ezs:.3e} */\n")
    out.write(f"#define AW_TAB_N {N_TAB}\n")
    out.write(f"static constexpr double AW_TSIN_C0 = {ps[0].hex()};\n")
    out.write("static constexpr double AW_TCOS_C[2] = {" + ", ".join(v.hex() for v in pc) + "};\n")
    out.write(f"static constexpr double AW_PI2K_A = {pa.hex()};\n")
    out.write(f"static constexpr double AW_PI2K_B = {pb.hex()};\n")
    out.write(f"static constexpr double AW_INV_PI2K = {inv.hex()};\n")
    out.write(f"static constexpr double AW_ZSIN_C0 = {zsc[0].hex()};\n")
    out.write("static constexpr double AW_ZCOS_C[2] = {" + ", ".join(v.hex() for v in zcc) + "};\n")
    out.write("/* (sin, cos)(k pi/2048), k = 0..4095, interleaved */\n")
    out.write("static constexpr double AW_TAB_SC[2 * AW_TAB_N] = {\n")
    for k in range(N_TAB):
        out.write(f"  {tab[2 * k].hex()}, {tab[2 * k + 1].hex()},\n")
    out.write("};\n")


if __name__ == "__main__":
    main()
