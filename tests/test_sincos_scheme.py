"""The device sin/cos of the link phasors and the FP32 phase of the winding filter
(ah_device.hpp), checked on the CPU.

The constants are read from the header and each scheme is replayed with every
operation rounded to the working precision: float32 through numpy with fused
multiply-adds taken exactly in float64 and rounded once; float64 through mpmath
at 60 digits, rounded once per operation.  The double sin/cos (reduction by
multiples of pi in two fused multiply-adds, odd and even minimax polynomials,
sign flip for odd multiples) is replayed whole; of the float sin/cos, which ends
in the hardware sine and cosine, the reduction.  A mistyped coefficient or a
wrong sign shows up as an error far above the bounds stated in the header.
"""
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1809_00995_amd", "csrc", "ah_device.hpp")
NUM = re.compile(r"[-+]?\d+\.\d*(?:e[-+]?\d+)?f?")


def _constants(sig):
    src = open(HDR).read()
    start = src.index(f"void sincos_t({sig} x")
    body = src[src.index("{", start):src.index("\n}\n", start)]
    vals = [float(v.rstrip("f")) for v in NUM.findall(body)]
    # 1/pi, pi high, pi low, P (highest power first), Q (highest first), 1.0
    return vals


def _split(vals, n_p):
    inv_pi, hi, lo = vals[:3]
    p = vals[3:3 + n_p]
    q = vals[3 + n_p:-1]
    assert vals[-1] == 1.0
    return inv_pi, hi, lo, p, q


def _reduce_f32(x, inv_2pi, hi, lo, inv_2pi_t):
    """The float reduction, every operation rounded to float32 (the fused
    multiply-adds taken exactly in float64 and rounded once): t = r / 2 pi in
    revolutions with x = 2 pi k + r."""
    f32 = np.float32

    def fma(a, b, c):
        return (np.asarray(a, np.float64) * np.asarray(b, np.float64)
                + np.asarray(c, np.float64)).astype(f32)

    x = x.astype(f32)
    k = np.rint((x * f32(inv_2pi)).astype(f32))
    r = fma(-k, f32(hi), x)
    r = fma(-k, f32(lo), r)
    return k, (r * f32(inv_2pi_t)).astype(f32)


def test_float_reduction_constants_and_error():
    """The float sin/cos reduces by multiples of 2 pi (2 pi split into a float
    high part and the float nearest the rest) and passes revolutions to the
    hardware sine and cosine, whose own error is measured on the GPU
    (test_gpu_sincos).  Here: the constants, and the reduction's share of the
    error (2 pi t against x - 2 pi k in exact arithmetic) within the bound its
    roundings give, for angles far beyond those the links hold."""
    vals = _constants("float")
    assert len(vals) == 4
    inv_2pi, hi, lo, inv_2pi_t = vals
    two_pi = 2 * np.pi
    assert np.float32(inv_2pi) == np.float32(1 / two_pi) and inv_2pi_t == inv_2pi
    assert np.float32(hi) == np.float32(two_pi)
    assert np.float32(lo) == np.float32(two_pi - float(np.float32(two_pi)))
    rng = np.random.default_rng(5)
    for lim in (2.0, 40.0, 1e3, 1e4):
        x = rng.uniform(-lim, lim, 400_000).astype(np.float32)
        k, t = _reduce_f32(x, inv_2pi, hi, lo, inv_2pi_t)
        # k rounds the float x / (2 pi), off by a few ulps of it near half-integers
        assert np.abs(t).max() <= 0.5 + lim / (2 * np.pi) * 2.0 ** -22, lim
        # x - 2 pi k in (nearly) exact arithmetic: float64 with 2 pi to 2^-52
        exact = x.astype(np.float64) - k.astype(np.float64) * two_pi
        err = np.abs(two_pi * t.astype(np.float64) - exact).max()
        # two roundings of r (half an ulp of 4 each), the float 1/(2 pi) (relative
        # error 4.0e-8, times |r| <= pi) and the rounding of t (half an ulp of 1/2)
        assert err < 2 * 2.0 ** -22 + 4.04e-8 * np.pi + 2 * np.pi * 2.0 ** -26, (lim, err)
    z = np.array([0.0, -0.0], np.float32)
    assert np.all(_reduce_f32(z, inv_2pi, hi, lo, inv_2pi_t)[1] == 0)
    x = rng.uniform(-30, 30, 10_000).astype(np.float32)
    t1 = _reduce_f32(x, inv_2pi, hi, lo, inv_2pi_t)[1]
    t2 = _reduce_f32(-x, inv_2pi, hi, lo, inv_2pi_t)[1]
    assert np.array_equal(t1, -t2)


def test_double_sincos_within_stated_error():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 60
    vals = _constants("double")
    assert len(vals) == 3 + 8 + 8 + 1
    inv_pi, hi, lo, p, q = _split(vals, 8)
    M = mp.mpf

    def rnd(v):
        return float(v)   # nearest double

    def fma(a, b, c):
        return rnd(M(a) * M(b) + M(c))

    rng = np.random.default_rng(6)
    worst = 0.0
    for x in np.concatenate([rng.uniform(-2, 2, 600), rng.uniform(-300, 300, 600)]):
        x = float(x)
        k = float(np.rint(rnd(M(x) * M(inv_pi))))
        r = fma(-k, hi, x)
        r = fma(-k, lo, r)
        u = rnd(M(r) * M(r))
        ps = fma(u, p[0], p[1])
        for cf in p[2:]:
            ps = fma(u, ps, cf)
        s = fma(rnd(M(r) * M(u)), ps, r)
        qs = fma(u, q[0], q[1])
        for cf in q[2:]:
            qs = fma(u, qs, cf)
        co = fma(u, qs, 1.0)
        if int(k) & 1:
            s, co = -s, -co
        worst = max(worst, abs(M(s) - mp.sin(M(x))), abs(M(co) - mp.cos(M(x))))
    # a few units of 2^-53 on results of magnitude up to 1
    assert worst < 4 * 2.0 ** -53, float(worst)


def _phase_constants():
    src = open(HDR).read()
    start = src.index("float phase_f32(float y, float x")
    body = src[src.index("{", start):src.index("\n}\n", start)]
    # floating literals with a point or an exponent (the guards are 1e-30f, 3.0e38f)
    lit = re.compile(r"[-+]?\d+(?:\.\d*)?e[-+]?\d+f?|[-+]?\d+\.\d*f?")
    vals = [float(v.rstrip("f")) for v in lit.findall(body)]
    # T (highest power first, 7 terms), pi/2, pi, the 1e-30 and 3e38 guards
    return vals[:7], vals[7], vals[8], vals[9], vals[10]


def _phase_f32(y, x, consts, rcp_ulp=0):
    T, half_pi, pi, lo, hi = consts
    f32 = np.float32

    def fma(a, b, c):
        return (np.asarray(a, np.float64) * np.asarray(b, np.float64)
                + np.asarray(c, np.float64)).astype(f32)

    ax, ay = np.abs(x), np.abs(y)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    with np.errstate(divide="ignore", invalid="ignore"):
        rc = (1.0 / mx.astype(np.float64)).astype(f32)
    if rcp_ulp:
        rc = np.nextafter(rc, np.float32(np.inf) if rcp_ulp > 0 else np.float32(0))
    with np.errstate(invalid="ignore", over="ignore"):
        a = (mn * rc).astype(f32)
        u = (a * a).astype(f32)
        t = fma(u, T[0], T[1])
        for cf in T[2:]:
            t = fma(u, t, cf)
        r = fma((a * u).astype(f32), t, a)
    r = np.where(ay > ax, (f32(half_pi) - r).astype(f32), r)
    r = np.where(np.signbit(x), (f32(pi) - r).astype(f32), r)
    r = np.copysign(r, y)
    return np.where((mx >= f32(lo)) & (mx <= f32(hi)), r, np.float32(np.nan))


def test_phase_f32_within_stated_error_and_conventions():
    """The FP32 phase of the winding filter: below 5e-7 from atan2 for every octant
    over 40 decades of magnitude (with the hardware reciprocal one ulp either way),
    atan2's signed-zero conventions, and NaN below 1e-30 or beyond the float range
    (where the measuring kernels fall back to FP64 phases)."""
    consts = _phase_constants()
    assert len(consts[0]) == 7
    rng = np.random.default_rng(7)
    m = 10.0 ** rng.uniform(-20, 20, 600_000)
    ang = rng.uniform(-np.pi, np.pi, m.size)
    ang[:100_000] = np.round(ang[:100_000] / (np.pi / 4)) * (np.pi / 4)   # octant edges
    x = (m * np.cos(ang)).astype(np.float32)
    y = (m * np.sin(ang)).astype(np.float32)
    ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    for ulp in (-1, 0, 1):
        got = _phase_f32(y, x, consts, ulp)
        assert np.abs(got.astype(np.float64) - ref).max() < 5e-7, ulp
    z = np.float32(0.0)
    cases = [(z, np.float32(1.0), 0.0), (-z, np.float32(1.0), -0.0),
             (z, np.float32(-1.0), np.pi), (-z, np.float32(-1.0), -np.pi),
             (np.float32(1.0), -z, np.pi / 2), (np.float32(-2.0), z, -np.pi / 2)]
    for yy, xx, want in cases:
        got = float(_phase_f32(np.array([yy]), np.array([xx]), consts)[0])
        assert got == pytest.approx(want, abs=3e-7) and np.signbit(got) == np.signbit(want)
    tiny = _phase_f32(np.array([1e-31], np.float32), np.array([-1e-31], np.float32), consts)
    both0 = _phase_f32(np.array([0.0], np.float32), np.array([-0.0], np.float32), consts)
    huge = _phase_f32(np.array([np.inf], np.float32), np.array([1.0], np.float32), consts)
    assert np.isnan(tiny).all() and np.isnan(both0).all() and np.isnan(huge).all()
