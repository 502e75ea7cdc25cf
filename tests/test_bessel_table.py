"""The device routines for K0 and K1 (bessel_k01) and for J0, J1, Y0, Y1 (bessel_jy01) in
pmx_internal.hpp, replayed on the host.

The interpolants' power-form tables are read from the header and the series coefficients are built
the way make_kseries builds them; the evaluation follows the routine step by step (Horner's rule in
t = z^2/4 for z <= 2, and in x = 4/z - 1 times exp(-z)/sqrt(z) above).  Against mpmath at 30
digits the relative error stays below 5e-15 from z = 1e-12 to 60, and the tables are those
bessel_k_table.py prints (degree 22, checked by the script itself).
"""
import math
import os
import re

import mpmath as mp
import numpy as np

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2401_12501_amd", "csrc",
                   "pmx_internal.hpp")
GAMMA = 0.57721566490153286061


def table(name):
    src = open(HDR).read()
    m = re.search(r"constexpr double " + name + r"\[(\d+)\] = \{(.*?)\};", src, re.S)
    vals = [float(v) for v in m.group(2).replace("\n", " ").split(",")]
    assert len(vals) == int(m.group(1))
    return vals


def series():
    i0, s0, i1, s1 = [], [], [], []
    f, g, h = 1.0, 1.0, 0.0
    for k in range(13):
        hn = h + 1.0 / (k + 1)
        i0.append(f)
        s0.append(h * f)
        i1.append(g)
        s1.append((h + hn) * g)
        f /= float(k + 1) * (k + 1)
        g /= float(k + 1) * (k + 2)
        h = hn
    return i0, s0, i1, s1


def horner(c, t):
    p = c[-1]
    for v in reversed(c[:-1]):
        p = math.fma(p, t, v) if hasattr(math, "fma") else p * t + v
    return p


def k01(z, S, C0, C1):
    if z <= 2.0:
        t = 0.25 * z * z
        L = 0.5 * math.log(t) + GAMMA
        i0, s0, i1, s1 = S
        return -L * horner(i0, t) + horner(s0, t), 1.0 / z + L * (0.5 * z * horner(i1, t)) - 0.25 * z * horner(s1, t)
    x = 4.0 / z - 1.0
    e = math.exp(-z) / math.sqrt(z)
    return horner(C0, x) * e, horner(C1, x) * e


def test_device_k01_against_mpmath():
    mp.mp.dps = 30
    S, C0, C1 = series(), table("kPolyK0"), table("kPolyK1")
    worst = [0.0, 0.0]
    zs = np.concatenate([np.logspace(-12, math.log10(2.0), 500), np.linspace(1.95, 2.05, 101),
                         np.geomspace(2.0, 60.0, 500)])
    for z in zs:
        got = k01(float(z), S, C0, C1)
        for nu in (0, 1):
            ref = mp.besselk(nu, z)
            worst[nu] = max(worst[nu], float(abs((got[nu] - ref) / ref)))
    assert worst[0] < 5e-15 and worst[1] < 5e-15, worst


def test_tables_match_the_generator():
    """The header's tables are the generator's output (degree 22: 23 power-form coefficients each;
    g_nu tends to sqrt(pi/2) = 1.2533 as z -> infinity, x -> -1)."""
    for name in ("kPolyK0", "kPolyK1"):
        c = table(name)
        assert len(c) == 23
        val_at_infinity = sum(cj * (-1) ** j for j, cj in enumerate(c))   # x = -1
        assert abs(val_at_infinity - math.sqrt(math.pi / 2)) < 1e-15


def jy01(z, T):
    """The device routine bessel_jy01 step by step (natural log in place of the device's log)."""
    cheb = horner
    k2pi = 2.0 / math.pi
    if z <= 8.0:
        w = z * z
        x = w / 32.0 - 1.0
        a0, a1, s0, s1 = (cheb(T[n], x) for n in ("kPolyJ0", "kPolyJ1z", "kPolyS0", "kPolyS1"))
        L = 0.5 * k2pi * math.log(0.25 * w)
        j1 = z * a1
        return a0, j1, L * a0 + s0, L * j1 + z * s1 - k2pi / z
    x = 16.0 / z - 1.0
    p0, q0, p1, q1 = (cheb(T[n], x) for n in ("kPolyP0", "kPolyQ0", "kPolyP1", "kPolyQ1"))
    sn, cs = math.sin(z), math.cos(z)
    env = math.sqrt(k2pi / z)
    c0, s0 = (cs + sn) * math.sqrt(0.5), (sn - cs) * math.sqrt(0.5)
    return env * (p0 * c0 - q0 * s0), env * (p1 * s0 + q1 * c0), env * (p0 * s0 + q0 * c0), env * (q1 * s0 - p1 * c0)


def test_device_jy01_against_mpmath():
    """J0, J1, Y0, Y1 of the device routine against mpmath at 30 digits from z = 1e-10 to 80: absolute
    error below 3e-15 for z <= 8 (Y0, Y1 relative near z = 0, where they diverge), and below
    3e-15 times the envelope sqrt(2 / (pi z)) beyond."""
    mp.mp.dps = 30
    T = {n: table(n) for n in ("kPolyJ0", "kPolyJ1z", "kPolyS0", "kPolyS1", "kPolyP0", "kPolyQ0", "kPolyP1",
                                "kPolyQ1")}
    zs = np.concatenate([np.logspace(-10, 0, 200), np.linspace(1.0, 8.0, 700), np.linspace(7.99, 8.01, 41),
                         np.linspace(8.0, 80.0, 1500)])
    worst = 0.0
    for z in zs:
        z = float(z)
        got = jy01(z, T)
        refs = (mp.besselj(0, z), mp.besselj(1, z), mp.bessely(0, z), mp.bessely(1, z))
        scale = 1.0 if z <= 8.0 else math.sqrt(2.0 / (math.pi * z))
        for g, ref in zip(got, refs):
            err = float(abs(g - ref)) / max(scale, float(abs(ref)) if z < 1.0 else scale)
            worst = max(worst, err)
    assert worst < 3e-15, worst


def test_jy_tables_limits():
    """Power forms in x: P_nu -> 1 and Q_nu -> 0 as z -> infinity (x = -1), and the small-range fits
    equal their values at z = 0 (x = -1): J0(0) = 1, J1(z)/z -> 1/2; and at z = 8 (x = 1) the
    small-range J0 meets the large-range Hankel form."""
    at = lambda c, x: sum(cj * x ** j for j, cj in enumerate(c))
    assert abs(at(table("kPolyP0"), -1.0) - 1.0) < 1e-15
    assert abs(at(table("kPolyP1"), -1.0) - 1.0) < 1e-15
    assert abs(at(table("kPolyQ0"), -1.0)) < 1e-15
    assert abs(at(table("kPolyQ1"), -1.0)) < 1e-15
    assert abs(at(table("kPolyJ0"), -1.0) - 1.0) < 1e-15
    assert abs(at(table("kPolyJ1z"), -1.0) - 0.5) < 1e-15
    z = 8.0
    env = math.sqrt(2.0 / (math.pi * z))
    chi = z - math.pi / 4
    j0_large = env * (at(table("kPolyP0"), 1.0) * math.cos(chi) - at(table("kPolyQ0"), 1.0) * math.sin(chi))
    assert abs(at(table("kPolyJ0"), 1.0) - j0_large) < 2e-15
