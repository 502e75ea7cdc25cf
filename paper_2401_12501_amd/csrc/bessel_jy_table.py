"""Chebyshev coefficients for the device routine bessel_jy01 (pmx_internal.hpp): J0, J1, Y0, Y1 of
a real argument z > 0, the Bessel functions of the Helmholtz-type kernel G = -(i / 4a) H0(k r).

Two ranges, each interpolated at the n + 1 Chebyshev points of the first kind (mpmath, 40 digits),
with the coefficients of the interpolant in the Chebyshev basis printed as C++ initialisers.

z <= 8, in x = z^2 / 32 - 1 (w = z^2 in [0, 64]), four entire functions of w:
    J0(z),   J1(z) / z,
    S0 = Y0(z) - (2/pi) log(z/2) J0(z),
    S1 = (Y1(z) - (2/pi) log(z/2) J1(z) + 2 / (pi z)) / z
(the power series of Y0 and Y1 split into these log and entire parts, so the device adds the
logarithm back: Y0 = (2/pi) log(z/2) J0 + S0, Y1 = (2/pi) log(z/2) J1 - 2/(pi z) + z S1).

z > 8, in x = 2 s - 1 with s = 8 / z in (0, 1), Hankel's form
    H_nu(z) = sqrt(2 / (pi z)) (P_nu(z) + i Q_nu(z)) exp(i chi),  chi = z - nu pi / 2 - pi / 4,
so J_nu = sqrt(2/(pi z)) (P cos chi - Q sin chi) and Y_nu = sqrt(2/(pi z)) (P sin chi + Q cos chi);
P_nu and Q_nu are smooth in s and tend to 1 and 0 as z -> infinity.

The script checks each fit on 4,001 points of its range before printing: the absolute error of the
fitted function evaluated in double precision by Clenshaw's recurrence stays below 1e-15 on the
small range (degree 16; the J0 fit's 9.8e-16 is rounding in the recurrence, not truncation) and
below 4e-16 on the large range (degree 14), where it is relative to the envelope sqrt(2 / (pi z)).

Run: python paper_2401_12501_amd/csrc/bessel_jy_table.py
"""
import mpmath as mp

Z0 = 8
DEG_SMALL = 16
DEG_LARGE = 14


def small(name: str, w):
    z = mp.sqrt(w) if w > 0 else mp.mpf(0)
    if name == "J0":
        return mp.besselj(0, z)
    if name == "J1z":
        return mp.mpf(1) / 2 if z == 0 else mp.besselj(1, z) / z
    if z == 0:   # limits of the entire parts at w = 0
        return (2 / mp.pi) * mp.euler if name == "S0" else (2 * mp.euler - 1) / (2 * mp.pi)
    L = (2 / mp.pi) * mp.log(z / 2)
    if name == "S0":
        return mp.bessely(0, z) - L * mp.besselj(0, z)
    return (mp.bessely(1, z) - L * mp.besselj(1, z) + 2 / (mp.pi * z)) / z


def large(name: str, s):
    z = mp.mpf(Z0) / s
    nu = 0 if name[1] == "0" else 1
    chi = z - nu * mp.pi / 2 - mp.pi / 4
    h = mp.hankel1(nu, z) * mp.sqrt(mp.pi * z / 2) * mp.exp(-1j * chi)
    return h.real if name[0] == "P" else h.imag


def chebyshev_coefficients(f, n: int):
    """Coefficients of the degree-n interpolant of f on [-1, 1] at the Chebyshev points."""
    nodes = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (n + 1)) for k in range(n + 1)]
    values = [f(x) for x in nodes]
    c = [2 * mp.fsum(values[k] * mp.cos(mp.pi * j * (k + mp.mpf(1) / 2) / (n + 1)) for k in range(n + 1)) / (n + 1)
         for j in range(n + 1)]
    c[0] /= 2
    return c


def clenshaw(c, x: float) -> float:
    b1 = b2 = 0.0
    for cj in reversed(c[1:]):
        b1, b2 = 2.0 * x * b1 - b2 + cj, b1
    return x * b1 - b2 + c[0]


def fits():
    """(name, coefficients, max abs error) for the eight fits, checked at 4,001 points."""
    mp.mp.dps = 40
    out = []
    for name in ("J0", "J1z", "S0", "S1"):
        f = lambda x, name=name: small(name, (x + 1) * 32)
        c = [float(v) for v in chebyshev_coefficients(f, DEG_SMALL)]
        err = max(abs(clenshaw(c, float(x)) - f(x)) for x in (mp.mpf(2 * k) / 4000 - 1 for k in range(4001)))
        out.append((name, c, float(err)))
    for name in ("P0", "Q0", "P1", "Q1"):
        f = lambda x, name=name: large(name, (x + 1) / 2)
        c = [float(v) for v in chebyshev_coefficients(f, DEG_LARGE)]
        # s = 0 (z = infinity) is a limit: sample s in [1e-4, 1]
        err = max(abs(clenshaw(c, float(x)) - f(x))
                  for x in (2 * (mp.mpf(1) / 10000 + (1 - mp.mpf(1) / 10000) * mp.mpf(k) / 4000) - 1
                            for k in range(4001)))
        out.append((name, c, float(err)))
    return out


def main():
    for name, c, err in fits():
        assert err < (1e-15 if name in ("J0", "J1z", "S0", "S1") else 4e-16), (name, err)
        body = ",\n    ".join(", ".join(f"{v:.17e}" for v in c[i:i + 3]) for i in range(0, len(c), 3))
        print(f"// {name}: max abs error {err:.1e}")
        print(f"constexpr double kCheb{name}[{len(c)}] = {{\n    {body}}};")


if __name__ == "__main__":
    main()
