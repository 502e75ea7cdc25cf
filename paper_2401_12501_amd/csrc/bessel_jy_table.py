"""Chebyshev coefficients for the device routine bessel_jy01 (pmx_internal.hpp): J0, J1, Y0, Y1 of
a real argument z > 0, the Bessel functions of the Helmholtz-type kernel G = -(i / 4a) H0(k r).

Two ranges, each interpolated at the n + 1 Chebyshev points of the first kind (mpmath, 40 digits).
The interpolant's coefficients in the Chebyshev basis are converted, still at 40 digits, to its
power form in x (T_0 = 1, T_1 = x, T_{k+1} = 2 x T_k - T_{k-1}), which the device evaluates by
Horner's rule: one fused multiply-add per degree instead of the two operations of each step of
Clenshaw's recurrence, with no loss of accuracy on these ranges (the power coefficients stay small:
their absolute sum is at most 4.2).  The coefficients are printed as C++ initialisers.

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
power form evaluated in double precision by Horner's rule stays below 1e-15 on the small range
(degree 16; J0's 7e-16 is rounding, not truncation) and below 4e-16 on the large range (degree
14), where it is relative to the envelope sqrt(2 / (pi z)).

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


def power_form(c):
    """Coefficients a_j of sum_k c_k T_k(x) = sum_j a_j x^j (at the working precision)."""
    n = len(c)
    T = [[mp.mpf(1)] + [mp.mpf(0)] * (n - 1), [mp.mpf(0), mp.mpf(1)] + [mp.mpf(0)] * (n - 2)]
    for _ in range(2, n):
        t = [mp.mpf(0)] + [2 * v for v in T[-1][:-1]]
        T.append([t[j] - T[-2][j] for j in range(n)])
    return [mp.fsum(c[k] * T[k][j] for k in range(n)) for j in range(n)]


def horner(a, x: float) -> float:
    p = a[-1]
    for v in reversed(a[:-1]):
        p = p * x + v
    return p


def fits():
    """(name, power-form coefficients, max abs error) for the eight fits, checked at 4,001 points."""
    mp.mp.dps = 40
    out = []
    for name in ("J0", "J1z", "S0", "S1"):
        f = lambda x, name=name: small(name, (x + 1) * 32)
        a = [float(v) for v in power_form(chebyshev_coefficients(f, DEG_SMALL))]
        err = max(abs(horner(a, float(x)) - f(x)) for x in (mp.mpf(2 * k) / 4000 - 1 for k in range(4001)))
        out.append((name, a, float(err)))
    for name in ("P0", "Q0", "P1", "Q1"):
        f = lambda x, name=name: large(name, (x + 1) / 2)
        a = [float(v) for v in power_form(chebyshev_coefficients(f, DEG_LARGE))]
        # s = 0 (z = infinity) is a limit: sample s in [1e-4, 1]
        err = max(abs(horner(a, float(x)) - f(x))
                  for x in (2 * (mp.mpf(1) / 10000 + (1 - mp.mpf(1) / 10000) * mp.mpf(k) / 4000) - 1
                            for k in range(4001)))
        out.append((name, a, float(err)))
    return out


def main():
    for name, c, err in fits():
        assert err < (1e-15 if name in ("J0", "J1z", "S0", "S1") else 4e-16), (name, err)
        body = ",\n    ".join(", ".join(f"{v:.17e}" for v in c[i:i + 3]) for i in range(0, len(c), 3))
        print(f"// {name}: max abs error {err:.1e}")
        print(f"constexpr double kPoly{name}[{len(c)}] = {{\n    {body}}};")


if __name__ == "__main__":
    main()
