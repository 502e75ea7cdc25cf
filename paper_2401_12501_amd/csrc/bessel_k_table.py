"""Interpolants of g_nu(z) = sqrt(z) e^z K_nu(z), nu = 0, 1, on z >= 2, for the device
routine bessel_k01 (pmx_internal.hpp).

g_nu is smooth in s = 2 / z on (0, 1] (it tends to sqrt(pi / 2) as z -> infinity), so it is
interpolated at the n + 1 Chebyshev points of the first kind in x = 2 s - 1 = 4 / z - 1 at 40
significant digits (mpmath).  The interpolant's coefficients in the Chebyshev basis are converted,
still at 40 digits, to its power form in x (T_0 = 1, T_1 = x, T_{k+1} = 2 x T_k - T_{k-1}), which
the device evaluates by Horner's rule, one fused multiply-add per degree; the power coefficients stay
small (their absolute sums are 1.25 and 1.47), so nothing is lost.  Degree 22 reaches 2e-16 relative
error on [2, infinity) in double precision, which the script checks on 2,001 points before printing
the coefficients as C++ initialisers.

Run: python paper_2401_12501_amd/csrc/bessel_k_table.py
"""
import mpmath as mp

DEGREE = 22


def g(nu: int, s):
    z = mp.mpf(2) / s
    return mp.sqrt(z) * mp.exp(z) * mp.besselk(nu, z)


def chebyshev_coefficients(f, n: int):
    nodes = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (n + 1)) for k in range(n + 1)]
    values = [f((x + 1) / 2) for x in nodes]
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


def main():
    mp.mp.dps = 40
    for nu in (0, 1):
        c = [float(v) for v in power_form(chebyshev_coefficients(lambda s: g(nu, s), DEGREE))]
        worst = 0.0
        for k in range(2001):
            s = mp.mpf(k + 1) / 2001
            ref = g(nu, s)
            worst = max(worst, float(abs(horner(c, float(2 * s - 1)) - ref) / ref))
        assert worst < 4e-16, (nu, worst)
        body = ",\n    ".join(", ".join(f"{v:.17e}" for v in c[i:i + 3]) for i in range(0, len(c), 3))
        print(f"// nu = {nu}: max relative error {worst:.1e} on [2, infinity)")
        print(f"constexpr double kPolyK{nu}[{DEGREE + 1}] = {{\n    {body}}};")


if __name__ == "__main__":
    main()
