"""Chebyshev coefficients of g_nu(z) = sqrt(z) e^z K_nu(z), nu = 0, 1, on z >= 2, for the device
routine bessel_k01 (pmx_internal.hpp).

g_nu is smooth in s = 2 / z on (0, 1] (it tends to sqrt(pi / 2) as z -> infinity), so it is
interpolated at the n + 1 Chebyshev points of the first kind in x = 2 s - 1 = 4 / z - 1 at 40
significant digits (mpmath), and the coefficients of the interpolant in the Chebyshev basis are
printed as C++ initialisers.  Degree 22 reaches 2e-16 relative error on [2, infinity), which the
script checks on 2,001 points before printing.

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


def clenshaw(c, x: float) -> float:
    b1 = b2 = 0.0
    for cj in reversed(c[1:]):
        b1, b2 = 2.0 * x * b1 - b2 + cj, b1
    return x * b1 - b2 + c[0]


def main():
    mp.mp.dps = 40
    for nu in (0, 1):
        c = [float(v) for v in chebyshev_coefficients(lambda s: g(nu, s), DEGREE)]
        worst = 0.0
        for k in range(2001):
            s = mp.mpf(k + 1) / 2001
            ref = g(nu, s)
            worst = max(worst, float(abs(clenshaw(c, float(2 * s - 1)) - ref) / ref))
        assert worst < 4e-16, (nu, worst)
        body = ",\n    ".join(", ".join(f"{v:.17e}" for v in c[i:i + 3]) for i in range(0, len(c), 3))
        print(f"// nu = {nu}: max relative error {worst:.1e} on [2, infinity)")
        print(f"constexpr double kChebK{nu}[{DEGREE + 1}] = {{\n    {body}}};")


if __name__ == "__main__":
    main()
