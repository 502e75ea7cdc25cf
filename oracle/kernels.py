"""Parametrix and remainder kernels (oracle, FP64).

Section 4.1: the planar Green's function G(r; a, c) of (a Delta_2 + c) G = delta is
G = log(r) / (2 pi a) for c = 0; the parametrix is K(x, x') = G(|x - x'|; a(x'), c(x'))
with the coefficients taken at the source.  For c != 0 the paper prints
G = (i / 4a) H0(sqrt(c/a) r), whose log part, -log(r) / (2 pi a), has the opposite sign of
the c = 0 function: it solves (a Delta_2 + c) G = -delta.  We read G = -(i / 4a) H0(sqrt(c/a) r),
which for c < 0 (modified Helmholtz type) is the real function
    G = -K0(kappa r) / (2 pi a),   kappa = sqrt(-c / a)
(H0(i z) = (2 / (i pi)) K0(z)), and tends to log(r) / (2 pi a) + const as c -> 0.  For c > 0
(the Helmholtz type of Section 7.3) the same reading gives the complex function
    G = -(i / 4a) H0(k r),   k = sqrt(c / a)   (H0 = H0^(1), the Hankel function of the first kind),
whose real part Y0(k r) / (4a) carries the log singularity and whose imaginary part
-J0(k r) / (4a) is smooth; R, the blocks, the system and u = K[sigma] are then complex.
eq:explicit_remainder gives the remainder for x != x':

  R = grad_G a(x) . r_hat G'  -  a(x) G'' (n.r)^2 / r^2  +  a(x) G' (n.r)^2 / r^3
      - 2 a(x) H(x) (n . r_hat) G'  +  (c(x) - a(x) c(x') / a(x')) G

with r = x - x', G' = dG/dr and G'' = d^2G/dr^2 (the definition line prints
G'' = d^2/dr^2 G', which we read as the second derivative of G).  Target
quantities n, H, a, c, grad_G a are at x.  The modified Bessel functions K0, K1 and the Hankel
functions H0, H1 come from the library (scipy.special).

Advection (eq:adv_remainder): with a first-order term b . grad_G u in the equation the same
parametrix serves and the remainder gains b(x) . grad_G K(x, x').  K depends on x through
r = |x - x'| only, so grad K = G' r_hat, and for a field b tangent at x the surface gradient's
projection drops: the added term is G' (b . r_hat).
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

INV_2PI = 1.0 / (2.0 * np.pi)


def green_c0(r, a):
    """G(r; a) = log(r) / (2 pi a) and its first two r-derivatives."""
    G = np.log(r) / (2 * np.pi * a)
    G1 = 1.0 / (2 * np.pi * a * r)
    G2 = -1.0 / (2 * np.pi * a * r * r)
    return G, G1, G2


def green_neg_c(r, a, c):
    """G(r; a, c) = -K0(kappa r) / (2 pi a), kappa = sqrt(-c/a), c < 0, and its first two
    r-derivatives: G' = kappa K1(kappa r) / (2 pi a) (K0' = -K1) and
    G'' = -kappa^2 (K0(kappa r) + K1(kappa r) / (kappa r)) / (2 pi a) (K1'(z) = -K0(z) - K1(z)/z)."""
    kappa = np.sqrt(-c / a)
    z = kappa * r
    k0, k1 = sp.k0(z), sp.k1(z)
    G = -k0 / (2 * np.pi * a)
    G1 = kappa * k1 / (2 * np.pi * a)
    G2 = -kappa ** 2 * (k0 + k1 / z) / (2 * np.pi * a)
    return G, G1, G2


def green_pos_c(r, a, c):
    """G(r; a, c) = -(i / 4a) H0(k r), k = sqrt(c/a), c > 0, and its first two r-derivatives:
    G' = (i k / 4a) H1(k r) (H0' = -H1) and G'' = (i k^2 / 4a) (H0(k r) - H1(k r) / (k r))
    (H1'(z) = H0(z) - H1(z) / z)."""
    k = np.sqrt(c / a)
    z = k * r
    h0, h1 = sp.hankel1(0, z), sp.hankel1(1, z)
    G = -1j * h0 / (4 * a)
    G1 = 1j * k * h1 / (4 * a)
    G2 = 1j * k ** 2 * (h0 - h1 / z) / (4 * a)
    return G, G1, G2


def green(r, a, c=None):
    """G, G', G'' of the planar Green's function: c = None (c = 0), c < 0 at every entry (real) or
    c > 0 at every entry (complex)."""
    if c is None:
        return green_c0(r, a)
    c = np.asarray(c)
    if np.all(c < 0):
        return green_neg_c(r, a, c)
    if np.all(c > 0):
        return green_pos_c(r, a, c)
    raise ValueError("the oracle's c != 0 kernels need c < 0 everywhere or c > 0 everywhere")


def remainder(x, n, H, a_t, gs_t, y, a_s, c_t=None, c_s=None, b_t=None):
    """R(x, y) of eq:explicit_remainder (R_b of eq:adv_remainder when b_t is given);
    broadcasts over leading axes.

    x, n, gs_t: (..., 3) target position, unit normal, surface gradient of a;
    H, a_t: (...) target mean curvature and coefficient; y: (..., 3) source
    position; a_s: (...) coefficient at the source; c_t, c_s: c at the target and the
    source (None: c = 0, the Laplace-Beltrami type); b_t: (..., 3) advection field at the
    target, tangent there (None: no first-order term).
    """
    r = x - y
    rn = np.linalg.norm(r, axis=-1)
    rhat = r / rn[..., None]
    G, G1, G2 = green(rn, a_s, c_s)
    nr = np.sum(n * r, axis=-1)
    R = (np.sum(gs_t * rhat, axis=-1) * G1
         - a_t * G2 * nr ** 2 / rn ** 2
         + a_t * G1 * nr ** 2 / rn ** 3
         - 2 * a_t * H * (nr / rn) * G1)
    if c_s is not None:
        R = R + (c_t - a_t * c_s / a_s) * G
    if b_t is not None:
        R = R + np.sum(b_t * rhat, axis=-1) * G1
    return R


def remainder_lb(x, n, H, y):
    """R_LB of eq:explicit_remainderLB: (1/pi)(n.r/r^2)^2 - (H/pi)(n.r/r^2)."""
    r = x - y
    r2 = np.sum(r * r, axis=-1)
    t = np.sum(n * r, axis=-1) / r2
    return t * t / np.pi - H * t / np.pi


def parametrix(x, y, a_s, c_s=None):
    """K(x, y) = G(|x - y|; a(y), c(y)): log|x - y| / (2 pi a(y)) for c = 0."""
    if c_s is None:
        return np.log(np.linalg.norm(x - y, axis=-1)) / (2 * np.pi * a_s)
    return green(np.linalg.norm(x - y, axis=-1), a_s, c_s)[0]
