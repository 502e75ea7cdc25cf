"""Parametrix and remainder kernels (oracle, FP64).

Section 4.1: for c = 0 the planar Green's function is G(r; a) = log(r) / (2 pi a)
and the parametrix is K(x, x') = G(|x - x'|; a(x')) with the coefficient taken at
the source.  eq:explicit_remainder gives the remainder for x != x':

  R = grad_G a(x) . r_hat G'  -  a(x) G'' (n.r)^2 / r^2  +  a(x) G' (n.r)^2 / r^3
      - 2 a(x) H(x) (n . r_hat) G'                       (c = 0 term dropped)

with r = x - x', G' = dG/dr and G'' = d^2G/dr^2 (the definition line prints
G'' = d^2/dr^2 G', which we read as the second derivative of G).  Target
quantities n, H, a, grad_G a are at x.
"""
from __future__ import annotations

import numpy as np

INV_2PI = 1.0 / (2.0 * np.pi)


def green_c0(r, a):
    """G(r; a) = log(r) / (2 pi a) and its first two r-derivatives."""
    G = np.log(r) / (2 * np.pi * a)
    G1 = 1.0 / (2 * np.pi * a * r)
    G2 = -1.0 / (2 * np.pi * a * r * r)
    return G, G1, G2


def remainder(x, n, H, a_t, gs_t, y, a_s):
    """R(x, y) of eq:explicit_remainder with c = 0; broadcasts over leading axes.

    x, n, gs_t: (..., 3) target position, unit normal, surface gradient of a;
    H, a_t: (...) target mean curvature and coefficient; y: (..., 3) source
    position; a_s: (...) coefficient at the source.
    """
    r = x - y
    rn = np.linalg.norm(r, axis=-1)
    rhat = r / rn[..., None]
    _, G1, G2 = green_c0(rn, a_s)
    nr = np.sum(n * r, axis=-1)
    return (np.sum(gs_t * rhat, axis=-1) * G1
            - a_t * G2 * nr ** 2 / rn ** 2
            + a_t * G1 * nr ** 2 / rn ** 3
            - 2 * a_t * H * (nr / rn) * G1)


def remainder_lb(x, n, H, y):
    """R_LB of eq:explicit_remainderLB: (1/pi)(n.r/r^2)^2 - (H/pi)(n.r/r^2)."""
    r = x - y
    r2 = np.sum(r * r, axis=-1)
    t = np.sum(n * r, axis=-1) / r2
    return t * t / np.pi - H * t / np.pi


def parametrix(x, y, a_s):
    """K(x, y) = log|x - y| / (2 pi a(y))."""
    return np.log(np.linalg.norm(x - y, axis=-1)) / (2 * np.pi * a_s)
