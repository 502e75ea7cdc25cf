"""Quadrature rules in the parameter square [-1, 1]^2 (oracle, FP64).

Self rule (Section 6.1.1, eq:radial_int): polar coordinates about the target
pre-image t0, Gauss-Legendre in both the angle and the radius.  The square is
split into four triangles (t0, c_k, c_k+1), one per edge.  On the triangle of
edge k the ray at angle theta leaves the square at L(theta) = d_k / cos(theta -
theta_k), where d_k is the distance from t0 to the edge and theta_k its
outward normal angle.  Because L is only piecewise smooth and nearly singular
when t0 is close to an edge, the angular panels are split at theta_k and
wherever L doubles (cos(theta - theta_k) = 2^-m, m = 1, 2, ...): a fixed,
tolerance-free stand-in for the paper's choice of panels that integrate
L^2(theta) to tolerance.  Each panel carries n_gl points in angle.  In the radius,
the remainder R (bounded, or O(1/r) for variable a, so that R rho is analytic
along each ray) uses one n_gl-point Gauss-Legendre panel on [0, L]; the
parametrix K (log singular) uses dyadically graded panels whose innermost one
is mapped by rho = t^3 so that rho log rho is smooth in t.

Near rule (Section 6.1.2): the paper subdivides the element adaptively.  Here
a sub-square S is split into four while the target lies within eta = 1.5
radii of S's centroid (the same centroid / radius definition as for whole
patches, from the images of S's corners), up to depth 20; every leaf gets an
n_gl x n_gl tensor Gauss-Legendre rule.

Both functions return points (u, v) and weights such that
sum_k w_k F(u_k, v_k) ~ int_[-1,1]^2 F du dv.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import gauss_legendre, interpolate_patch, centroid_radius


def _angle_breaks(phi_end: float, split: float):
    """Panel edges on [0, phi_end] (phi_end > 0): 0, arccos(split^-m) inside, phi_end."""
    br = [0.0]
    m = 1
    while True:
        b = math.acos(split ** (-m))
        if b >= phi_end:
            break
        br.append(b)
        m += 1
    br.append(phi_end)
    return br


def _radial_rule(n_gl: int, radial: str):
    """Nodes s in (0, 1] and weights for int_0^L F(rho) rho drho = L^2 sum w_k F(L s_k).

    "plain": one Gauss-Legendre panel in rho (F rho analytic along the ray: the
    remainder R, bounded or O(1/r), times the polar Jacobian).
    "log": F has a log(rho) singularity (the parametrix K): dyadic panels
    [1/2, 1], [1/4, 1/2], [1/8, 1/4] and an innermost [0, 1/8] panel in the
    variable t with rho = t^3 / 8, which makes rho log(rho) drho smooth in t.
    "dyadic": the same four dyadic panels, each a plain Gauss-Legendre panel in rho
    (the remainder R with c != 0, whose rho^m log(rho) parts, m >= 2 with the
    Jacobian, need the grading but not the t^3 map: that map puts points within
    1e-10 of the target, where r = x - y keeps too few digits of its normal component
    for R's (n.r)^2 / r^4 terms).
    """
    tg, wg = gauss_legendre(n_gl)
    t = 0.5 * (tg + 1.0)
    wt = 0.5 * wg
    if radial == "plain":
        return t, wt * t
    if radial not in ("log", "dyadic"):
        raise ValueError(radial)
    s_parts, w_parts = [], []
    for a, b in ((0.5, 1.0), (0.25, 0.5), (0.125, 0.25)) + (((0.0, 0.125),) if radial == "dyadic" else ()):
        s = a + (b - a) * t
        s_parts.append(s)
        w_parts.append((b - a) * wt * s)
    if radial == "dyadic":
        return np.concatenate(s_parts), np.concatenate(w_parts)
    # rho = t^3 / 8: rho drho = (t^3 / 8) (3 t^2 / 8) dt
    s_parts.append(t ** 3 / 8.0)
    w_parts.append(wt * 3.0 * t ** 5 / 64.0)
    return np.concatenate(s_parts), np.concatenate(w_parts)


def self_rule(u0: float, v0: float, n_gl: int = 16, split: float = 2.0, radial: str = "plain"):
    """Polar rule about (u0, v0) in (-1, 1)^2.  Returns (u, v, w)."""
    tg, wg = gauss_legendre(n_gl)
    s_rad, w_rad = _radial_rule(n_gl, radial)
    # edge k: (outward normal angle, distance from t0), corners c_k -> c_k+1 counter-clockwise
    edges = [(-math.pi / 2, v0 + 1.0), (0.0, 1.0 - u0), (math.pi / 2, 1.0 - v0), (math.pi, u0 + 1.0)]
    corners = [(-1.0, -1.0), (1.0, -1.0), (1.0, 1.0), (-1.0, 1.0)]
    us, vs, ws = [], [], []
    for k in range(4):
        th_n, d = edges[k]
        tan_dir = (-math.sin(th_n), math.cos(th_n))
        ca, cb = corners[k], corners[(k + 1) % 4]
        s_a = (ca[0] - u0) * tan_dir[0] + (ca[1] - v0) * tan_dir[1]
        s_b = (cb[0] - u0) * tan_dir[0] + (cb[1] - v0) * tan_dir[1]
        phi_a = math.atan2(s_a, d)          # < 0
        phi_b = math.atan2(s_b, d)          # > 0
        panels = []
        pos = _angle_breaks(phi_b, split)
        panels += list(zip(pos[:-1], pos[1:]))
        neg = _angle_breaks(-phi_a, split)
        panels += [(-b1, -b0) for b0, b1 in zip(neg[:-1], neg[1:])]
        for p0, p1 in panels:
            mid, half = 0.5 * (p0 + p1), 0.5 * (p1 - p0)
            phi = mid + half * tg
            wphi = half * wg
            L = d / np.cos(phi)                                   # (n_angle,)
            rho = L[:, None] * s_rad[None, :]                      # (angle, radius)
            w = wphi[:, None] * L[:, None] ** 2 * w_rad[None, :]
            ang = th_n + phi
            us.append((u0 + rho * np.cos(ang)[:, None]).ravel())
            vs.append((v0 + rho * np.sin(ang)[:, None]).ravel())
            ws.append(w.ravel())
    return np.concatenate(us), np.concatenate(vs), np.concatenate(ws)


def near_leaves(x_target: np.ndarray, Xp: np.ndarray, tnodes: np.ndarray, eta: float = 1.5,
                max_depth: int = 20):
    """Leaves [ua, ub, va, vb] of the subdivision of [-1,1]^2 for a target off the patch."""
    leaves = []

    def visit(ua, ub, va, vb, depth):
        cu = np.array([ua, ub, ub, ua])
        cv = np.array([va, va, vb, vb])
        corners = interpolate_patch(Xp, tnodes, cu, cv)
        c, rad = centroid_radius(corners)
        if np.linalg.norm(x_target - c) < eta * rad and depth < max_depth:
            um, vm = 0.5 * (ua + ub), 0.5 * (va + vb)
            visit(ua, um, va, vm, depth + 1)
            visit(um, ub, va, vm, depth + 1)
            visit(ua, um, vm, vb, depth + 1)
            visit(um, ub, vm, vb, depth + 1)
        else:
            leaves.append((ua, ub, va, vb))

    visit(-1.0, 1.0, -1.0, 1.0, 0)
    return leaves


def near_rule(x_target: np.ndarray, Xp: np.ndarray, tnodes: np.ndarray, n_gl: int = 16,
              eta: float = 1.5, max_depth: int = 20):
    """Tensor Gauss-Legendre rule on every leaf of the subdivision.  Returns (u, v, w)."""
    tg, wg = gauss_legendre(n_gl)
    us, vs, ws = [], [], []
    for ua, ub, va, vb in near_leaves(x_target, Xp, tnodes, eta, max_depth):
        hu, hv = 0.5 * (ub - ua), 0.5 * (vb - va)
        uu = 0.5 * (ua + ub) + hu * tg
        vv = 0.5 * (va + vb) + hv * tg
        us.append(np.repeat(uu, n_gl))
        vs.append(np.tile(vv, n_gl))
        ws.append(np.outer(wg * hu, wg * hv).ravel())
    return np.concatenate(us), np.concatenate(vs), np.concatenate(ws)
