"""Seeded synthetic surfaces as quad patches with tensor Gauss-Legendre nodes.

Every surface is a union of patches, each the image of the reference square
[-1,1]^2 under a smooth map y_P(u, v).  Node ``i = P*q*q + iu*q + iv`` sits at the
image of the Gauss-Legendre pair (t_iu, t_iv).  For each node the generator
returns the position and its first and second derivatives with respect to the
reference coordinates, computed by forward-mode differentiation of the
analytic map (exact to rounding).  These are the inputs a user of the method
supplies (Section 6.1 describes the surface as a union of parameterized
patches); nothing here computes normals, curvature, weights or any other
quantity the method derives from them.

Surfaces (all outward oriented, u x v pointing out of the enclosed volume):

* ``cube_sphere``: equiangular gnomonic cube-sphere, 6 k^2 patches, optionally
  scaled per axis (ellipsoid), radially deformed (star shape) and rotated.
* ``torus``: n_theta x n_phi patches in (toroidal, poloidal) angle, with an
  optional angle-dependent tube radius (wobbly torus), whole or a band of toroidal angle.
* ``torus_boundary_curve``: samples of a poloidal circle bounding such a band.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch
from torch.func import jvp

__all__ = ["Surface", "gl_nodes", "cube_sphere", "torus", "torus_boundary_curve", "real_sph_harm_cartesian"]


@dataclass
class Surface:
    """Node data of a patch surface (FP64, row-major N x 3 arrays)."""

    name: str
    n_patches: int
    q: int
    x: np.ndarray
    xu: np.ndarray
    xv: np.ndarray
    xuu: np.ndarray
    xuv: np.ndarray
    xvv: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.n_patches * self.q * self.q


def gl_nodes(q: int) -> np.ndarray:
    """Gauss-Legendre nodes on [-1, 1] in increasing order (placement only)."""
    t, _ = np.polynomial.legendre.leggauss(q)
    return t


def _reference_grid(n_patches: int, q: int):
    t = torch.tensor(gl_nodes(q), dtype=torch.float64)
    uu = t.repeat_interleave(q)          # iu slow
    vv = t.repeat(q)                     # iv fast
    u = uu.repeat(n_patches)
    v = vv.repeat(n_patches)
    pid = torch.arange(n_patches).repeat_interleave(q * q)
    return pid, u, v


def _derivatives(fmap, u: torch.Tensor, v: torch.Tensor):
    """x, x_u, x_v, x_uu, x_uv, x_vv of a pointwise map (u, v) -> (N, 3)."""
    one = torch.ones_like(u)

    def d_u(uu, vv):
        return jvp(lambda w: fmap(w, vv), (uu,), (one,))[1]

    def d_v(uu, vv):
        return jvp(lambda w: fmap(uu, w), (vv,), (one,))[1]

    x = fmap(u, v)
    xu = d_u(u, v)
    xv = d_v(u, v)
    xuu = jvp(lambda w: d_u(w, v), (u,), (one,))[1]
    xuv = jvp(lambda w: d_u(u, w), (v,), (one,))[1]
    xvv = jvp(lambda w: d_v(u, w), (v,), (one,))[1]
    return [a.detach().cpu().numpy().copy() for a in (x, xu, xv, xuu, xuv, xvv)]


# Face frames (e, t1, t2) with t1 x t2 = e so that the face map is outward.
_FACES = [
    ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((-1, 0, 0), (0, 0, 1), (0, 1, 0)),
    ((0, 1, 0), (0, 0, 1), (1, 0, 0)),
    ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
    ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
    ((0, 0, -1), (0, 1, 0), (1, 0, 0)),
]


def cube_sphere(k: int, q: int, axes=(1.0, 1.0, 1.0), radial=None, rotation=None,
                name: str = "sphere") -> Surface:
    """Equiangular cube-sphere with k x k patches per face.

    ``radial``: optional torch function s -> r(s) > 0 of the unit vector s
    (N, 3), giving the star-shaped surface s * r(s).  ``axes`` scales the
    result per axis (ellipsoid), ``rotation`` (3x3 orthogonal, det +1) is then
    applied.
    """
    n_patches = 6 * k * k
    pid, u, v = _reference_grid(n_patches, q)
    face = pid // (k * k)
    ij = pid % (k * k)
    pi_ = ij // k
    pj = ij % k
    E = torch.tensor([f[0] for f in _FACES], dtype=torch.float64)[face]
    T1 = torch.tensor([f[1] for f in _FACES], dtype=torch.float64)[face]
    T2 = torch.tensor([f[2] for f in _FACES], dtype=torch.float64)[face]
    h = (math.pi / 2) / k
    ax = torch.tensor(axes, dtype=torch.float64)
    rot = None if rotation is None else torch.tensor(np.asarray(rotation), dtype=torch.float64)

    def fmap(uu, vv):
        xi = -math.pi / 4 + (pi_.to(torch.float64) + (uu + 1) / 2) * h
        eta = -math.pi / 4 + (pj.to(torch.float64) + (vv + 1) / 2) * h
        c = E + torch.tan(xi)[:, None] * T1 + torch.tan(eta)[:, None] * T2
        s = c / torch.linalg.norm(c, dim=1, keepdim=True)
        if radial is not None:
            s = s * radial(s)[:, None]
        y = s * ax
        if rot is not None:
            y = y @ rot.T
        return y

    arrs = _derivatives(fmap, u, v)
    return Surface(name, n_patches, q, *arrs, meta={"k": k, "axes": tuple(axes)})


def torus(n_theta: int, n_phi: int, q: int, R=1.0, r=0.4, name: str = "torus",
          theta_range: tuple[float, float] | None = None) -> Surface:
    """Torus with patches in (theta toroidal, phi poloidal).

    ``R`` and ``r`` are constants or torch functions of (theta, phi).
    x = ((R + r cos phi) cos theta, (R + r cos phi) sin theta, r sin phi);
    (u, v) <-> (theta, phi) gives the outward orientation.  ``theta_range`` = (theta0, theta1)
    covers only that band of toroidal angle (an open surface bounded by the two poloidal circles
    theta = theta0 and theta = theta1); None covers the whole torus.
    """
    n_patches = n_theta * n_phi
    pid, u, v = _reference_grid(n_patches, q)
    it = (pid // n_phi).to(torch.float64)
    ip = (pid % n_phi).to(torch.float64)

    def fmap(uu, vv):
        if theta_range is None:
            th = 2 * math.pi * (it + (uu + 1) / 2) / n_theta
        else:
            th = theta_range[0] + (theta_range[1] - theta_range[0]) * (it + (uu + 1) / 2) / n_theta
        ph = 2 * math.pi * (ip + (vv + 1) / 2) / n_phi
        rr = r(th, ph) if callable(r) else r * torch.ones_like(th)
        RR = R(th, ph) if callable(R) else R
        ring = RR + rr * torch.cos(ph)
        return torch.stack([ring * torch.cos(th), ring * torch.sin(th), rr * torch.sin(ph)], dim=1)

    arrs = _derivatives(fmap, u, v)
    meta = {"n_theta": n_theta, "n_phi": n_phi}
    if theta_range is not None:
        meta["theta_range"] = tuple(theta_range)
    return Surface(name, n_patches, q, *arrs, meta=meta)


def torus_boundary_curve(theta0: float, n: int, side: int, R=1.0, r=0.4) -> dict:
    """n equispaced samples t_j = 2 pi j / n of the poloidal circle theta = theta0 of the torus map
    of ``torus`` (t = phi, a smooth periodic parameterization of a boundary curve of a theta band).

    Returns the position ``x`` = y(theta0, t_j), its derivative along the curve ``xt`` = dy/dphi and
    ``d`` = side * dy/dtheta, the map's derivative across the curve, pointing out of the band for
    side = +1 at its upper end (theta0 = theta1) and side = -1 at its lower end.  All (n, 3), exact to
    rounding; the conormal and the arc-length element are left to the method.
    """
    t = torch.arange(n, dtype=torch.float64) * (2 * math.pi / n)
    th0 = torch.full_like(t, float(theta0))

    def fmap(th, ph):
        rr = r(th, ph) if callable(r) else r * torch.ones_like(th)
        RR = R(th, ph) if callable(R) else R
        ring = RR + rr * torch.cos(ph)
        return torch.stack([ring * torch.cos(th), ring * torch.sin(th), rr * torch.sin(ph)], dim=1)

    one = torch.ones_like(t)
    x = fmap(th0, t)
    xt = jvp(lambda w: fmap(th0, w), (t,), (one,))[1]
    xth = jvp(lambda w: fmap(w, t), (th0,), (one,))[1]
    return {"x": x.numpy().copy(), "xt": xt.numpy().copy(), "d": (side * xth).numpy().copy()}


def _legendre_deriv_coeffs(l: int, m: int) -> np.ndarray:
    """Power-series coefficients (ascending) of d^m/dz^m P_l(z)."""
    c = np.zeros(l + 1)
    c[l] = 1.0
    p = np.polynomial.legendre.leg2poly(c)
    for _ in range(m):
        p = np.polynomial.polynomial.polyder(p)
    return p


def real_sph_harm_cartesian(l: int, m: int, x: torch.Tensor, homogeneous: bool = False) -> torch.Tensor:
    """Orthonormal real spherical harmonic Y_lm of the direction of x (N, 3).

    m > 0 uses cos(m phi), m < 0 uses sin(|m| phi).  With ``homogeneous`` the
    result is the solid harmonic |x|^l Y_lm(x / |x|), a harmonic polynomial.
    """
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    if m != 0:
        norm *= math.sqrt(2.0)
    rn = torch.linalg.norm(x, dim=1)
    z = x[:, 2]
    coeffs = _legendre_deriv_coeffs(l, am)
    # sum_k c_k z^k r^(l-am-k): homogeneous of degree l-am (parity l-am).
    poly = torch.zeros_like(z)
    deg = l - am
    for kk, ck in enumerate(coeffs):
        if ck != 0.0:
            poly = poly + ck * z ** kk * rn ** (deg - kk)
    w = torch.complex(x[:, 0], x[:, 1]) ** am
    ang = w.real if m >= 0 else w.imag
    val = norm * poly * ang
    if not homogeneous:
        val = val / rn ** l
    return val
