"""The synthetic workloads: surfaces, coefficients and right-hand sides, all seeded.

=====  ==========================================================================
name   workload
=====  ==========================================================================
sphere unit sphere, cube-sphere k=2, q=8 (24 patches, 1,536 nodes);
       a = 1 + 0.5 sin(2 x1) cos(x2) (or a = 1); f from u = (x^2 - y^2) z
ellip  ellipsoid (1, 0.8, 0.6), cube-sphere k=16, q=10 (1,536 patches,
       153,600 nodes); a = exp(0.3 x1 x2); f = 20 solid harmonics, N(0,1)
star   r = 1 + 0.25 sum_8 w_k Y_k (1 <= l <= 4, w ~ U(-1,1)), cube-sphere
       k=37, q=8 (8,214 patches, 525,696 nodes); a = 2^tanh(s(x)) seed field
torus  wobbly torus R = 1, r = 0.4 (1 + 0.2 cos 5 theta sin 3 phi), 256 x 128
       patches, q=8 (2,097,152 nodes); a = 1 + 0.5 tanh(sin 3 x1); 16 RHS
serve  request stream: sphere / random-axis ellipsoid / torus, 2e3..2e5 nodes
edge   the paper's wavy torus cut to the band 4 pi / 3 < u < 2 pi (17 x 18 patches, q=8,
       19,584 nodes) and its two boundary circles, 200 equispaced samples each;
       a = 1 or exp(0.3 x1 x2); boundary density mu = exp(x1)
=====  ==========================================================================

Every builder takes a size knob so that tests can run the same family at
oracle-friendly sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import fields as F
from .surfaces import Surface, cube_sphere, real_sph_harm_cartesian, torus, torus_boundary_curve

__all__ = [
    "Problem", "sphere_problem", "ellipsoid_problem", "star_problem", "wobbly_torus_problem",
    "wavy_torus_problem", "helmholtz_sphere_problem", "helmholtz_ellipsoid_problem", "serving_requests",
    "random_density", "EdgeSamples", "wavy_torus_piece_problem",
]


@dataclass
class Problem:
    surface: Surface
    a: np.ndarray            # (N,)
    grad_a: np.ndarray       # (N, 3) ambient gradient
    f: np.ndarray            # (N, n_rhs)
    name: str = ""
    meta: dict = field(default_factory=dict)
    c: np.ndarray | None = None   # (N,) zero-order coefficient c < 0, or None for c = 0
    b: np.ndarray | None = None   # (N, 3) advection field (ambient vectors), or None

    @property
    def n(self) -> int:
        return self.surface.n


def _sphere_manufactured_rhs(x: np.ndarray, a_fn, b: np.ndarray | None = None) -> tuple[np.ndarray, np.ndarray]:
    """On the unit sphere (exact normal = position): u = (x^2 - y^2) z and
    f = div_G(a grad_G u) = a * (-12 u) + grad_G a . grad_G u (u is a degree-3 harmonic),
    plus b . grad_G u when an advection field b is given."""
    X = torch.tensor(x, dtype=torch.float64)
    nrm = X / torch.linalg.norm(X, dim=1, keepdim=True)
    u = (X[:, 0] ** 2 - X[:, 1] ** 2) * X[:, 2]
    gu = torch.stack([2 * X[:, 0] * X[:, 2], -2 * X[:, 1] * X[:, 2], X[:, 0] ** 2 - X[:, 1] ** 2], dim=1)
    a, ga = F.eval_field(a_fn, x)
    ga = torch.tensor(ga)
    tang = lambda g: g - nrm * (nrm * g).sum(dim=1, keepdim=True)
    f = torch.tensor(a) * (-12.0 * u) + (tang(ga) * tang(gu)).sum(dim=1)
    if b is not None:
        f = f + (torch.tensor(b) * tang(gu)).sum(dim=1)
    return f.numpy().copy(), u.numpy().copy()


def sphere_problem(k: int = 2, q: int = 8, const_a: bool = False) -> Problem:
    s = cube_sphere(k, q, name="sphere")
    a_fn = F.a_const(1.0) if const_a else F.a_sphere_cfg
    a, ga = F.eval_field(a_fn, s.x)
    f, u = _sphere_manufactured_rhs(s.x, a_fn)
    return Problem(s, a, ga, f[:, None], name=f"sphere_k{k}_q{q}" + ("_a1" if const_a else ""),
                   meta={"u_exact": u})


def ellipsoid_problem(k: int = 16, q: int = 10, axes=(1.0, 0.8, 0.6), seed: int = 1, n_rhs: int = 1) -> Problem:
    s = cube_sphere(k, q, axes=axes, name="ellipsoid")
    a, ga = F.eval_field(F.a_exp_xy, s.x)
    f = np.stack([F.solid_harmonic_rhs(s.x, seed + 100 * r) for r in range(n_rhs)], axis=1)
    return Problem(s, a, ga, f, name=f"ellipsoid_k{k}_q{q}")


def _star_radial(seed: int):
    rng = np.random.default_rng(seed)
    pool = [(l, m) for l in range(1, 5) for m in range(-l, l + 1)]
    pick = rng.choice(len(pool), size=8, replace=False)
    lms = [pool[i] for i in sorted(pick)]
    w = rng.uniform(-1, 1, 8)

    def radial(s):
        acc = torch.zeros(s.shape[0], dtype=s.dtype)
        for wk, (l, m) in zip(w, lms):
            acc = acc + float(wk) * real_sph_harm_cartesian(l, m, s)
        return 1.0 + 0.25 * acc

    return radial


def star_problem(k: int = 37, q: int = 8, seed: int = 2, n_rhs: int = 1) -> Problem:
    s = cube_sphere(k, q, radial=_star_radial(seed), name="star")
    a, ga = F.eval_field(F.a_seed_field(seed), s.x)
    f = np.stack([F.solid_harmonic_rhs(s.x, seed + 100 * r) for r in range(n_rhs)], axis=1)
    return Problem(s, a, ga, f, name=f"star_k{k}_q{q}")


def wobbly_torus_problem(n_theta: int = 256, n_phi: int = 128, q: int = 8, n_rhs: int = 16) -> Problem:
    rfun = lambda th, ph: 0.4 * (1.0 + 0.2 * torch.cos(5 * th) * torch.sin(3 * ph))
    s = torus(n_theta, n_phi, q, R=1.0, r=rfun, name="wobbly_torus")
    a, ga = F.eval_field(F.a_tanh_sin, s.x)
    f = np.stack([F.solid_harmonic_rhs(s.x, 4 * 100 + r) for r in range(n_rhs)], axis=1)
    return Problem(s, a, ga, f, name=f"wobbly_torus_{n_theta}x{n_phi}_q{q}")


def helmholtz_sphere_problem(k: int = 2, q: int = 8, c0: float | None = None, omega: float | None = None,
                             swirl: bool = False, positive: bool = False) -> Problem:
    """Unit sphere for div_G(a grad_G u) + b . grad_G u + c u = f with c < 0 (the modified Helmholtz
    type) or, with ``positive``, c > 0 (the Helmholtz type); b = 0 unless ``omega`` (the rotation
    omega e3 x x) or ``swirl`` (fields.b_swirl) is given.

    c0 given: a = 1 and c = c0 (constant, either sign; f = 0, the caller chooses f, e.g. spherical
    harmonics).  c0 None: a = 2 + x3 and c = -4 - exp(x1 / 2) (or c = 2 (1 + 0.2 x2) with
    ``positive``), with the manufactured solution u = (x^2 - y^2) z (a degree-3 harmonic,
    Delta_G u = -12 u on the unit sphere): f = grad_G a . grad_G u - 12 a u + b . grad_G u + c u.
    """
    s = cube_sphere(k, q, name="sphere")
    b = F.b_rotation_z(s.x, omega) if omega is not None else (F.b_swirl(s.x) if swirl else None)
    tag = (f"_w{omega}" if omega is not None else "") + ("_swirl" if swirl else "")
    if c0 is not None:
        a, ga = F.eval_field(F.a_const(1.0), s.x)
        c = np.full(s.n, float(c0))
        return Problem(s, a, ga, np.zeros((s.n, 1)), name=f"helmholtz_sphere_k{k}_q{q}_c{c0}{tag}", c=c, b=b)
    a_fn = F.a_linear_z
    a, ga = F.eval_field(a_fn, s.x)
    c, _ = F.eval_field(F.c_pos_y if positive else F.c_exp_x, s.x)
    f, u = _sphere_manufactured_rhs(s.x, a_fn, b)
    tag += "_pos" if positive else ""
    return Problem(s, a, ga, (f + c * u)[:, None], name=f"helmholtz_sphere_k{k}_q{q}_var{tag}", c=c, b=b,
                   meta={"u_exact": u})


def helmholtz_ellipsoid_problem(k: int = 4, q: int = 8, axes=(1.0, 0.8, 0.6), seed: int = 1, n_rhs: int = 1,
                                swirl: bool = False, positive: bool = False, c_scale: float = 1.0):
    """Ellipsoid with the variable coefficients a = 2 + x3 and c = -4 - exp(x1 / 2) (c < 0; with
    ``positive`` c = 2 (1 + 0.2 x2) > 0), c multiplied by ``c_scale``, and right-hand sides of 20 solid
    harmonics (seeded); with ``swirl`` the advection field fields.b_swirl as well."""
    s = cube_sphere(k, q, axes=axes, name="ellipsoid")
    a, ga = F.eval_field(F.a_linear_z, s.x)
    c, _ = F.eval_field(F.c_pos_y if positive else F.c_exp_x, s.x)
    c = c * c_scale
    f = np.stack([F.solid_harmonic_rhs(s.x, seed + 100 * r) for r in range(n_rhs)], axis=1)
    name = (f"helmholtz_ellipsoid_k{k}_q{q}" + ("_swirl" if swirl else "") + ("_pos" if positive else "") +
            (f"_cx{c_scale:g}" if c_scale != 1.0 else ""))
    return Problem(s, a, ga, f, name=name, c=c, b=F.b_swirl(s.x) if swirl else None)


def wavy_torus_problem(n_u: int = 51, n_v: int = 18, q: int = 8, seed: int = 5) -> Problem:
    """The paper's wavy torus, x(u, v) = ((3 + cos v + 0.6 cos 5u) cos u, (3 + cos v + 0.6 cos 5u) sin u,
    sin v), as n_u x n_v patches (51 x 18 x 8 x 8 = 58,752 nodes by default), with a = 1 (the
    Laplace-Beltrami remainder) and the N-body density sigma_i = (x_i)_1 + eta_i, eta ~ N(0, 1)
    (seeded), in ``meta["sigma"]``; f is that density too."""
    rfun = lambda th, ph: 1.0 + 0.0 * th
    s = torus(n_u, n_v, q, R=lambda th, ph: 3.0 + 0.6 * torch.cos(5 * th), r=rfun, name="wavy_torus")
    a, ga = F.eval_field(F.a_const(1.0), s.x)
    sigma = s.x[:, 0] + np.random.default_rng(seed).normal(size=s.n)
    return Problem(s, a, ga, sigma[:, None].copy(), name=f"wavy_torus_{n_u}x{n_v}_q{q}", meta={"sigma": sigma})


@dataclass
class EdgeSamples:
    """Equispaced samples of the closed boundary curves of an open surface, curve after curve:
    curve k owns rows [offsets[k], offsets[k + 1]), sample j of a curve of n samples sits at
    t = 2 pi j / n of its periodic parameterization.  x, xt (= dx/dt) and d (the surface map's
    derivative across the curve, pointing out of the surface) are (M, 3); a (M,) and grad_a (M, 3,
    ambient) are the coefficient there; mu (M, n_rhs) is a boundary density."""

    x: np.ndarray
    xt: np.ndarray
    d: np.ndarray
    a: np.ndarray
    grad_a: np.ndarray
    mu: np.ndarray
    offsets: np.ndarray

    @property
    def m(self) -> int:
        return self.x.shape[0]


def wavy_torus_piece_problem(n_u: int = 17, n_v: int = 18, q: int = 8, n_edge=200, variable_a: bool = False,
                             n_rhs: int = 1, seed: int = 7) -> Problem:
    """The paper's wavy torus (``wavy_torus_problem``'s map) restricted to the band 4 pi / 3 < u < 2 pi
    (the open surface of Section 7.5), n_u x n_v patches (17 x 18 x 8 x 8 = 19,584 nodes by default:
    the band's third of the 51 x 18 closed surface), and its two boundary circles u = 4 pi / 3 and
    u = 2 pi with ``n_edge`` samples each (an int, or one count per curve).  a = 1 (the
    Laplace-Beltrami problem) or exp(0.3 x1 x2).  The boundary density is mu = exp(x1) in column 0
    (Section 7.5's edge-quadrature test) and seeded N(0, 1) values in the other columns; it is in
    ``meta["edge"]`` (EdgeSamples), with f = exp(x1) at the nodes."""
    Rf = lambda th, ph: 3.0 + 0.6 * torch.cos(5 * th)
    rf = lambda th, ph: 1.0 + 0.0 * th
    band = (4 * math.pi / 3, 2 * math.pi)
    s = torus(n_u, n_v, q, R=Rf, r=rf, name="wavy_torus_piece", theta_range=band)
    fa = F.a_exp_xy if variable_a else F.a_const(1.0)
    a, ga = F.eval_field(fa, s.x)
    counts = [n_edge, n_edge] if isinstance(n_edge, int) else list(n_edge)
    curves = [torus_boundary_curve(band[0], counts[0], -1, R=Rf, r=rf),
              torus_boundary_curve(band[1], counts[1], +1, R=Rf, r=rf)]
    x = np.concatenate([c["x"] for c in curves])
    ea, ega = F.eval_field(fa, x)
    mu = np.empty((x.shape[0], n_rhs))
    mu[:, 0] = np.exp(x[:, 0])
    if n_rhs > 1:
        mu[:, 1:] = np.random.default_rng(seed).normal(size=(x.shape[0], n_rhs - 1))
    edge = EdgeSamples(x, np.concatenate([c["xt"] for c in curves]), np.concatenate([c["d"] for c in curves]),
                       ea, ega, mu, np.array([0, counts[0], counts[0] + counts[1]], dtype=np.int64))
    f = np.exp(s.x[:, 0])[:, None].copy()
    name = f"wavy_torus_piece_{n_u}x{n_v}_q{q}_e{counts[0]}" + ("_vara" if variable_a else "")
    return Problem(s, a, ga, f, name=name, meta={"edge": edge})


def serving_requests(n_requests: int = 256, seed: int = 3, n_min: float = 2e3, n_max: float = 2e5, q: int = 8):
    """Yield ``n_requests`` (kind, Problem) pairs with log-uniform node counts."""
    rng = np.random.default_rng(seed)
    for r in range(n_requests):
        kind = ["sphere", "ellipsoid", "torus"][rng.integers(3)]
        n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        if kind == "torus":
            n = max(4, int(round(math.sqrt(n_target / (2 * q * q)))))
            rr = float(rng.uniform(0.3, 0.5))
            s = torus(2 * n, n, q, R=1.0, r=rr, name="torus")
        else:
            k = max(2, int(round(math.sqrt(n_target / (6 * q * q)))))
            axes = (1.0, 1.0, 1.0) if kind == "sphere" else tuple(rng.uniform(0.5, 1.5, 3))
            s = cube_sphere(k, q, axes=axes, name=kind)
        a, ga = F.eval_field(F.a_seed_field(int(rng.integers(1 << 30))), s.x)
        f = F.solid_harmonic_rhs(s.x, int(rng.integers(1 << 30)))[:, None]
        yield kind, Problem(s, a, ga, f, name=f"req{r}_{kind}_{s.n}")


def random_density(n: int, n_rhs: int = 1, seed: int = 0) -> np.ndarray:
    """Seeded N(0,1) density (N, n_rhs) for operator-apply tests."""
    return np.random.default_rng(seed).normal(size=(n, n_rhs))
