"""Pins of the oracle's edge operators (open surfaces: eq:BC_rep, eq:DirichletRep, Lemma lem:surf_term,
Lemma lem:Dirichlet_surf_term; edge quadrature of Section 6.1.4; the edge-quadrature test of Section 7.5)
against facts that do not come from the oracle's own formulas:

* trigonometric interpolation reproduces trigonometric polynomials of degree <= n/2 exactly (with the
  Nyquist mode cos(n t / 2) for even n), and converges spectrally for an analytic periodic function;
* the conormal at the circle u = 2 pi of the wavy-torus band, which lies in the plane y = 0 where the
  map's u-derivative is (0, ring, 0), is exactly +e_y;
* N and T are the derivatives of the parametrix and of the remainder along nu at the source, with the
  coefficient a(x') moving with the source: fourth-order central differences of the oracle's K and R
  (R is pinned against eq:diff_remainder elsewhere);
* on a planar region with a = 1, N_gamma[1](x) = 1 inside the boundary curve and 0 outside (the
  angle the curve subtends, over 2 pi), K_gamma[1] at the centre of a circle of radius rho is
  rho log(rho), and R_gamma and T_gamma vanish (n . r = 0, H = 0, grad a = 0);
* the oversampled trapezoid sums equal adaptive quadrature (scipy's quad) of the exact integrand on
  the exact curve, with the conormal built independently as n x tau;
* Section 7.5's observation: the error at targets near the edge falls quickly once the oversampling
  resolves the near singularity;
* Lemma lem:surf_term and Lemma lem:Dirichlet_surf_term: away from the boundary, div_G(a grad_G .)
  applied to K_gamma[mu] and N_gamma[mu] (spectral differentiation on the patches) gives R_gamma[mu] and
  T_gamma[mu], with an error that falls spectrally in the patch order;
* Theorem thm:NeumannBCsrep for the curve potential: the conormal derivative of K_gamma[mu] on the
  surface side, extrapolated to gamma, equals -mu / (2a) + K'_gamma[mu] (the jump and the edge-to-edge
  operator of the Neumann row), the error falling spectrally with the patch order;
* the double-layer jump for the Dirichlet representation (a = 1): N_gamma[mu] extrapolated to gamma
  equals +mu / (2a) + D_gamma[mu] (D_gamma the double layer on the curve), the sign fixed by
  K = log r / (2 pi a) and the outward conormal;
* K'_gamma (targets on gamma): on a circle of radius rho in a plane with a = 1 the kernel is the
  constant 1 / (4 pi rho), so K'_gamma[1] = 1/2 at every sample; the diagonal limit equals the kernel
  at nearby points of the exact curve; the trapezoid sums on an ellipse and on the wavy-torus circles
  equal adaptive quadrature of the exact integrand; the spectral derivative is exact on trigonometric
  polynomials.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si

from paper_2401_12501_amd.inputs import EdgeSamples, wavy_torus_piece_problem
from oracle.edge import (conormal, dlayer_gamma, edge_apply, edge_points, fourier_derivative, fourier_upsample,
                         kprime_gamma, n_kernel, t_kernel, targets_of)
from oracle.kernels import parametrix, remainder
from oracle.operator import OracleOperator


@pytest.mark.parametrize("n", [16, 15])
@pytest.mark.parametrize("m", [1, 3, 8])
def test_fourier_upsample_trig_polynomial(n, m):
    def f(t):
        v = 1.0 + np.cos(t) - 0.7 * np.sin(2 * t) + 0.3 * np.sin(3 * t) + 0.1 * np.cos(7 * t)
        if n % 2 == 0:
            v = v + 0.2 * np.cos(n / 2 * t)
        return v
    t = 2 * np.pi * np.arange(n) / n
    tf = 2 * np.pi * np.arange(m * n) / (m * n)
    g = fourier_upsample(np.stack([f(t), 2 * f(t)], axis=1), m)
    assert np.abs(g[:, 0] - f(tf)).max() < 1e-13
    assert np.abs(g[:, 1] - 2 * f(tf)).max() < 2e-13


def test_fourier_upsample_analytic_spectral():
    n, m = 64, 5
    t = 2 * np.pi * np.arange(n) / n
    tf = 2 * np.pi * np.arange(m * n) / (m * n)
    g = fourier_upsample(np.exp(np.cos(t)), m)
    assert np.abs(g - np.exp(np.cos(tf))).max() < 1e-13


def test_conormal_on_the_plane_y0_circle():
    p = wavy_torus_piece_problem(n_u=4, n_v=6, q=6, n_edge=40)
    e = p.meta["edge"]
    upper = slice(int(e.offsets[1]), int(e.offsets[2]))
    nu = conormal(e.xt[upper], e.d[upper])
    np.testing.assert_allclose(nu, np.tile([0.0, 1.0, 0.0], (40, 1)), atol=1e-14)
    lower = slice(int(e.offsets[0]), int(e.offsets[1]))
    nl = conormal(e.xt[lower], e.d[lower])
    assert np.abs(np.sum(nl * e.xt[lower], axis=1)).max() < 1e-13
    # out of the band at u = 4 pi / 3: against increasing u (the map's u-derivative is -d there)
    assert np.all(np.sum(nl * e.d[lower], axis=1) > 0.5)


def _a(y):
    return np.exp(0.3 * y[0] * y[1])


def _grad_a(y):
    return _a(y) * 0.3 * np.array([y[1], y[0], 0.0])


def _d4(f, h):
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


def test_n_and_t_kernels_are_source_derivatives():
    rng = np.random.default_rng(11)
    for _ in range(6):
        x, y = rng.normal(size=3), rng.normal(size=3)
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        nu = rng.normal(size=3)
        nu /= np.linalg.norm(nu)
        gs = rng.normal(size=3)
        gs -= n * (n @ gs)
        H, a_t = rng.normal(), 1.0 + rng.random()
        nga = nu @ _grad_a(y)
        for h in (1e-3, 5e-4):
            dK = _d4(lambda s: parametrix(x, y + s * nu, _a(y + s * nu)), h)
            dR = _d4(lambda s: remainder(x, n, H, a_t, gs, y + s * nu, _a(y + s * nu)), h)
            vK = n_kernel(x, y, nu, _a(y), nga)
            vT = t_kernel(x, n, H, a_t, gs, y, nu, _a(y), nga)
            assert abs(vK - dK) <= 1e-8 * max(1.0, abs(vK)), (vK, dK)
            assert abs(vT - dR) <= 1e-7 * max(1.0, abs(vT)), (vT, dR)


def _planar_edge(n, A=1.3, B=0.8):
    t = 2 * np.pi * np.arange(n) / n
    x = np.stack([A * np.cos(t), B * np.sin(t), 0 * t], axis=1)
    xt = np.stack([-A * np.sin(t), B * np.cos(t), 0 * t], axis=1)
    d = np.stack([np.cos(t), np.sin(t), 0 * t], axis=1)     # outward, not normal to the curve
    one = np.ones(n)
    return EdgeSamples(x, xt, d, one, np.zeros((n, 3)), one[:, None].copy(), np.array([0, n]))


def _planar_targets(pts):
    k = len(pts)
    return {"x": np.asarray(pts, dtype=np.float64), "n": np.tile([0.0, 0.0, 1.0], (k, 1)), "H": np.zeros(k),
            "a": np.ones(k), "gs": np.zeros((k, 3))}


def test_planar_gauss_identity_and_vanishing_remainder():
    e = _planar_edge(96)
    inside = [[0.0, 0.0, 0.0], [0.5, 0.2, 0.0], [-0.9, -0.3, 0.0], [1.2, 0.0, 0.0]]
    outside = [[1.6, 0.0, 0.0], [0.0, 1.5, 0.0], [3.0, 2.0, 0.0]]
    tgt = _planar_targets(inside + outside)
    N = edge_apply("N", tgt, e, e.mu, 16)[:, 0]
    np.testing.assert_allclose(N[:4], 1.0, atol=1e-10)
    np.testing.assert_allclose(N[4:], 0.0, atol=1e-10)
    for kind in ("R", "T"):
        assert np.abs(edge_apply(kind, tgt, e, e.mu, 4)).max() < 1e-13


def test_circle_centre_single_layer():
    rho, n = 0.7, 32
    e = _planar_edge(n, rho, rho)
    K = edge_apply("K", _planar_targets([[0.0, 0.0, 0.0]]), e, e.mu, 1)[0, 0]
    assert abs(K - rho * math.log(rho)) < 1e-14


# ------------------------------------------------------------------ exact curve, adaptive quadrature
_BAND = (4 * math.pi / 3, 2 * math.pi)


def _curve(th0, t):
    """Exact boundary circle theta = th0 of the wavy torus: y, dy/dt, dy/dtheta."""
    R = 3.0 + 0.6 * math.cos(5 * th0)
    dR = -3.0 * math.sin(5 * th0)
    ring = R + math.cos(t)
    y = np.array([ring * math.cos(th0), ring * math.sin(th0), math.sin(t)])
    yt = np.array([-math.sin(t) * math.cos(th0), -math.sin(t) * math.sin(th0), math.cos(t)])
    yth = np.array([dR * math.cos(th0) - ring * math.sin(th0), dR * math.sin(th0) + ring * math.cos(th0), 0.0])
    return y, yt, yth


def _exact_integral(kind, tgt, i, th0, side):
    x, n, H, a_t, gs = tgt["x"][i], tgt["n"][i], tgt["H"][i], tgt["a"][i], tgt["gs"][i]

    def g(t):
        y, yt, yth = _curve(th0, t)
        ns = np.cross(yth, yt)
        ns /= np.linalg.norm(ns)
        nu = np.cross(ns, yt / np.linalg.norm(yt))
        nu *= np.sign(side * (nu @ yth))
        w = np.linalg.norm(yt) * math.exp(y[0])
        if kind == "K":
            k = parametrix(x, y, _a(y))
        elif kind == "N":
            k = n_kernel(x, y, nu, _a(y), nu @ _grad_a(y))
        elif kind == "R":
            k = remainder(x, n, H, a_t, gs, y, _a(y))
        else:
            k = t_kernel(x, n, H, a_t, gs, y, nu, _a(y), nu @ _grad_a(y))
        return float(k) * w

    # break points at the closest sample of the curve to the target
    ts = np.linspace(0, 2 * np.pi, 721)
    tc = ts[np.argmin([np.linalg.norm(_curve(th0, t)[0] - x) for t in ts])]
    brk = sorted({0.0, float(tc), 2 * np.pi})
    return sum(si.quad(g, lo, hi, epsabs=1e-14, epsrel=1e-13, limit=400)[0] for lo, hi in zip(brk[:-1], brk[1:])
               if hi > lo)


@pytest.fixture(scope="module")
def piece():
    p = wavy_torus_piece_problem(n_u=4, n_v=6, q=6, n_edge=200, variable_a=True)
    orc = OracleOperator.from_problem(p)
    return p, targets_of(orc)


def _near_far(tgt):
    x = tgt["x"]
    th = np.mod(np.arctan2(x[:, 1], x[:, 0]), 2 * np.pi)
    dist = np.minimum(np.abs(th - _BAND[0]), np.abs(2 * np.pi - th))
    return int(np.argmin(dist)), int(np.argmax(dist))


@pytest.mark.parametrize("kind", ["K", "N", "R", "T"])
def test_trapezoid_matches_adaptive_quadrature(piece, kind):
    p, tgt = piece
    e = p.meta["edge"]
    near, far = _near_far(tgt)
    for i, m, tol in ((far, 1, 1e-12), (near, 64, 1e-9)):
        val = edge_apply(kind, tgt, e, e.mu, m, targets=[i])[0, 0]
        ref = _exact_integral(kind, tgt, i, _BAND[0], -1) + _exact_integral(kind, tgt, i, _BAND[1], +1)
        assert abs(val - ref) <= tol * max(1.0, abs(ref)), (kind, i, m, val, ref)


@pytest.fixture(scope="module")
def fine_piece():
    p = wavy_torus_piece_problem(n_u=16, n_v=4, q=8, n_edge=200, variable_a=True)
    return p, targets_of(OracleOperator.from_problem(p))


@pytest.mark.parametrize("kind", ["R", "T"])
def test_error_falls_with_oversampling(fine_piece, kind):
    """Section 7.5: at the nodes nearest the boundary (within about a third of the sample spacing of
    the curve on this surface, 16 patches across the band) the error against the finest rule falls by
    orders of magnitude as the oversampling factor grows."""
    p, tgt = fine_piece
    e = p.meta["edge"]
    x = tgt["x"]
    th = np.mod(np.arctan2(x[:, 1], x[:, 0]), 2 * np.pi)
    dist = np.minimum(np.abs(th - _BAND[0]), np.abs(2 * np.pi - th))
    idx = np.argsort(dist)[:12]
    ref = edge_apply(kind, tgt, e, e.mu, 128, targets=idx)[:, 0]
    errs = [np.abs(edge_apply(kind, tgt, e, e.mu, m, targets=idx)[:, 0] - ref).max() / np.abs(ref).max()
            for m in (1, 4, 16, 64)]
    assert errs[0] > 1e-2 and errs[-1] < 1e-9, errs
    assert all(b < a or b < 1e-13 for a, b in zip(errs, errs[1:])), errs


def test_edge_points_weights_sum_to_length():
    """The trapezoid weights of a circle of radius rho sum to its length at any oversampling."""
    e = _planar_edge(24, 0.9, 0.9)
    for m in (1, 2, 7):
        assert abs(edge_points(e, m)["w"].sum() - 2 * math.pi * 0.9) < 1e-13


# ------------------------------------------------------------------ K'_gamma, targets on the curve
@pytest.mark.parametrize("n", [16, 15])
def test_fourier_derivative_trig_polynomial(n):
    t = 2 * np.pi * np.arange(n) / n
    f = 1.0 + np.cos(t) - 0.7 * np.sin(2 * t) + 0.3 * np.sin(5 * t)
    df = -np.sin(t) - 1.4 * np.cos(2 * t) + 1.5 * np.cos(5 * t)
    if n % 2 == 0:
        f = f + 0.2 * np.cos(n / 2 * t)      # its derivative vanishes at the samples
    assert np.abs(fourier_derivative(f) - df).max() < 1e-13


def test_kprime_circle_is_one_half():
    for rho, n in ((0.7, 12), (2.0, 33)):
        e = _planar_edge(n, rho, rho)
        v = kprime_gamma(e, np.ones(n))[:, 0]
        np.testing.assert_allclose(v, 0.5, atol=1e-14)


def _ellipse(t, A=1.3, B=0.8):
    return (np.array([A * np.cos(t), B * np.sin(t), 0.0]), np.array([-A * np.sin(t), B * np.cos(t), 0.0]),
            np.array([-A * np.cos(t), -B * np.sin(t), 0.0]))


def test_kprime_limit_is_the_kernel_near_the_diagonal():
    """The diagonal value equals the kernel at x' = gamma(t + h) as h -> 0 (first order in h)."""
    n = 64
    e = _planar_edge(n)
    j = 5
    t0 = 2 * np.pi * j / n
    x, xt, _ = _ellipse(t0)
    nu = conormal(xt[None], np.array([[np.cos(t0), np.sin(t0), 0.0]]))[0]
    mu = np.zeros(n)
    mu[j] = 1.0
    lim = kprime_gamma(e, mu)[j, 0] / (2 * np.pi / n * np.linalg.norm(xt))
    vals = []
    for h in (1e-3, 5e-4):
        y = _ellipse(t0 + h)[0]
        vals.append(nu @ (x - y) / (2 * np.pi * np.sum((x - y) ** 2)))
    extrap = 2 * vals[1] - vals[0]          # Richardson: the kernel is smooth in h
    assert abs(extrap - lim) < 1e-6 * abs(lim), (extrap, lim)


def _kprime_exact(x, nu, curve, a_fn, mu_fn, t_at):
    def g(t):
        y, yt = curve(t)
        r = x - y
        return float(nu @ r / (2 * np.pi * a_fn(y) * (r @ r))) * np.linalg.norm(yt) * mu_fn(y)
    return si.quad(g, t_at, t_at + 2 * np.pi, epsabs=1e-14, epsrel=1e-13, limit=400)[0]


def test_kprime_ellipse_matches_adaptive_quadrature():
    n = 96
    e = _planar_edge(n)
    e.mu[:, 0] = np.exp(e.x[:, 0])
    v = kprime_gamma(e, e.mu)[:, 0]
    nu = conormal(e.xt, e.d)
    for j in (0, 17, 50):
        t0 = 2 * np.pi * j / n
        ref = _kprime_exact(e.x[j], nu[j], lambda t: _ellipse(t)[:2], lambda y: 1.0, lambda y: np.exp(y[0]), t0)
        assert abs(v[j] - ref) < 1e-12 * max(1.0, abs(ref)), (j, v[j], ref)


def test_kprime_torus_circles_match_adaptive_quadrature():
    """Both boundary circles of the band: the target's own circle (smooth kernel through the
    diagonal) and the other circle (far), variable a, mu = exp(x1)."""
    p = wavy_torus_piece_problem(n_u=4, n_v=6, q=6, n_edge=120, variable_a=True)
    e = p.meta["edge"]
    v = kprime_gamma(e, e.mu)[:, 0]
    nu = conormal(e.xt, e.d)
    for j in (0, 37, 150):
        own = 0 if j < 120 else 1
        t0 = 2 * np.pi * (j - 120 * own) / 120
        ref = 0.0
        for c, (th0, side) in enumerate(((_BAND[0], -1), (_BAND[1], +1))):
            ref += _kprime_exact(e.x[j], nu[j], lambda t, th0=th0: _curve(th0, t)[:2], _a, lambda y: math.exp(y[0]),
                                 t0 if c == own else 0.0)
        assert abs(v[j] - ref) < 1e-11 * max(1.0, abs(ref)), (j, v[j], ref)


# ------------------------------------------------------------------ the lemmas: D K_gamma = R_gamma, D N_gamma = T_gamma
def _lemma_errors(n_u, q):
    from _surface_ops import middle_row_nodes, surface_operator
    p = wavy_torus_piece_problem(n_u=n_u, n_v=12, q=q, n_edge=200, variable_a=True)
    tgt = targets_of(OracleOperator.from_problem(p))
    e = p.meta["edge"]
    idx = middle_row_nodes(n_u, 12, q)
    v = {k: edge_apply(k, tgt, e, e.mu, 16, targets=idx)[:, 0] for k in "KNRT"}
    s = p.surface
    DK = surface_operator(v["K"], p.a[idx], s.xu[idx], s.xv[idx], q)
    DN = surface_operator(v["N"], p.a[idx], s.xu[idx], s.xv[idx], q)
    return (np.abs(DK - v["R"]).max() / np.abs(v["R"]).max(), np.abs(DN - v["T"]).max() / np.abs(v["T"]).max())


def test_surface_operator_of_edge_potentials():
    """div_G(a grad_G K_gamma[mu]) = R_gamma[mu] and div_G(a grad_G N_gamma[mu]) = T_gamma[mu] in the
    interior (the lemmas), on the middle row of the band, 12 x 12 patches of 12 x 12 nodes; and the
    differentiation error falls spectrally with the patch order (q = 10 to 14 on 8 rows)."""
    eK, eN = _lemma_errors(12, 12)
    assert eK < 1e-6 and eN < 1e-6, (eK, eN)
    lo, hi = _lemma_errors(8, 10), _lemma_errors(8, 14)
    assert hi[0] < lo[0] / 100 and hi[1] < lo[1] / 100, (lo, hi)


def _jump_error(q, K_fn, Kp_fn):
    """max |nu . grad K_gamma[mu] at gamma - (-mu / 2a + K'_gamma[mu])| / max|...| on the band's upper
    circle (u = 2 pi, the last row of patches), mu = exp(x1), a = exp(0.3 x1 x2); K_fn(problem, node
    indices) and Kp_fn(problem) supply the two operators' values."""
    from _surface_ops import conormal_derivative_at_edge, trig_eval
    n_u, n_v = 8, 12
    p = wavy_torus_piece_problem(n_u=n_u, n_v=n_v, q=q, n_edge=200, variable_a=True)
    patches = [(n_u - 1) * n_v + c for c in (0, 5, 9)]      # three patches of the last row
    idx = np.concatenate([np.arange(P * q * q, (P + 1) * q * q) for P in patches])
    s = p.surface
    lhs, tq, xe = conormal_derivative_at_edge(K_fn(p, idx), s.xu[idx], s.xv[idx], s.x[idx], q, patches, n_v)
    Kp = Kp_fn(p)[200:400]                     # the upper circle's samples
    rhs = -np.exp(xe[:, 0]) / (2 * np.exp(0.3 * xe[:, 0] * xe[:, 1])) + trig_eval(Kp, tq)
    return float(np.abs(lhs - rhs).max() / np.abs(rhs).max())


def test_neumann_jump_relation():
    def K_fn(p, idx):
        return edge_apply("K", targets_of(OracleOperator.from_problem(p)), p.meta["edge"], p.meta["edge"].mu, 64,
                          targets=idx)[:, 0]

    def Kp_fn(p):
        return kprime_gamma(p.meta["edge"], p.meta["edge"].mu)[:, 0]
    lo, hi = _jump_error(12, K_fn, Kp_fn), _jump_error(16, K_fn, Kp_fn)
    assert hi < 1e-8 and hi < lo / 100, (lo, hi)


def test_dirichlet_jump_relation():
    from _surface_ops import trig_eval, values_at_edge
    errs = []
    for q in (12, 16):
        n_u, n_v = 8, 12
        p = wavy_torus_piece_problem(n_u=n_u, n_v=n_v, q=q, n_edge=200, variable_a=False)
        e = p.meta["edge"]
        patches = [(n_u - 1) * n_v + c for c in (0, 5, 9)]  # three patches of the last row
        idx = np.concatenate([np.arange(P * q * q, (P + 1) * q * q) for P in patches])
        Nv = edge_apply("N", targets_of(OracleOperator.from_problem(p)), e, e.mu, 64, targets=idx)[:, 0]
        lhs, tq = values_at_edge(Nv, q, patches, n_v)
        up, lo = slice(200, 400), slice(0, 200)
        D_all = dlayer_gamma(e, e.mu)[up, 0]          # both circles' double layer at the upper samples
        rhs = trig_eval(e.mu[up, 0] / (2 * e.a[up]) + D_all, tq)
        errs.append(float(np.abs(lhs - rhs).max() / np.abs(rhs).max()))
    assert errs[1] < 1e-10 and errs[1] < errs[0] / 100, errs



def test_dlayer_circle_and_quadrature():
    """D_gamma[1] = 1/2 on a circle (a = 1: the kernel is the constant 1 / (4 pi rho)); on an ellipse the
    trapezoid sums equal adaptive quadrature of the exact integrand; a varying along the curve is refused."""
    for rho, n in ((0.7, 12), (2.0, 33)):
        e = _planar_edge(n, rho, rho)
        np.testing.assert_allclose(dlayer_gamma(e, np.ones(n))[:, 0], 0.5, atol=1e-14)
    n = 96
    e = _planar_edge(n)
    v = dlayer_gamma(e, np.exp(e.x[:, 0]))[:, 0]
    for j in (0, 17, 50):
        t0 = 2 * np.pi * j / n
        x = e.x[j]

        def g(t):
            y, yt, _ = _ellipse(t)
            nuy = conormal(yt[None], np.array([[np.cos(t), np.sin(t), 0.0]]))[0]
            r = y - x
            return float(nuy @ r / (2 * np.pi * (r @ r))) * np.linalg.norm(yt) * np.exp(y[0])
        ref = si.quad(g, t0, t0 + 2 * np.pi, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
        assert abs(v[j] - ref) < 1e-12 * max(1.0, abs(ref)), (j, v[j], ref)
    p = wavy_torus_piece_problem(n_u=4, n_v=6, q=6, n_edge=40, variable_a=True)
    with pytest.raises(ValueError):
        dlayer_gamma(p.meta["edge"], p.meta["edge"].mu)
