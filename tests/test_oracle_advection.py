"""Pins of the oracle's advection term (eq:adv_remainder, eq:IE_adv) against facts fixed by the
paper and by mathematics.

* eq:adv_remainder with eq:diff_remainder: for x != x', R_b(x, x') equals the surface operator
  div_G(a grad_G .) + b . grad_G + c(x) applied in x to K(x, x') = G(|x - x'|; a(x'), c(x')),
  with K differentiated numerically at 40 digits (mpmath), independently of the explicit formula.
* Section 7.1 with a rotation: on the unit sphere with a = 1, c = c0 and b = omega e3 x x,
  b . grad_G acts as omega d/dphi, which maps the harmonic pair (Y_l^m cos, Y_l^m sin) into itself;
  f = Y_l^m cos then has the closed-form solution alpha Y_l^m cos + beta Y_l^m sin with
  alpha = (lam + c0) / ((lam + c0)^2 + (m omega)^2), beta = m omega / ((lam + c0)^2 + (m omega)^2)
  and lam = -l(l+1) (tests/golden/sphere_lb_eigenvalues.txt).
* Method of manufactured solutions (Section 7.2) with Section 7.4's kind of variable coefficients
  and a non-tangent ambient field b (its tangential part acts): the error falls under refinement.
* Only the tangential part of b enters: adding a normal component changes no block.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest
import torch

from paper_2401_12501_amd.inputs import helmholtz_sphere_problem, real_sph_harm_cartesian
from oracle.kernels import remainder
from oracle.operator import OracleOperator
from oracle.system import blocks_parallel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rand_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_advection_remainder_equals_operator_of_parametrix():
    mp.mp.dps = 40
    rng = np.random.default_rng(31)
    for _ in range(4):
        x0, y = rng.normal(size=3), rng.normal(size=3)
        n = _rand_unit(rng)
        gs = rng.normal(size=3)
        gs -= n * (n @ gs)
        b = rng.normal(size=3)
        b -= n * (n @ b)
        a_t, H, c_t = 0.9, -0.3, -1.7
        a_s, c_s = 1.4, -3.2
        kap = mp.sqrt(mp.mpf(-c_s) / a_s)

        def K(*z):
            r = mp.sqrt(sum((mp.mpf(z[k]) - y[k]) ** 2 for k in range(3)))
            return -mp.besselk(0, kap * r) / (2 * mp.pi * a_s)

        xs = [mp.mpf(v) for v in x0]
        grad = np.array([float(mp.diff(K, xs, tuple(1 if k == j else 0 for k in range(3)))) for j in range(3)])
        hess = np.array([[float(mp.diff(K, xs, tuple((k == i) + (k == j) for k in range(3)))) for j in range(3)]
                         for i in range(3)])
        ref = gs @ grad - 2 * a_t * H * (n @ grad) + a_t * (np.trace(hess) - n @ hess @ n) + c_t * float(K(*xs)) \
            + b @ grad
        val = remainder(x0, n, H, a_t, gs, y, a_s, c_t, c_s, b)
        assert abs(val - ref) <= 1e-12 * max(1.0, abs(ref)), (val, ref)
        # the advection part alone is b . grad K
        d = val - remainder(x0, n, H, a_t, gs, y, a_s, c_t, c_s)
        assert abs(d - b @ grad) <= 1e-12 * max(1.0, abs(b @ grad))


def _golden(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return {int(r[0]): float(r[1]) for r in rows}


def rotation_solution(l, m, omega, c0, X):
    """Closed form of div_G grad_G u + omega du/dphi + c0 u = Y_l^m cos on the unit sphere."""
    lam = -l * (l + 1)
    Uc = real_sph_harm_cartesian(l, m, X).numpy()
    Us = real_sph_harm_cartesian(l, -m, X).numpy()
    d = (lam + c0) ** 2 + (m * omega) ** 2
    return Uc, ((lam + c0) / d) * Uc + (m * omega / d) * Us


def test_sphere_rotation_closed_form():
    """a = 1, c = -4, b = 1.5 e3 x x on the unit sphere (24 patches, q = 8)."""
    omega, c0 = 1.5, -4.0
    lams = _golden("sphere_lb_eigenvalues.txt")
    p = helmholtz_sphere_problem(k=2, q=8, c0=c0, omega=omega)
    op = OracleOperator.from_problem(p)
    B = blocks_parallel(("paper_2401_12501_amd.inputs", "helmholtz_sphere_problem",
                         {"k": 2, "q": 8, "c0": c0, "omega": omega}), ROOT, np.arange(op.N), kernels=("R", "K"),
                        workers=min(8, os.cpu_count() or 1))
    A = op.dense_matrix(B)
    X = torch.tensor(p.surface.x)
    for l, m in ((1, 1), (2, 1), (3, 2), (4, 3), (2, 0)):
        assert lams[l] == -l * (l + 1)
        f, ref = rotation_solution(l, m, omega, c0, X)
        u = op.represent(op.solve(f[:, None], A), B)[:, 0]
        err = np.abs(u - ref).max() / np.abs(ref).max()
        assert err < 1e-6, (l, m, err)


def test_manufactured_with_advection_converges():
    """a = 2 + z, c = -4 - exp(x/2) and b = fields.b_swirl (not tangent: its tangential part acts)
    with u = (x^2 - y^2) z on the unit sphere: the error of u falls by more than 2^4 when the patch
    size halves."""
    errs = []
    for k in (1, 2):
        p = helmholtz_sphere_problem(k=k, q=6, swirl=True)
        op = OracleOperator.from_problem(p)
        B = blocks_parallel(("paper_2401_12501_amd.inputs", "helmholtz_sphere_problem",
                             {"k": k, "q": 6, "swirl": True}), ROOT, np.arange(op.N), kernels=("R", "K"),
                            workers=min(8, os.cpu_count() or 1))
        sig = op.solve(p.f, op.dense_matrix(B))
        u = op.represent(sig, B)[:, 0]
        ue = p.meta["u_exact"]
        errs.append(math.sqrt(op.w @ (u - ue) ** 2 / (op.w @ ue ** 2)))
    assert errs[1] < errs[0] / 16 and errs[1] < 1e-5, errs


def test_only_the_tangential_part_of_b_acts():
    p = helmholtz_sphere_problem(k=1, q=5, swirl=True)
    s = p.surface
    ops = [OracleOperator(s.q, s.x, s.xu, s.xv, s.xuu, s.xuv, s.xvv, p.a, p.grad_a, c=p.c, b=b)
           for b in (p.b, p.b + 2.5 * s.x / np.linalg.norm(s.x, axis=1)[:, None])]
    tg = np.arange(0, p.n, 7)
    B0, B1 = (op.blocks(tg) for op in ops)
    for (_, b0), (_, b1) in zip(B0, B1):
        np.testing.assert_allclose(b1["R"], b0["R"], rtol=0, atol=1e-12 * np.abs(b0["R"]).max())
    sig = np.random.default_rng(5).normal(size=(p.n, 1))
    np.testing.assert_allclose(ops[1].far_rows(tg, sig), ops[0].far_rows(tg, sig), rtol=1e-12, atol=1e-12)
    with pytest.raises(ValueError):
        OracleOperator(s.q, s.x, s.xu, s.xv, s.xuu, s.xuv, s.xvv, p.a, p.grad_a, b=p.b)   # c = 0 with b
