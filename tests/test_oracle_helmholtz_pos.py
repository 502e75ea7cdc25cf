"""Pins of the oracle's c > 0 path (the Helmholtz type, Section 7.3) against facts fixed by the
paper and by mathematics.  The kernel is complex here: G = -(i / 4a) H0(k r), k = sqrt(c / a).

* eq:diff_remainder: R(x, x') = grad_G a . grad K - 2 a H d_n K + a (Delta K - d_n^2 K) + c(x) K
  for x != x', with K(x) = G(|x - x'|; a(x'), c(x')) differentiated numerically at 40 digits
  (mpmath's own Hankel function), independently of the explicit formula eq:explicit_remainder.
* The constant-coefficient corollary eq:bdd_remainder_helm as printed, with the real wavenumber
  k = sqrt(c0 / a0): a different formula of the paper (H1, H2 from the library).
* The log part of G: G - log(r) / (2 pi a) tends to a constant as r -> 0 (the sign reading of the
  printed Hankel form, the same as for c < 0).
* Section 7.1 and Section 7.3: on the unit sphere with a = 1 and c = 4, the spherical harmonics
  solve the problem with the eigenvalues -l(l+1) + 4 (tests/golden/sphere_lb_eigenvalues.txt
  shifted by c); u = K[sigma] is real up to the discretization error although sigma is complex.
* Method of manufactured solutions with variable a and c > 0: the error falls under patch
  refinement, and so does the imaginary part of u.
* Scaling: a -> s a, c -> s c leaves k and R unchanged, so sigma is unchanged and u scales by 1/s.
"""
import math
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sp
import torch

from paper_2401_12501_amd.inputs import helmholtz_sphere_problem, real_sph_harm_cartesian
from oracle.kernels import green, remainder
from oracle.operator import OracleOperator
from oracle.system import blocks_parallel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rand_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def test_remainder_equals_surface_operator_of_parametrix_c_positive():
    mp.mp.dps = 40
    rng = np.random.default_rng(31)
    for _ in range(4):
        x0, y = rng.normal(size=3), rng.normal(size=3)
        n = _rand_unit(rng)
        gs = rng.normal(size=3)
        gs -= n * (n @ gs)
        a_t, H, c_t = 1.3, 0.45, 2.7
        a_s, c_s = 0.8, 4.1
        k = mp.sqrt(mp.mpf(c_s) / a_s)

        def K(*z):
            r = mp.sqrt(sum((mp.mpf(z[j]) - y[j]) ** 2 for j in range(3)))
            return -1j * mp.hankel1(0, k * r) / (4 * a_s)

        xs = [mp.mpf(v) for v in x0]
        grad = [mp.diff(K, xs, tuple(1 if j == i else 0 for j in range(3))) for i in range(3)]
        hess = [[mp.diff(K, xs, tuple((j == i) + (j == l) for j in range(3))) for l in range(3)] for i in range(3)]
        g = np.array([complex(v) for v in grad])
        Hs = np.array([[complex(v) for v in row] for row in hess])
        ref = gs @ g - 2 * a_t * H * (n @ g) + a_t * (np.trace(Hs) - n @ Hs @ n) + c_t * complex(K(*xs))
        val = remainder(x0, n, H, a_t, gs, y, a_s, c_t, c_s)
        assert abs(val - ref) <= 1e-12 * max(1.0, abs(ref)), (val, ref)


def test_constant_coefficient_helmholtz_form_real_wavenumber():
    """eq:bdd_remainder_helm as printed, for a = a0 and c = c0 > 0 (k = sqrt(c0 / a0) real):
    R = -(c0 / (4 i a0)) H2(k r) (n.r)^2 / r^2 + (sqrt(c0) / (2 i sqrt(a0))) H1(k r) H n.r / r."""
    rng = np.random.default_rng(32)
    for a0, c0 in ((1.0, 4.0), (2.5, 1.3), (0.6, 9.0)):
        for _ in range(6):
            x, y = rng.normal(size=3), rng.normal(size=3)
            n = _rand_unit(rng)
            H = rng.normal()
            r = x - y
            rn = np.linalg.norm(r)
            k = math.sqrt(c0 / a0)
            ref = -(c0 / (4j * a0)) * sp.hankel1(2, k * rn) * (n @ r) ** 2 / rn ** 2 \
                + (math.sqrt(c0) / (2j * math.sqrt(a0))) * sp.hankel1(1, k * rn) * H * (n @ r) / rn
            val = remainder(x, n, H, a0, np.zeros(3), y, a0, c0, c0)
            assert abs(val - ref) <= 1e-12 * max(1.0, abs(ref)), (a0, c0, val, ref)


def test_log_part_of_g_c_positive():
    """Re G - log(r) / (2 pi a) and Im G tend to constants as r -> 0 (the constant from the small-z
    form of H0: (log(k / 2) + gamma) / (2 pi a) and -1 / (4a))."""
    for a, c in ((1.0, 4.0), (0.7, 2.2)):
        k = math.sqrt(c / a)
        lim = (math.log(k / 2) + np.euler_gamma) / (2 * math.pi * a) - 1j / (4 * a)
        for r in (1e-6, 1e-8):
            G = green(np.array([r]), a, np.array([c]))[0][0]
            d = G - math.log(r) / (2 * math.pi * a)
            assert abs(d - lim) < 1e-9, (a, c, r, d, lim)


def _golden(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return [(int(r[0]), float(r[1])) for r in rows]


def test_sphere_eigenvalues_shift_by_c_positive():
    """Section 7.3's c = 4 with a = 1 on the unit sphere (24 patches, q = 8): solving with f = Y_lm
    and representing gives u = f / (-l(l+1) + 4), real."""
    c0 = 4.0
    p = helmholtz_sphere_problem(k=2, q=8, c0=c0)
    op = OracleOperator.from_problem(p)
    assert op.complex
    B = blocks_parallel(("paper_2401_12501_amd.inputs", "helmholtz_sphere_problem", {"k": 2, "q": 8, "c0": c0}),
                        ROOT, np.arange(op.N), kernels=("R", "K"), workers=min(8, os.cpu_count() or 1))
    A = op.dense_matrix(B)
    assert A.dtype == np.complex128 and np.abs(A.imag).max() > 1e-3
    X = torch.tensor(p.surface.x)
    for l, lam in _golden("sphere_lb_eigenvalues.txt"):
        f = real_sph_harm_cartesian(l, min(l, 1), X).numpy()[:, None]
        sig = op.solve(f, A)
        u = op.represent(sig, B)
        ref = f / (lam + c0)
        assert np.abs(sig.imag).max() > 1e-6   # sigma itself is complex
        assert np.abs(u - ref).max() < 1e-4 * np.abs(ref).max(), (l, np.abs(u - ref).max() / np.abs(ref).max())


def test_manufactured_variable_coefficients_converge_c_positive():
    """a = 2 + z and c = 2 (1 + 0.2 y) with u = (x^2 - y^2) z on the unit sphere: the error of u
    falls by more than 2^4 when the patch size halves, and Im u falls with it."""
    errs, imag = [], []
    for k in (1, 2):
        p = helmholtz_sphere_problem(k=k, q=6, positive=True)
        op = OracleOperator.from_problem(p)
        B = blocks_parallel(("paper_2401_12501_amd.inputs", "helmholtz_sphere_problem",
                             {"k": k, "q": 6, "positive": True}), ROOT, np.arange(op.N), kernels=("R", "K"),
                            workers=min(8, os.cpu_count() or 1))
        sig = op.solve(p.f, op.dense_matrix(B))
        u = op.represent(sig, B)[:, 0]
        ue = p.meta["u_exact"]
        errs.append(math.sqrt(op.w @ np.abs(u - ue) ** 2 / (op.w @ ue ** 2)))
        imag.append(np.abs(u.imag).max() / np.abs(ue).max())
    assert errs[1] < errs[0] / 16 and errs[1] < 1e-5, errs
    assert imag[1] < imag[0] and imag[1] < 1e-5, imag


def test_coefficient_scaling_c_positive():
    p = helmholtz_sphere_problem(k=1, q=4, positive=True)
    s = p.surface
    ops = [OracleOperator(s.q, s.x, s.xu, s.xv, s.xuu, s.xuv, s.xvv, sc * p.a, sc * p.grad_a, c=sc * p.c)
           for sc in (1.0, 3.0)]
    sig = [op.solve(p.f) for op in ops]
    np.testing.assert_allclose(sig[1], sig[0], rtol=1e-10, atol=1e-12)
    u = [op.represent(sg) for op, sg in zip(ops, sig)]
    np.testing.assert_allclose(3.0 * u[1], u[0], rtol=1e-10, atol=1e-12)


def test_mixed_sign_c_is_rejected():
    p = helmholtz_sphere_problem(k=1, q=4, c0=2.0)
    s = p.surface
    c = p.c.copy()
    c[0] = -1.0
    with pytest.raises(ValueError):
        OracleOperator(s.q, s.x, s.xu, s.xv, s.xuu, s.xuv, s.xvv, p.a, p.grad_a, c=c)
