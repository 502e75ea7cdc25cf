"""The c > 0 path (div_G(a grad_G u) + b . grad_G u + c u = f, the Helmholtz-Beltrami type of
Section 7.3, with the complex kernel G = -(i / 4a) H0(k r)) through the C ABI against the FP64
oracle, element by element (max-abs error over max-abs value, complex).

Cases: an ellipsoid with 6 patches of 7 x 7 nodes (294 nodes, not a multiple of any launch tile)
and the unit sphere (24 patches, q = 8), both with a = 2 + z and c = 2 (1 + 0.2 y), the ellipsoid
also with a non-tangent advection field (eq:adv_remainder).  Bars: the real and imaginary parts of
the correction blocks C and D within 1e-13 of the largest entry (plus 16x the oracle's one-ulp
sensitivity where the rules sample close to the target); FP64 applies over 1, 2 and 8 complex
densities at once, solves and the representation within 1e-12; with c scaled by 50 the blocks and
applies take both ranges of the device Bessel functions; Section 7.3's c = 4 with a = 1 on the
sphere gives the eigenvalues -l(l+1) + 4 within the discretization error.
"""
import os
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import (helmholtz_ellipsoid_problem, helmholtz_sphere_problem, random_density,
                                         real_sph_harm_cartesian)
from oracle.operator import OracleOperator
from oracle.system import blocks_parallel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def max_rel(a, b):
    a = np.asarray(a).reshape(np.shape(b)[0], -1)
    b = np.asarray(b).reshape(np.shape(b)[0], -1)
    return max(float(np.abs(a[:, r] - b[:, r]).max() / np.abs(b[:, r]).max()) for r in range(b.shape[1]))


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_12501_amd import pmx
    return pmx.Context(0)


class Case:
    def __init__(self, factory, kw, ctx):
        from paper_2401_12501_amd import pmx
        prob = factory(**kw)
        self.prob = prob
        say(f"[case] {prob.name}: N={prob.n}, c in [{prob.c.min():.3f}, {prob.c.max():.3f}]")
        self.surf = pmx.Surface.from_inputs(ctx, prob.surface)
        self.op = pmx.Operator(self.surf, prob.a, prob.grad_a, c=prob.c, b=prob.b)
        assert self.op.complex
        self.orc = OracleOperator.from_problem(prob)
        self.blocks = blocks_parallel(("paper_2401_12501_amd.inputs", factory.__name__, kw), ROOT,
                                      np.arange(prob.n), kernels=("R", "K"), workers=min(8, os.cpu_count() or 1))
        self.A = self.orc.dense_matrix(self.blocks)
        say(f"[case] {prob.name}: oracle blocks and matrix ready")


@pytest.fixture(scope="module")
def ragged(ctx):
    return Case(helmholtz_ellipsoid_problem, {"k": 1, "q": 7, "positive": True}, ctx)


@pytest.fixture(scope="module")
def sphere(ctx):
    return Case(helmholtz_sphere_problem, {"k": 2, "q": 8, "positive": True}, ctx)


@pytest.fixture(scope="module")
def ragged_b(ctx):
    return Case(helmholtz_ellipsoid_problem, {"k": 1, "q": 7, "positive": True, "swirl": True}, ctx)


@pytest.fixture(scope="module")
def ragged_hi(ctx):
    """c multiplied by 50 (k = sqrt(c/a) from 6.0 to 8.6): k r runs to about 15 (half the pairs above 8),
    so the Bessel functions take both of their ranges, also within one pair of sources."""
    return Case(helmholtz_ellipsoid_problem, {"k": 1, "q": 7, "positive": True, "c_scale": 50.0}, ctx)


CASES = ["ragged", "sphere", "ragged_b"]


@pytest.mark.parametrize("which", CASES + ["ragged_hi"])
def test_blocks_cpos(which, request):
    """Real and imaginary parts of the correction blocks C (remainder) and D (parametrix) against the
    oracle's complex blocks: 1e-13 of the largest entry, plus 16x the oracle's own change under
    one-ulp moves of the target for the targets above that (as for c < 0)."""
    from test_gpu_parity import ulp_sensitivity
    case = request.getfixturevalue(which)
    ptr, patch, Cr, Dr = case.op.export_near(with_D=True)
    Ci, Di = case.op.export_near_imag(with_D=True)
    G = {"R": Cr + 1j * Ci, "K": Dr + 1j * Di}
    err = {"R": np.zeros(case.prob.n), "K": np.zeros(case.prob.n)}
    scale = {"R": 0.0, "K": 0.0}
    for i in range(case.prob.n):
        plist, blk = case.blocks[i]
        assert np.array_equal(patch[ptr[i]:ptr[i + 1]], plist)
        for k in ("R", "K"):
            scale[k] = max(scale[k], np.abs(blk[k]).max())
            err[k][i] = np.abs(G[k][ptr[i]:ptr[i + 1]] - blk[k]).max()
    imag_part = max(np.abs(case.blocks[i][1]["R"].imag).max() for i in range(case.prob.n))
    say(f"[blocks c>0] {which}: C {err['R'].max() / scale['R']:.2e}, D {err['K'].max() / scale['K']:.2e} of max "
        f"(largest imaginary part of C {imag_part:.2e})")
    assert imag_part > 1e-6 * scale["R"]      # the imaginary parts are really there
    for k in ("R", "K"):
        over = np.nonzero(err[k] > 1e-13 * scale[k])[0]
        for i in over:
            plist, blk = case.blocks[i]
            sens = ulp_sensitivity(case.orc, int(i), plist, (k,), {k: blk[k]})[k]
            assert err[k][i] <= 1e-13 * scale[k] + 16.0 * sens, (k, i, err[k][i], sens)
        say(f"[blocks c>0] {which} {k}: {len(over)} targets above 1e-13 of max, all within 16x their 1-ulp "
            f"sensitivity")


@pytest.mark.parametrize("which", CASES)
def test_apply_solve_represent_cpos(which, request):
    from paper_2401_12501_amd import pmx
    case = request.getfixturevalue(which)
    N = case.prob.n
    # 11 complex densities: the direct sum's groups of 8, 2 and 1
    sig = random_density(N, 11, seed=91) + 1j * random_density(N, 11, seed=92)
    y = case.op.apply(np.ascontiguousarray(sig.T), pmx.PMX_PREC_FP64_DIRECT).T
    e_apply = max_rel(y, case.A @ sig)
    y1 = case.op.apply(np.ascontiguousarray(sig[:, 3:4].T), pmx.PMX_PREC_FP64_DIRECT).T
    e_one = max_rel(y1, case.A @ sig[:, 3:4])
    o = pmx.pmx_default_options()
    o.gmres_tol = 1e-14
    s, u, info = case.op.solve(np.ascontiguousarray(case.prob.f.T), o, want_u=True)
    s_ref = case.orc.solve(case.prob.f, case.A)
    u_ref = case.orc.represent(s_ref, case.blocks)
    e_s, e_u = max_rel(s.T, s_ref), max_rel(u.T, u_ref)
    say(f"[c>0 path] {which}: apply {e_apply:.2e} (one density {e_one:.2e}), sigma {e_s:.2e}, u {e_u:.2e}, "
        f"iters {info[0].iters_total}, residual {info[0].rel_residual:.1e}")
    assert np.abs(s.imag).max() > 1e-6 * np.abs(s).max()
    assert e_apply <= 1e-12 and e_one <= 1e-12 and e_s <= 1e-12 and e_u <= 1e-12
    assert info[0].removed_mean == 0.0
    if "u_exact" in case.prob.meta:   # manufactured solution: the discretization error, and u is real
        ue = case.prob.meta["u_exact"]
        err = float(np.abs(u[0] - ue).max() / np.abs(ue).max())
        say(f"[c>0 path] {which}: manufactured u error {err:.2e}, max |Im u| {np.abs(u[0].imag).max():.2e}")
        assert err < 1e-5


def test_apply_cpos_both_bessel_ranges(ragged_hi):
    """Applies over 1, 2 and 8 complex densities with k r up to about 15 (both ranges of the device
    Bessel functions, and pairs of sources that straddle z = 8) against the oracle's dense matrix."""
    from paper_2401_12501_amd import pmx
    case = ragged_hi
    x = case.prob.surface.x
    kap = np.sqrt(case.prob.c / case.prob.a)
    z = kap[None, :] * np.linalg.norm(x[:, None, :] - x[None, :, :], axis=2)
    frac_large = float(np.mean(z > 8.0))
    sig = random_density(case.prob.n, 11, seed=93) + 1j * random_density(case.prob.n, 11, seed=94)
    y = case.op.apply(np.ascontiguousarray(sig.T), pmx.PMX_PREC_FP64_DIRECT).T
    e = max_rel(y, case.A @ sig)
    say(f"[c>0 hi] apply {e:.2e}, pairs with k r > 8: {frac_large:.2f}")
    assert 0.1 < frac_large < 0.9
    assert e <= 1e-12


def test_sphere_eigenvalues_cpos_gpu(ctx):
    """Section 7.3's c = 4 with a = 1 on the unit sphere (24 patches, q = 8): f = Y_lm gives
    u = f / (-l(l+1) + 4), real, on the GPU."""
    import torch
    from paper_2401_12501_amd import pmx
    p = helmholtz_sphere_problem(k=2, q=8, c0=4.0)
    surf = pmx.Surface.from_inputs(ctx, p.surface)
    op = pmx.Operator(surf, p.a, p.grad_a, c=p.c)
    X = torch.tensor(p.surface.x)
    worst = 0.0
    for l in (0, 1, 2, 3, 4):
        f = real_sph_harm_cartesian(l, min(l, 1), X).numpy()
        _, u, info = op.solve(f[None, :].copy(), want_u=True)
        ref = f / (-l * (l + 1) + 4.0)
        e = float(np.abs(u[0] - ref).max() / np.abs(ref).max())
        worst = max(worst, e)
        say(f"[c>0 eigen] l={l}: u error {e:.2e}, iters {info[0].iters_total}")
    assert worst < 1e-4


def test_cpos_device_arrays_and_contract(ctx):
    """Device tensors in and out (complex torch tensors, planar on the library side); the one-sign rule
    for c; the low-precision paths refuse a complex operator; a real operator has no imaginary
    blocks."""
    import torch
    from paper_2401_12501_amd import pmx
    p = helmholtz_ellipsoid_problem(k=1, q=5, positive=True)
    surf = pmx.Surface.from_inputs(ctx, p.surface)
    op = pmx.Operator(surf, p.a, p.grad_a, c=p.c)
    sig = random_density(p.n, 2, seed=5).T + 1j * random_density(p.n, 2, seed=6).T
    y_host = op.apply(np.ascontiguousarray(sig))
    y_dev = op.apply(torch.tensor(sig, device="cuda:0"))
    assert y_dev.is_cuda and y_dev.is_complex()
    assert np.array_equal(y_dev.cpu().numpy(), y_host)
    for prec in (pmx.PMX_PREC_MIXED_FMM, pmx.PMX_PREC_FP32_DIRECT):
        with pytest.raises(pmx.PmxError) as e:
            op.apply(sig, prec)
        assert e.value.code == pmx.PMX_ERR_INVALID
    mixed = np.where(np.arange(p.n) == 17, -p.c, p.c)
    with pytest.raises(pmx.PmxError) as e:
        pmx.Operator(surf, p.a, p.grad_a, c=mixed)
    assert e.value.code == pmx.PMX_ERR_INVALID
    real_op = pmx.Operator(surf, p.a, p.grad_a, c=-p.c)
    assert not real_op.complex
    with pytest.raises(pmx.PmxError) as e:
        real_op.export_near_imag()
    assert e.value.code == pmx.PMX_ERR_INVALID


def test_cpos_largest_call(ragged):
    """1,024 complex densities in one apply (the largest n_rhs; 2,048 real columns through the complex
    direct sum's groups of 8): sampled columns equal their single-density applies bit for bit (each
    column's arithmetic and order do not depend on the group) and match the oracle's matrix."""
    import torch
    from paper_2401_12501_amd import pmx
    case = ragged
    N = case.prob.n
    rng = np.random.default_rng(95)
    sig = rng.normal(size=(1024, N)) + 1j * rng.normal(size=(1024, N))
    y = case.op.apply(torch.tensor(sig, device="cuda:0")).cpu().numpy()
    assert y.shape == (1024, N) and np.all(np.isfinite(y))
    for r in (0, 7, 8, 513, 1023):
        y1 = case.op.apply(torch.tensor(sig[r:r + 1], device="cuda:0")).cpu().numpy()
        assert np.array_equal(y1[0], y[r]), r
    ref = (case.A @ sig[[0, 1023]].T).T
    e = max(float(np.abs(y[[0, 1023]][k] - ref[k]).max() / np.abs(ref[k]).max()) for k in range(2))
    say(f"[c>0 1024] sampled columns vs oracle {e:.2e}")
    assert e <= 1e-12


def test_cpos_multi_rhs_solve_and_warm_start(ragged):
    """Three right-hand sides solved together (complex GMRES in lockstep): a
    real one and two complex ones, each column against the oracle's dense solve and against its own
    single-column solve; then a warm start from the solution, which returns it after at most one
    iteration (tolerance 1e-12 there)."""
    from paper_2401_12501_amd import pmx
    case = ragged
    N = case.prob.n
    rng = np.random.default_rng(96)
    F = np.stack([case.prob.f[:, 0], rng.normal(size=N) + 1j * rng.normal(size=N),
                  1j * case.prob.f[:, 0] + rng.normal(size=N)], axis=0)
    o = pmx.pmx_default_options()
    o.gmres_tol = 1e-14
    s, u, info = case.op.solve(F.copy(), o, want_u=True)
    ref = np.linalg.solve(case.A, F.T).T
    u_ref = case.orc.represent(ref.T, case.blocks).T
    errs = [float(np.abs(s[k] - ref[k]).max() / np.abs(ref[k]).max()) for k in range(3)]
    errs_u = [float(np.abs(u[k] - u_ref[k]).max() / np.abs(u_ref[k]).max()) for k in range(3)]
    say(f"[c>0 3 rhs] sigma {max(errs):.2e}, u {max(errs_u):.2e}, iters {[i.iters_total for i in info]}")
    assert max(errs) <= 1e-12 and max(errs_u) <= 1e-12
    s1, _, _ = case.op.solve(F[1:2].copy(), o)
    assert np.abs(s1[0] - s[1]).max() <= 1e-13 * np.abs(s[1]).max()
    o2 = pmx.pmx_default_options()
    o2.gmres_tol = 1e-12   # the solution's residual (about 1e-14) is below this: no iteration is needed
    s2, _, info2 = case.op.solve(F.copy(), o2, sigma0=s)
    assert all(i.iters_total <= 1 for i in info2), [i.iters_total for i in info2]
    assert np.abs(s2 - s).max() <= 1e-13 * np.abs(s).max()
