"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Cases: the unit-sphere workload (24 patches, q = 8, 1,536 nodes, variable a and
a = 1), a small ellipsoid whose node count is not a multiple of any launch tile
(6 patches, q = 7, 294 nodes), and the full ellipsoid workload (1,536 patches,
q = 10, 153,600 nodes) on sampled rows.  Bars, element by element (max-abs error over max-abs
value, per right-hand side): FP64 path within 1e-12, index work bit-exact, FP32 far field within
1e-5.
"""
import math
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import sphere_problem, ellipsoid_problem, random_density
from oracle.operator import OracleOperator

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def max_rel(a, b):
    """Largest column-wise max |a - b| / max |b| of (N, n_rhs) arrays."""
    a = np.asarray(a).reshape(np.shape(b)[0], -1)
    b = np.asarray(b).reshape(np.shape(b)[0], -1)
    return max(float(np.abs(a[:, r] - b[:, r]).max() / np.abs(b[:, r]).max()) for r in range(b.shape[1]))


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_12501_amd import pmx
    import torch
    assert torch.cuda.is_available()
    return pmx.Context(0)


class Case:
    def __init__(self, prob, ctx, kernels=("R",), full=True):
        from paper_2401_12501_amd import pmx
        self.prob = prob
        say(f"[case] {prob.name}: N={prob.n}")
        self.surf = pmx.Surface.from_inputs(ctx, prob.surface)
        self.op = pmx.Operator(self.surf, prob.a, prob.grad_a)
        self.orc = OracleOperator.from_problem(prob)
        self.blocks = self.orc.blocks(np.arange(prob.n), kernels=kernels) if full else None
        self.A = self.orc.dense_matrix(self.blocks) if full else None


@pytest.fixture(scope="module")
def sphere(ctx):
    return Case(sphere_problem(k=2, q=8), ctx)


@pytest.fixture(scope="module")
def ragged(ctx):
    return Case(ellipsoid_problem(k=1, q=7), ctx, kernels=("R", "K"))


def test_geometry_parity(ragged):
    g = ragged.op.export_geometry()
    o = ragged.orc
    np.testing.assert_allclose(g["n"], o.n, rtol=0, atol=1e-14)
    np.testing.assert_allclose(g["H"], o.H, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(g["w"], o.w, rtol=1e-13, atol=0)   # independent Gauss-Legendre generators
    np.testing.assert_allclose(g["gs"], o.gs, rtol=0, atol=1e-14)


@pytest.mark.parametrize("which", ["ragged", "sphere"])
def test_near_lists_and_blocks(which, request):
    case = request.getfixturevalue(which)
    ptr, patch, Cb, _ = case.op.export_near()
    N = case.prob.n
    scale = 0.0
    worst = 0.0
    for i in range(N):
        plist, blk = case.blocks[i]
        got = patch[ptr[i]:ptr[i + 1]]
        assert np.array_equal(got, plist), f"near list of target {i}"
        scale = max(scale, np.abs(blk["R"]).max())
        worst = max(worst, np.abs(Cb[ptr[i]:ptr[i + 1]] - blk["R"]).max())
    say(f"[blocks] {which}: max |C_gpu - C_oracle| = {worst:.3e} (max |C| = {scale:.3e})")
    assert worst <= 1e-13 * scale


def test_parametrix_blocks(ragged):
    ptr, patch, _, Db = ragged.op.export_near(with_D=True)
    worst = scale = 0.0
    for i in range(ragged.prob.n):
        blk = ragged.blocks[i][1]["K"]
        scale = max(scale, np.abs(blk).max())
        worst = max(worst, np.abs(Db[ptr[i]:ptr[i + 1]] - blk).max())
    say(f"[blocks K] max diff {worst:.3e} scale {scale:.3e}")
    assert worst <= 1e-13 * scale


def ulp_sensitivity(orc, i, plist, kernels, base):
    """max |C(x_i + du t) - C(x_i)| over one-ulp moves du of target i's kernel argument along its
    tangents and normal t; the patch nodes that the rules interpolate stay where they are.

    With normals taken from the given derivatives, n_i . r is O(eps rho + rho^2) on the
    interpolated patch (eps: angle between n_i and the interpolant's tangent plane), so
    (n.r)^2 / r^4 carries an eps^2 / rho^2 part and the rounding of r = x_i - y(u, v) near the
    target is amplified by about eps^2 / rho_min.  An interpolated source point y is exact only to
    a few ulps, which is what the move models; on under-resolved surfaces (one patch per cube
    face) this bounds how closely two correct FP64 evaluations of the self blocks agree."""
    x_saved = orc.x
    du = np.spacing(np.abs(x_saved[i]).max())
    out = {k: 0.0 for k in kernels}
    try:
        for t in (orc.xu[i], orc.xv[i], orc.n[i]):
            orc.x = x_saved.copy()          # patch node arrays keep viewing x_saved
            orc.x[i] = x_saved[i] + du * t / np.linalg.norm(t)
            for P, *blk in zip(plist, *(base[k] for k in kernels)):
                moved = orc.correction_blocks(int(i), int(P), kernels)
                for k, b in zip(kernels, blk):
                    out[k] = max(out[k], np.abs(moved[k] - b).max())
    finally:
        orc.x = x_saved
    return out


@pytest.mark.parametrize("q,n_gl", [(3, 16), (5, 16), (12, 16), (16, 16), (8, 8), (6, 11)])
def test_blocks_patch_orders_and_rules(ctx, q, n_gl):
    """The local-rule kernels are specialised per patch order q and take any n_gl <= 16:
    correction blocks C (and D for some) on sampled targets match the oracle's, each target within
    1e-13 of max |C| plus 16 times the oracle's own change under a one-ulp move of the target."""
    from paper_2401_12501_amd import pmx
    prob = ellipsoid_problem(k=1, q=q)
    o = pmx.pmx_default_options()
    o.n_gl = n_gl
    surf = pmx.Surface.from_inputs(ctx, prob.surface)
    op = pmx.Operator(surf, prob.a, prob.grad_a, o)
    with_D = q in (5, 16)
    ptr, patch, Cb, Db = op.export_near(with_D=with_D)
    orc = OracleOperator.from_problem(prob, n_gl=n_gl)
    rng = np.random.default_rng(q * 100 + n_gl)
    tg = np.unique(np.concatenate([[0, prob.n - 1], rng.choice(prob.n, 30, replace=False)]))
    kernels = ("R", "K") if with_D else ("R",)
    rows = []
    for i, (plist, blk) in zip(tg, orc.blocks(tg, kernels=kernels)):
        assert np.array_equal(patch[ptr[i]:ptr[i + 1]], plist)
        sens = ulp_sensitivity(orc, i, plist, kernels, blk)
        for k, got in (("R", Cb), ("K", Db)):
            if k in kernels:
                rows.append((k, i, np.abs(got[ptr[i]:ptr[i + 1]] - blk[k]).max(), np.abs(blk[k]).max(),
                             sens[k]))
    scale = {k: max(r[3] for r in rows if r[0] == k) for k in kernels}
    worst = {k: max(r[2] for r in rows if r[0] == k) for k in kernels}
    say(f"[blocks] q={q} n_gl={n_gl}: " + ", ".join(
        f"{k} {worst[k] / scale[k]:.2e} (max 1-ulp sensitivity "
        f"{max(r[4] for r in rows if r[0] == k) / scale[k]:.2e})" for k in kernels))
    for k, i, err, _, sens in rows:
        assert err <= 1e-13 * scale[k] + 16.0 * sens, f"kernel {k} target {i}: {err:.3e} (1-ulp {sens:.3e})"


@pytest.mark.parametrize("which", ["ragged", "sphere"])
def test_apply_fp64(which, request):
    from paper_2401_12501_amd import pmx
    case = request.getfixturevalue(which)
    N = case.prob.n
    sig = random_density(N, 3, seed=11)                   # (N, 3)
    ref = case.A @ sig
    y = case.op.apply(np.ascontiguousarray(sig.T), pmx.PMX_PREC_FP64_DIRECT).T
    err = max_rel(y, ref)
    say(f"[apply64] {which}: rel err {err:.3e}")
    assert err <= 1e-12
    # one right-hand side at a time gives the same numbers
    y1 = case.op.apply(np.ascontiguousarray(sig[:, 1]), pmx.PMX_PREC_FP64_DIRECT)
    assert np.array_equal(y1.ravel(), y[:, 1])


def test_apply_many_rhs(ragged):
    """27 right-hand sides run as groups of 16, 8, 2 and 1 through the direct sums (FP64 and FP32):
    every column matches the oracle, and the FP64 columns equal single-column applies exactly."""
    from paper_2401_12501_amd import pmx
    case = ragged
    sig = random_density(case.prob.n, 27, seed=15)
    ref = case.A @ sig
    y = case.op.apply(np.ascontiguousarray(sig.T), pmx.PMX_PREC_FP64_DIRECT).T
    err = max_rel(y, ref)
    y32 = case.op.apply(np.ascontiguousarray(sig.T), pmx.PMX_PREC_FP32_DIRECT).T
    err32 = max_rel(y32, ref)
    say(f"[apply64] 27 rhs: max rel err {err:.3e}; FP32 direct {err32:.3e}")
    assert err <= 1e-12 and err32 <= 1e-5
    for r in (3, 20, 26):
        y1 = case.op.apply(np.ascontiguousarray(sig[:, r]), pmx.PMX_PREC_FP64_DIRECT)
        assert np.array_equal(y1.ravel(), y[:, r])


@pytest.mark.parametrize("which", ["ragged", "sphere"])
def test_apply_fp32_direct(which, request):
    from paper_2401_12501_amd import pmx
    case = request.getfixturevalue(which)
    sig = random_density(case.prob.n, 1, seed=12)
    ref = case.A @ sig
    y = case.op.apply(np.ascontiguousarray(sig.T), pmx.PMX_PREC_FP32_DIRECT).T
    err = max_rel(y, ref)
    say(f"[apply32] {which}: rel err {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("which", ["ragged", "sphere"])
def test_solve_fp64(which, request):
    from paper_2401_12501_amd import pmx
    case = request.getfixturevalue(which)
    f = case.prob.f
    ref = case.orc.solve(f, case.A)
    o = pmx.pmx_default_options()
    o.gmres_tol = 1e-14
    sig, _, info = case.op.solve(np.ascontiguousarray(f.T), o)
    err = max_rel(sig.T, ref)
    say(f"[solve64] {which}: rel err {err:.3e}, iters {info[0].iters_total}, res {info[0].rel_residual:.2e}")
    assert err <= 1e-12
    _, mean = case.orc.project_mean_zero(f)
    assert abs(info[0].removed_mean - mean[0]) <= 1e-13 * max(1.0, abs(mean[0]))


def test_represent(ragged):
    sig = random_density(ragged.prob.n, 2, seed=13)
    ref = ragged.orc.represent(sig, ragged.blocks)
    u = ragged.op.represent(np.ascontiguousarray(sig.T)).T
    err = max_rel(u, ref)
    say(f"[represent] rel err {err:.3e}")
    assert err <= 1e-12


def test_sphere_eigenvalue(ctx):
    """a = 1 on the unit sphere: u = (x^2 - y^2) z solves Delta u = -12 u; the solve
    returns the mean-zero u and <f, u>_w / <u, u>_w = -12."""
    from paper_2401_12501_amd import pmx
    p = sphere_problem(k=2, q=8, const_a=True)
    surf = pmx.Surface.from_inputs(ctx, p.surface)
    op = pmx.Operator(surf, p.a, p.grad_a)
    sig, u, info = op.solve(np.ascontiguousarray(p.f.T), want_u=True)
    w = op.export_geometry()["w"]
    lam = float((w * p.f[:, 0] * u[0]).sum() / (w * u[0] * u[0]).sum())
    ue = p.meta["u_exact"]
    err = math.sqrt(float(w @ (u[0] - ue) ** 2) / float(w @ ue ** 2))
    say(f"[eigen] lambda {lam:.12f}, u err {err:.2e}, iters {info[0].iters_total}")
    assert abs(lam + 12) < 1e-6 and err < 1e-7
    assert info[0].iters_total <= 3
