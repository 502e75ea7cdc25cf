"""Full-size workloads on sampled outputs: the ellipsoid (1,536 patches, q = 10, 153,600 nodes), the
star (8,214 patches, q = 8, 525,696 nodes; apply, mixed solve and representation) and the wobbly
torus (256 x 128 patches, q = 8, 2,097,152 nodes, 16 right-hand sides; applies and the joint mixed
solve).

The oracle evaluates rows of the operator (near blocks from worker processes, smooth-rule sums over
all sources in C on every host core) at 1,024 or more stratified targets: first and last nodes of
seeded patches, the targets with the most near patches, and seeded random nodes.  The GPU applies
the whole operator in the launch configuration the benchmark uses (library defaults).  Element-wise
bars (max-abs error / max-abs value over the sampled rows): FP64 path 1e-12; mixed path 1e-5 (the
FP32 interpolation FMM at p = 6, measured 2-4e-6; refinement removes it); solve residuals in the
oracle's discrete system 1e-8.
"""
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import ellipsoid_problem, star_problem, wobbly_torus_problem, random_density
from oracle.operator import OracleOperator

from _oracle_rows import apply_rows, stratified_targets

pytestmark = pytest.mark.gpu
N_ROWS = 1024


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def max_rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_12501_amd import pmx
    return pmx.Context(0)


def check_rows(ctx, prob, factory, n_rhs_64, n_rhs_mixed, seed):
    import torch
    from paper_2401_12501_amd import pmx
    say(f"[fullsize] {prob.name}: N={prob.n}")
    surf = pmx.Surface.from_inputs(ctx, prob.surface)
    op = pmx.Operator(surf, prob.a, prob.grad_a)
    st = op.stats()
    say(f"[fullsize] near pairs {st.near_pairs}, device MB {st.device_bytes / 2**20:.0f}")
    sig = random_density(prob.n, max(n_rhs_64, n_rhs_mixed), seed=seed)
    dev = torch.tensor(np.ascontiguousarray(sig.T), device="cuda:0")
    ym = op.apply(dev[:n_rhs_mixed].contiguous(), pmx.PMX_PREC_MIXED_FMM).cpu().numpy().T
    y64 = op.apply(dev[:n_rhs_64].contiguous(), pmx.PMX_PREC_FP64_DIRECT).cpu().numpy().T
    st = op.stats()
    say(f"[fullsize] fmm levels {st.fmm_levels}, boxes {st.fmm_boxes}, m2l pairs {st.fmm_m2l_pairs}")
    ptr, _, _, _ = op.export_near()
    orc = OracleOperator.from_problem(prob)
    tg = stratified_targets(prob.n, prob.surface.q, ptr, N_ROWS, seed=seed + 1)
    ref = apply_rows(orc, factory, tg, sig)
    e64 = max(max_rel(y64[tg, r], ref[:, r]) for r in range(n_rhs_64))
    em = max(max_rel(ym[tg, r], ref[:, r]) for r in range(n_rhs_mixed))
    say(f"[fullsize] {len(tg)} sampled rows: FP64 err {e64:.2e} ({n_rhs_64} rhs), mixed err {em:.2e} "
        f"({n_rhs_mixed} rhs)")
    assert e64 <= 1e-12 and em <= 1e-5
    return op, orc, tg


def residual_rows(orc, factory, prob, tg, sig):
    """max-abs of f - A sigma over the sampled rows / max-abs of f there (f mean-zero)."""
    f0 = prob.f - (prob.f * orc.w[:, None]).sum(0) / orc.w.sum()
    r = f0[tg] - apply_rows(orc, factory, tg, sig)
    return float(np.abs(r).max() / np.abs(f0[tg]).max())


def test_ellipsoid_full(ctx):
    check_rows(ctx, ellipsoid_problem(), ("ellipsoid_problem", {}), 2, 2, seed=14)


def test_star_full(ctx):
    """Rows of both applies, then the mixed solve (FMM inner GMRES, FP64 refinement) to 1e-8: the
    returned density's residual in the oracle's discrete system, on the sampled rows, is at that level."""
    from paper_2401_12501_amd import pmx
    prob = star_problem()
    factory = ("star_problem", {})
    op, orc, tg = check_rows(ctx, prob, factory, 1, 1, seed=41)
    o = pmx.pmx_default_options()
    o.precision = pmx.PMX_PREC_MIXED_FMM
    o.ir_tol = 1e-8
    sig, _, info = op.solve(np.ascontiguousarray(prob.f.T), o)
    rel = residual_rows(orc, factory, prob, tg, sig.T)
    say(f"[fullsize] star mixed solve: ir {info[0].ir_steps}, inner iters {info[0].iters_total}, "
        f"residual {info[0].rel_residual:.2e}, oracle-row residual {rel:.2e}")
    assert info[0].rel_residual <= 1e-8 and rel <= 1e-8
    # representation u = K[sigma] of that solution (FP64 log-kernel direct sum plus the parametrix
    # near blocks D), mean removed.  The oracle's rows come before the mean is removed, so the GPU
    # rows differ from them by one constant: the spread of the differences is the error.
    u = op.represent(np.ascontiguousarray(sig)).T
    ref_u = apply_rows(orc, factory, tg, sig.T, kernel="K")
    d = u[tg] - ref_u
    err_u = np.abs(d - d.mean(0)).max() / np.abs(ref_u - ref_u.mean(0)).max()
    mean_u = abs(float(orc.w @ u[:, 0])) / orc.w.sum() / np.abs(u).max()
    say(f"[fullsize] star representation: sampled-row error {err_u:.2e}, weighted mean {mean_u:.1e}")
    assert err_u <= 1e-12 and mean_u <= 1e-12


def test_wobbly_torus_full_16rhs(ctx):
    """Applies with 2 (FP64) and 16 (mixed) right-hand sides on sampled rows, then the joint mixed
    solve of the 16 right-hand sides with FP64 refinement to 1e-8, as the workload runs it: every
    column's residual in the oracle's discrete system, on the sampled rows, is at that level."""
    from paper_2401_12501_amd import pmx
    prob = wobbly_torus_problem()
    factory = ("wobbly_torus_problem", {})
    op, orc, tg = check_rows(ctx, prob, factory, 2, 16, seed=42)
    import torch
    o = pmx.pmx_default_options()
    o.precision = pmx.PMX_PREC_MIXED_FMM
    o.ir_tol = 1e-8
    f = torch.tensor(np.ascontiguousarray(prob.f.T), device="cuda:0")
    sig, _, info = op.solve(f, o)
    sig = sig.cpu().numpy()
    rel = residual_rows(orc, factory, prob, tg, sig.T)
    say(f"[fullsize] torus 16-rhs mixed solve: ir {info[0].ir_steps}, inner iters "
        f"{[i.iters_total for i in info][:4]}..., residual {max(i.rel_residual for i in info):.2e}, "
        f"oracle-row residual {rel:.2e}, t {info[0].t_solve:.2f}s")
    assert max(i.rel_residual for i in info) <= 1e-8 and rel <= 1e-8
