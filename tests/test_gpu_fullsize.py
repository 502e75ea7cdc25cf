"""Full-size workloads on sampled outputs: the star (8,214 patches, q = 8, 525,696 nodes;
apply, mixed solve and representation) and the wobbly torus (256 x 128 patches, q = 8,
2,097,152 nodes, 16 right-hand sides).

The oracle evaluates single rows of the operator (near blocks and the far sum over all
sources) at seeded random targets; the GPU applies the whole operator in the launch
configuration the benchmark uses.  FP64 path: within 1e-12 of the oracle rows; mixed
path (FMM far field): within 1e-4 (FP32 interpolation error, removed by refinement).
"""
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import star_problem, wobbly_torus_problem, random_density
from oracle.operator import OracleOperator

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_12501_amd import pmx
    return pmx.Context(0)


def check_rows(ctx, prob, n_rhs_64, n_rhs_mixed, n_rows, seed):
    from paper_2401_12501_amd import pmx
    say(f"[fullsize] {prob.name}: N={prob.n}")
    surf = pmx.Surface.from_inputs(ctx, prob.surface)
    op = pmx.Operator(surf, prob.a, prob.grad_a)
    st = op.stats()
    say(f"[fullsize] near pairs {st.near_pairs}, device MB {st.device_bytes / 2**20:.0f}")
    import torch
    sig = random_density(prob.n, max(n_rhs_64, n_rhs_mixed), seed=seed)
    dev = torch.tensor(np.ascontiguousarray(sig.T), device="cuda:0")
    ym = op.apply(dev[:n_rhs_mixed].contiguous(), pmx.PMX_PREC_MIXED_FMM).cpu().numpy().T
    y64 = op.apply(dev[:n_rhs_64].contiguous(), pmx.PMX_PREC_FP64_DIRECT).cpu().numpy().T
    st = op.stats()
    say(f"[fullsize] fmm levels {st.fmm_levels}, boxes {st.fmm_boxes}, m2l pairs {st.fmm_m2l_pairs}")
    orc = OracleOperator.from_problem(prob)
    rng = np.random.default_rng(seed + 1)
    tg = np.concatenate([[0, prob.n - 1], rng.choice(prob.n, n_rows - 2, replace=False)])
    ref = orc.apply_rows(tg, sig)
    e64 = np.abs(y64[tg] - ref[:, :n_rhs_64]).max() / np.abs(ref[:, :n_rhs_64]).max()
    em = np.abs(ym[tg] - ref[:, :n_rhs_mixed]).max() / np.abs(ref[:, :n_rhs_mixed]).max()
    say(f"[fullsize] sampled rows: FP64 rel err {e64:.2e} ({n_rhs_64} rhs), mixed rel err {em:.2e} "
        f"({n_rhs_mixed} rhs)")
    assert e64 <= 1e-12 and em <= 1e-4
    return op, orc


def test_star_full(ctx):
    """Rows of both applies, then the mixed solve (FMM inner GMRES, FP64 refinement) to 1e-8: the
    returned density's residual in the oracle's discrete system, on sampled rows, is at that level."""
    from paper_2401_12501_amd import pmx
    prob = star_problem()
    op, orc = check_rows(ctx, prob, 1, 1, 12, seed=41)
    o = pmx.pmx_default_options()
    o.precision = pmx.PMX_PREC_MIXED_FMM
    o.ir_tol = 1e-8
    sig, _, info = op.solve(np.ascontiguousarray(prob.f.T), o)
    rng = np.random.default_rng(43)
    tg = np.concatenate([[0, prob.n - 1], rng.choice(prob.n, 10, replace=False)])
    f0 = prob.f - (prob.f * orc.w[:, None]).sum(0) / orc.w.sum()
    r = f0[tg] - orc.apply_rows(tg, sig.T)
    rel = np.abs(r).max() / np.abs(f0[tg]).max()
    say(f"[fullsize] star mixed solve: ir {info[0].ir_steps}, inner iters {info[0].iters_total}, "
        f"residual {info[0].rel_residual:.2e}, oracle-row residual {rel:.2e}")
    assert info[0].rel_residual <= 1e-8 and rel <= 1e-7
    # representation u = K[sigma] of that solution (FP64 log-kernel direct sum plus the parametrix
    # near blocks D), mean removed.  The oracle's rows come before the mean is removed, so the GPU
    # rows differ from them by one constant: the spread of the differences is the error.  FP64
    # throughout; the small-case bar (weighted over all nodes) is 1e-12, the max over sampled rows
    # gets 10x that.
    u = op.represent(np.ascontiguousarray(sig)).T
    ref_u = orc.represent_rows(tg, sig.T)
    d = u[tg] - ref_u
    err_u = np.abs(d - d.mean(0)).max() / np.abs(ref_u - ref_u.mean(0)).max()
    mean_u = abs(float(orc.w @ u[:, 0])) / orc.w.sum() / np.abs(u).max()
    say(f"[fullsize] star representation: sampled-row error {err_u:.2e}, weighted mean {mean_u:.1e}")
    assert err_u <= 1e-11 and mean_u <= 1e-12


def test_wobbly_torus_full_16rhs(ctx):
    check_rows(ctx, wobbly_torus_problem(), 2, 16, 10, seed=42)
