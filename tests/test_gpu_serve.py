"""Continuous-batching server: results alone vs in the mix, admission, failure handling.

Requests are small members of the serving workload families (sphere, random-axis
ellipsoid, torus) with seeded coefficient fields and right-hand sides.  Every kernel
of the path reduces in a fixed order, so a request's solution in the mix must equal
its solution alone (checked to 1e-12; the mixed-path bar is 1e-8).
"""
import sys
import time

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import cube_sphere, torus
from paper_2401_12501_amd.inputs import fields as F

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problems():
    rng = np.random.default_rng(31)
    out = []
    for k, kind in enumerate(["sphere", "ellipsoid", "torus", "ellipsoid", "sphere"]):
        if kind == "torus":
            s = torus(8, 4, 8, R=1.0, r=float(rng.uniform(0.3, 0.5)))
        else:
            axes = (1.0, 1.0, 1.0) if kind == "sphere" else tuple(rng.uniform(0.5, 1.5, 3))
            s = cube_sphere(2 + k % 2, 8, axes=axes)
        a, ga = F.eval_field(F.a_seed_field(100 + k), s.x)
        f = F.solid_harmonic_rhs(s.x, 200 + k)
        out.append((kind, s, a, ga, f))
    return out


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_12501_amd import pmx
    return pmx.Context(0)


def run_all(server, tickets, timeout=120.0):
    res = {}
    t0 = time.time()
    max_active = 0
    while len(res) < len(tickets):
        na, nq = server.step()
        max_active = max(max_active, na)
        for t in tickets:
            if t not in res:
                r = server.poll(t)
                if r is not None:
                    res[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return res, max_active


def test_alone_vs_mixed(ctx):
    from paper_2401_12501_amd import pmx
    probs = problems()
    alone = []
    for kind, s, a, ga, f in probs:
        sv = pmx.Server(ctx, max_active=1)
        t = sv.submit(s, a, ga, f, want_u=True)
        res, _ = run_all(sv, [t])
        code, sig, u, info, times = res[t]
        assert code == pmx.PMX_OK, pmx.pmx_last_error()
        assert info.rel_residual <= 1e-8
        alone.append((sig, u))
        say(f"[serve alone] {kind} N={s.n}: ir {info.ir_steps}, iters {info.iters_total}, res "
            f"{info.rel_residual:.2e}, service {times[1]:.3f}s")
        sv.close()
    sv = pmx.Server(ctx, max_active=3)
    tickets = [sv.submit(s, a, ga, f, want_u=True) for (_, s, a, ga, f) in probs]
    res, max_active = run_all(sv, tickets)
    assert max_active >= 2
    bs = sv.stats()
    say(f"[serve mix] batches {bs['batches']}, applies {bs['applies']}, largest batch {bs['max_batch']}")
    assert bs["max_batch"] >= 2 and bs["applies"] > bs["batches"]      # applies shared launches
    for (sig0, u0), t, (kind, s, *_rest) in zip(alone, tickets, probs):
        code, sig, u, info, times = res[t]
        assert code == pmx.PMX_OK
        d = np.abs(sig - sig0).max() / np.abs(sig0).max()
        du = np.abs(u - u0).max() / np.abs(u0).max()
        say(f"[serve mix] {kind} N={s.n}: max rel diff sigma {d:.2e}, u {du:.2e}, queued {times[0]:.3f}s")
        assert d <= 1e-12 and du <= 1e-12
    # the server's answer equals a direct pmx_solve with the same options
    kind, s, a, ga, f = probs[1]
    surf = pmx.Surface.from_inputs(ctx, s)
    o = pmx.pmx_default_options()
    o.precision = pmx.PMX_PREC_MIXED_FMM
    op = pmx.Operator(surf, a, ga, o)
    sig_d, _, _ = op.solve(f[None, :].copy(), o)
    assert np.abs(sig_d[0] - alone[1][0]).max() <= 1e-12 * np.abs(sig_d).max()


def test_admission_budget_and_rejection(ctx):
    from paper_2401_12501_amd import pmx
    probs = problems()[:3]
    small = pmx.Context(0, hbm_budget_bytes=50 << 20)
    sv = pmx.Server(small, max_active=3)
    tickets = [sv.submit(s, a, ga, f) for (_, s, a, ga, f) in probs]
    res, max_active = run_all(sv, tickets)
    bs = sv.stats()
    say(f"[serve budget] 50 MiB budget: max active {max_active}, held for memory {bs['held_for_memory']}, "
        f"peak reserved {bs['peak_reserved_bytes'] / 2**20:.1f} MiB")
    assert max_active == 1                                    # one request's footprint at a time
    assert bs["held_for_memory"] >= 1 and 0 < bs["peak_reserved_bytes"] <= 50 << 20
    assert all(r[0] == pmx.PMX_OK for r in res.values())
    big = torus(64, 32, 8)                                    # 131,072 nodes: over the budget
    a, ga = F.eval_field(F.a_const(1.0), big.x)
    with pytest.raises(pmx.PmxError) as e:
        sv.submit(big, a, ga, np.ones(big.n))
    assert e.value.code == pmx.PMX_ERR_TOO_LARGE
    sv.close()


def test_not_converged_and_cancel(ctx):
    from paper_2401_12501_amd import pmx
    probs = problems()[:3]
    o = pmx.pmx_default_options()
    o.precision = pmx.PMX_PREC_MIXED_FMM
    o.max_ir = 0                                              # no refinement step allowed
    sv = pmx.Server(ctx, opts=o, max_active=1)
    t_bad = sv.submit(*probs[0][1:])
    res, _ = run_all(sv, [t_bad])
    code, sig, u, info, times = res[t_bad]
    assert code == pmx.PMX_ERR_NOT_CONVERGED and info.rel_residual > 1e-8
    sv.close()
    sv = pmx.Server(ctx, max_active=1)
    t = [sv.submit(*p[1:]) for p in probs]
    sv.cancel(t[2])                                           # still queued
    res, _ = run_all(sv, t)
    assert res[t[2]][0] == pmx.PMX_ERR_CANCELLED
    assert res[t[0]][0] == pmx.PMX_OK and res[t[1]][0] == pmx.PMX_OK
    sv.close()
