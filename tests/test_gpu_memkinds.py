"""Host and device buffers through the C ABI give the same bits: a surface and operator built from
host arrays or from device tensors, applies on both paths, the mixed solve with its representation,
and an apply issued on a caller's own stream (default priority) instead of torch's current one."""
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import ellipsoid_problem, random_density

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2401_12501_amd import pmx
    ctx = pmx.Context(0)
    p = ellipsoid_problem(k=4, q=8)          # 96 patches x 8x8 = 6,144 nodes
    s = p.surface
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda:0")
    surf_h = pmx.Surface.from_inputs(ctx, s)
    surf_d = pmx.Surface(ctx, s.n_patches, s.q, *[dev(getattr(s, k)) for k in ("x", "xu", "xv", "xuu", "xuv", "xvv")])
    op_h = pmx.Operator(surf_h, p.a, p.grad_a)
    op_d = pmx.Operator(surf_d, dev(p.a), dev(p.grad_a))
    return p, op_h, op_d


def test_applies_host_vs_device(setup):
    import torch
    from paper_2401_12501_amd import pmx
    p, op_h, op_d = setup
    sig = np.ascontiguousarray(random_density(p.n, 3, seed=17).T)
    sig_d = torch.tensor(sig, device="cuda:0")
    for prec in (pmx.PMX_PREC_FP64_DIRECT, pmx.PMX_PREC_MIXED_FMM, pmx.PMX_PREC_FP32_DIRECT):
        yh = op_h.apply(sig, prec)
        yd = op_d.apply(sig_d, prec).cpu().numpy()
        assert np.array_equal(yh, yd), prec
        # the host-built operator with device buffers, and the device-built one with host buffers
        assert np.array_equal(op_h.apply(sig_d, prec).cpu().numpy(), yh), prec
        assert np.array_equal(op_d.apply(sig, prec), yh), prec
    say(f"[memkinds] N={p.n}: applies on three paths identical for host and device buffers and surfaces")


def test_solve_and_representation_host_vs_device(setup):
    import torch
    from paper_2401_12501_amd import pmx
    p, op_h, op_d = setup
    o = pmx.pmx_default_options()
    o.precision = pmx.PMX_PREC_MIXED_FMM
    f = np.ascontiguousarray(p.f.T)
    sh, uh, ih = op_h.solve(f, o, want_u=True)
    sd, ud, idv = op_d.solve(torch.tensor(f, device="cuda:0"), o, want_u=True)
    assert ih[0].rel_residual <= 1e-8 and ih[0].iters_total == idv[0].iters_total
    assert np.array_equal(sh, sd.cpu().numpy()) and np.array_equal(uh, ud.cpu().numpy())
    assert np.array_equal(op_h.represent(sh), op_d.represent(sd).cpu().numpy())
    say(f"[memkinds] mixed solve ({ih[0].iters_total} inner iterations) and representation identical")


def test_apply_on_caller_stream(setup):
    import torch
    from paper_2401_12501_amd import pmx
    p, op_h, op_d = setup
    sig_d = torch.tensor(np.ascontiguousarray(random_density(p.n, 1, seed=19).T), device="cuda:0")
    ref = op_d.apply(sig_d, pmx.PMX_PREC_MIXED_FMM).cpu().numpy()
    st = torch.cuda.Stream()                 # default priority
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        y = op_d.apply(sig_d, pmx.PMX_PREC_MIXED_FMM)
    st.synchronize()
    assert np.array_equal(y.cpu().numpy(), ref)
    say("[memkinds] apply on a caller's stream identical")
