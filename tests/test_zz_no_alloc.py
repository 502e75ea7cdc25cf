"""The allocation-free apply (pmx_apply_noalloc) against pmx_apply with the FP64 direct far field.

pmx_apply_noalloc runs the same kernels as the FP64 direct apply with its scratch in the
library's static device array instead of buffers the operator allocates, so its output must
equal pmx_apply's bit for bit.  Two calls in a row, the second on a smaller input (another
operator, fewer nodes and right-hand sides), check that what the first call left in the shared
array does not leak into the second.  The operator used only through the allocation-free call
must hold no more device memory afterwards than before, and the library must refuse inputs
whose scratch exceeds the array and host arrays (before any device work).  A complex operator
(c > 0) takes its densities in the library's layout of 2N doubles each.
"""
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import sphere_problem, ellipsoid_problem, random_density

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def build(ctx, prob):
    from paper_2401_12501_amd import pmx
    surf = pmx.Surface.from_inputs(ctx, prob.surface)
    return surf, pmx.Operator(surf, prob.a, prob.grad_a)


def test_noalloc_matches_apply_twice():
    import torch
    from paper_2401_12501_amd import pmx
    ctx = pmx.Context(0)
    cases = [(sphere_problem(k=2, q=8), 3, 51), (ellipsoid_problem(k=1, q=7), 1, 52)]   # 1,536 then 294 nodes
    for prob, n_rhs, seed in cases:
        say(f"[noalloc] {prob.name}: N={prob.n}, {n_rhs} rhs")
        surf, op_ref = build(ctx, prob)
        _, op_na = build(ctx, prob)
        sig = torch.tensor(random_density(prob.n, n_rhs, seed=seed).T.copy(), device="cuda:0")
        bytes_before = op_na.stats().device_bytes
        y_na = op_na.apply_noalloc(sig)
        torch.cuda.synchronize()
        assert op_na.stats().device_bytes == bytes_before      # no operator buffer was allocated
        y_ref = op_ref.apply(sig, pmx.PMX_PREC_FP64_DIRECT)
        torch.cuda.synchronize()
        assert torch.equal(y_na, y_ref), f"max diff {(y_na - y_ref).abs().max().item():.3e}"
        # a repeat on the same operator gives the same bits
        assert torch.equal(op_na.apply_noalloc(sig), y_ref)
        say(f"[noalloc] {prob.name}: identical to pmx_apply (FP64 direct)")


def test_noalloc_complex_matches_apply_twice():
    """A complex operator (c > 0): densities in the library's layout (n_rhs, 2, N), real parts then
    imaginary parts; the allocation-free apply equals pmx_apply bit for bit, on two calls in a row,
    the second with fewer nodes and densities."""
    import torch
    from paper_2401_12501_amd import pmx
    from paper_2401_12501_amd.inputs import helmholtz_ellipsoid_problem, helmholtz_sphere_problem
    ctx = pmx.Context(0)
    cases = [(helmholtz_sphere_problem(k=2, q=8, positive=True), 3, 61),
             (helmholtz_ellipsoid_problem(k=1, q=7, positive=True), 1, 62)]   # 1,536 then 294 nodes
    for prob, n_rhs, seed in cases:
        say(f"[noalloc c>0] {prob.name}: N={prob.n}, {n_rhs} complex densities")
        surf = pmx.Surface.from_inputs(ctx, prob.surface)
        op_ref = pmx.Operator(surf, prob.a, prob.grad_a, c=prob.c)
        op_na = pmx.Operator(surf, prob.a, prob.grad_a, c=prob.c)
        assert op_na.complex
        d = np.stack([random_density(prob.n, n_rhs, seed=seed).T, random_density(prob.n, n_rhs, seed=seed + 1).T],
                     axis=1)
        sig = torch.tensor(np.ascontiguousarray(d), device="cuda:0")
        bytes_before = op_na.stats().device_bytes
        y_na = op_na.apply_noalloc(sig)
        torch.cuda.synchronize()
        assert op_na.stats().device_bytes == bytes_before
        y_ref = op_ref.apply_planar(sig, pmx.PMX_PREC_FP64_DIRECT)
        torch.cuda.synchronize()
        assert torch.equal(y_na, y_ref), f"max diff {(y_na - y_ref).abs().max().item():.3e}"
        assert torch.equal(op_na.apply_noalloc(sig), y_ref)
        say(f"[noalloc c>0] {prob.name}: identical to pmx_apply (FP64 direct)")


def test_noalloc_rejections():
    import torch
    from paper_2401_12501_amd import pmx
    ctx = pmx.Context(0)
    # 1,024 densities on 1,536 nodes need about 315 MB of scratch, above PMX_NOALLOC_SCRATCH_BYTES:
    # refused on the host before any launch
    sph = sphere_problem(k=2, q=8)
    _, op_big = build(ctx, sph)
    big = torch.zeros((1024, sph.n), dtype=torch.float64, device="cuda:0")
    code = op_big.apply_noalloc(big, out=torch.empty_like(big), check=False)
    assert code == pmx.PMX_ERR_TOO_LARGE, code
    assert "scratch" in pmx.pmx_last_error()
    prob = ellipsoid_problem(k=1, q=7)
    surf, op = build(ctx, prob)
    # host arrays are refused (the call takes device arrays only)
    h = np.zeros(prob.n)
    code = pmx.lib().pmx_apply_noalloc(op.h, 1, h.ctypes.data, h.ctypes.data, None)
    assert code == pmx.PMX_ERR_INVALID, code
    # the operator still works afterwards
    sig = torch.tensor(random_density(prob.n, 1, seed=53).T.copy(), device="cuda:0")
    assert torch.equal(op.apply_noalloc(sig), op.apply(sig, pmx.PMX_PREC_FP64_DIRECT))
    say("[noalloc] rejections: TOO_LARGE and host arrays refused; operator usable afterwards")
