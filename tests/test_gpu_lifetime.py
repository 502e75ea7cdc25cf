"""Handle lifetime: operators (with their FMM tree, multi-RHS buffers and D blocks built by use)
and surfaces return their device memory when destroyed, and the device-memory figure an operator
reports grows as those parts are built."""
import gc
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import ellipsoid_problem, random_density

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def free_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_create_use_destroy_returns_memory():
    import torch
    from paper_2401_12501_amd import pmx
    ctx = pmx.Context(0)
    p = ellipsoid_problem(k=4, q=8)          # 6,144 nodes
    sig = np.ascontiguousarray(random_density(p.n, 16, seed=3).T)
    # one full cycle first, so that one-time runtime allocations are not counted
    surf = pmx.Surface.from_inputs(ctx, p.surface)
    op = pmx.Operator(surf, p.a, p.grad_a)
    op.apply(sig, pmx.PMX_PREC_MIXED_FMM)
    op.close()
    surf.close()
    gc.collect()
    base = free_bytes()
    held = []
    for k in range(6):
        surf = pmx.Surface.from_inputs(ctx, p.surface)
        op = pmx.Operator(surf, p.a, p.grad_a)
        b0 = op.stats().device_bytes
        op.apply(sig[:1], pmx.PMX_PREC_MIXED_FMM)          # builds the FMM tree
        op.apply(sig, pmx.PMX_PREC_MIXED_FMM)              # 16 right-hand sides: block buffers
        op.represent(sig[:1])                              # D blocks
        b1 = op.stats().device_bytes
        assert b1 > b0 > 0
        held.append(b1)
        op.close()
        surf.close()
    gc.collect()
    after = free_bytes()
    # every cycle's memory is back: the free figure moves by less than one operator's footprint
    assert base - after < min(held), (base, after, held)
    say(f"[lifetime] 6 create/use/destroy cycles: operator footprint {held[0] / 2**20:.1f} MiB, "
        f"free memory change {(base - after) / 2**20:.2f} MiB")


def test_destroy_in_any_order():
    """A surface holds a reference on its context and an operator on its surface: the context may
    be destroyed first and the operator still applies (the same values), then the surface, then
    the operator; a garbage cycle holding all three (finalizers in arbitrary order) is collected
    cleanly."""
    from paper_2401_12501_amd import pmx
    p = ellipsoid_problem(k=2, q=6)
    sig = np.ascontiguousarray(random_density(p.n, 1, seed=4).T)
    ctx = pmx.Context(0)
    surf = pmx.Surface.from_inputs(ctx, p.surface)
    op = pmx.Operator(surf, p.a, p.grad_a)
    y0 = op.apply(sig, pmx.PMX_PREC_FP64_DIRECT)
    ctx.close()
    y1 = op.apply(sig, pmx.PMX_PREC_FP64_DIRECT)
    surf.close()
    y2 = op.apply(sig, pmx.PMX_PREC_FP64_DIRECT)
    op.close()
    assert np.array_equal(y0, y1) and np.array_equal(y0, y2)
    for _ in range(3):
        ctx = pmx.Context(0)
        surf = pmx.Surface.from_inputs(ctx, p.surface)
        holder = {"ops": [pmx.Operator(surf, p.a, p.grad_a) for _ in range(2)], "surf": surf, "ctx": ctx}
        holder["self"] = holder
        del ctx, surf, holder
        gc.collect()
    say("[lifetime] out-of-order destroys and garbage cycles: clean")
