"""The largest call the C ABI accepts: 1,024 right-hand sides in one apply (64 blocks of 16 on the
mixed path, groups of 16 on the FP64 path).  FP64 columns equal single-rhs applies bit for bit; mixed
columns agree to the FP32 summation order of the block kernels (1e-5 of the far field)."""
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import sphere_problem, random_density

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_1024_rhs():
    from paper_2401_12501_amd import pmx
    ctx = pmx.Context(0)
    p = sphere_problem(k=2, q=6)             # 864 nodes
    surf = pmx.Surface.from_inputs(ctx, p.surface)
    op = pmx.Operator(surf, p.a, p.grad_a)
    sig = np.ascontiguousarray(random_density(p.n, 1024, seed=51).T)     # (1024, N)
    y64 = op.apply(sig, pmx.PMX_PREC_FP64_DIRECT)
    ym = op.apply(sig, pmx.PMX_PREC_MIXED_FMM)
    w = op.export_geometry()["w"]
    worst = 0.0
    for r in (0, 1, 15, 16, 511, 1008, 1023):
        s1 = sig[r:r + 1].copy()
        assert np.array_equal(op.apply(s1, pmx.PMX_PREC_FP64_DIRECT)[0], y64[r]), r
        y1 = op.apply(s1, pmx.PMX_PREC_MIXED_FMM)[0]
        far = y1 - s1[0] - s1[0] @ w
        worst = max(worst, float(np.abs(ym[r] - y1).max() / np.abs(far).max()))
    say(f"[limits] 1024 rhs: FP64 columns identical to single applies; mixed columns within {worst:.2e} of the far field")
    assert worst < 1e-5
