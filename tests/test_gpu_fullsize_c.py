"""Full-size c != 0 applies against oracle rows: the 153,600-node ellipsoid surface of the bench's
c < 0 and c > 0 legs (a = 2 + x3, variable c, the non-tangent advection field), two densities (complex
for c > 0) in one apply, in the launch configuration the bench times, compared element by element
at 256 stratified targets (first and last nodes of seeded patches, the targets with the most near
patches, seeded random nodes).  The oracle's smooth-rule sums for c != 0 are NumPy rows over all
153,599 sources (tens of ms each, with scipy's Bessel and Hankel functions), so the sample is smaller
than the 1,024 rows of the c = 0 full-size tests, whose sums run in C.  Bar: 1e-12 of the largest
value of each density's rows.
"""
import ctypes as C
import os
import sys

import numpy as np
import pytest

from _oracle_rows import stratified_targets, workers
from paper_2401_12501_amd.inputs import helmholtz_ellipsoid_problem, random_density
from oracle.operator import OracleOperator
from oracle.system import blocks_parallel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_12501_amd import pmx
    return pmx.Context(0)


@pytest.mark.parametrize("positive", [False, True])
def test_helmholtz_ellipsoid_full(ctx, positive):
    from paper_2401_12501_amd import pmx
    kw = {"k": 16, "q": 10, "swirl": True, "positive": positive}
    prob = helmholtz_ellipsoid_problem(**kw)
    N = prob.n
    say(f"[full c] {prob.name}: N={N}, c in [{prob.c.min():.3f}, {prob.c.max():.3f}]")
    op = pmx.Operator(pmx.Surface.from_inputs(ctx, prob.surface), prob.a, prob.grad_a, c=prob.c, b=prob.b)
    assert op.complex == positive
    sig = random_density(N, 2, seed=41)
    if positive:
        sig = sig + 1j * random_density(N, 2, seed=42)
    y = op.apply(np.ascontiguousarray(sig.T), pmx.PMX_PREC_FP64_DIRECT).T
    ptr = np.empty(N + 1, dtype=np.int64)
    pmx._check(pmx.lib().pmx_operator_export_near(op.h, ptr.ctypes.data_as(C.c_void_p), None, None, None))
    tg = stratified_targets(N, prob.surface.q, ptr, 256, seed=43)
    orc = OracleOperator.from_problem(prob)
    blocks = blocks_parallel(("paper_2401_12501_amd.inputs", "helmholtz_ellipsoid_problem", kw), ROOT, tg,
                             kernels=("R",), workers=workers())
    say(f"[full c] {prob.name}: oracle blocks of {len(tg)} targets ready")
    ref = orc.apply_rows(tg, sig, blocks)
    errs = [float(np.abs(y[tg, r] - ref[:, r]).max() / np.abs(ref[:, r]).max()) for r in range(2)]
    say(f"[full c] {prob.name}: {len(tg)} rows, errors {errs[0]:.2e} {errs[1]:.2e}")
    assert max(errs) <= 1e-12
