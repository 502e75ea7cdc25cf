"""The C ABI's error contract on the GPU: invalid shapes, data and options are rejected with
PMX_ERR_INVALID and an inward-oriented surface with PMX_ERR_ORIENTATION, each with a message, and a
rejected call leaves the handles it was given usable.  The checks run on the host or in validation
kernels that only flag bad values, so every kernel exits normally."""
import sys

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import sphere_problem, random_density

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2401_12501_amd import pmx
    return pmx.Context(0)


@pytest.fixture(scope="module")
def prob():
    return sphere_problem(k=2, q=6)       # 24 patches x 6x6 nodes = 864 nodes


def status_of(fn):
    """The status code of the PmxError that fn raises (its message must not be empty)."""
    from paper_2401_12501_amd import pmx
    with pytest.raises(pmx.PmxError) as e:
        fn()
    assert "):" in str(e.value) and str(e.value).split("):", 1)[1].strip()
    return e.value.code


def make_surface(ctx, s, q=None, **replace):
    from paper_2401_12501_amd import pmx
    arr = {k: np.array(getattr(s, k), dtype=np.float64) for k in ("x", "xu", "xv", "xuu", "xuv", "xvv")}
    arr.update(replace)
    return pmx.Surface(ctx, s.n_patches, s.q if q is None else q, arr["x"], arr["xu"], arr["xv"], arr["xuu"],
                       arr["xuv"], arr["xvv"])


def test_surface_errors(ctx, prob):
    from paper_2401_12501_amd import pmx
    s = prob.surface
    assert status_of(lambda: make_surface(ctx, s, q=1)) == pmx.PMX_ERR_INVALID
    assert status_of(lambda: make_surface(ctx, s, q=17)) == pmx.PMX_ERR_INVALID
    x = np.array(s.x, dtype=np.float64)
    x[5, 1] = np.nan
    assert status_of(lambda: make_surface(ctx, s, x=x)) == pmx.PMX_ERR_INVALID
    # u and v exchanged: the same surface with normals x_u x x_v pointing inward
    inward = dict(xu=np.array(s.xv), xv=np.array(s.xu), xuu=np.array(s.xvv), xvv=np.array(s.xuu))
    assert status_of(lambda: make_surface(ctx, s, **inward)) == pmx.PMX_ERR_ORIENTATION
    make_surface(ctx, s).close()                     # the valid surface is still accepted
    say("[errors] surface: q out of range, non-finite node, inward normals rejected")


def test_operator_and_apply_errors(ctx, prob):
    from paper_2401_12501_amd import pmx
    surf = make_surface(ctx, prob.surface)
    a, ga = np.array(prob.a, dtype=np.float64), np.array(prob.grad_a, dtype=np.float64)
    for bad in (0.0, -1.0, np.nan):
        ab = a.copy()
        ab[7] = bad
        assert status_of(lambda: pmx.Operator(surf, ab, ga)) == pmx.PMX_ERR_INVALID
    gb = ga.copy()
    gb[3, 2] = np.inf
    assert status_of(lambda: pmx.Operator(surf, a, gb)) == pmx.PMX_ERR_INVALID
    for field, value in (("fmm_order", 7), ("fmm_order", 3), ("overlap", 2), ("n_gl", 17), ("eta_near", 0.0),
                         ("precision", 5), ("gmres_restart", 0)):
        o = pmx.pmx_default_options()
        setattr(o, field, value)
        assert status_of(lambda: pmx.Operator(surf, a, ga, o)) == pmx.PMX_ERR_INVALID, field
    # a valid operator, then rejected apply calls, then the same applies as before them
    op = pmx.Operator(surf, a, ga)
    sig = np.ascontiguousarray(random_density(prob.n, 2, seed=5).T)
    y64 = op.apply(sig, pmx.PMX_PREC_FP64_DIRECT)
    ym = op.apply(sig, pmx.PMX_PREC_MIXED_FMM)
    assert status_of(lambda: op.apply(sig, 7)) == pmx.PMX_ERR_INVALID
    assert status_of(lambda: op.apply(np.zeros((1025, prob.n)), pmx.PMX_PREC_FP64_DIRECT)) == pmx.PMX_ERR_INVALID
    assert np.array_equal(op.apply(sig, pmx.PMX_PREC_FP64_DIRECT), y64)
    assert np.array_equal(op.apply(sig, pmx.PMX_PREC_MIXED_FMM), ym)
    say("[errors] operator: bad coefficient, gradient and options rejected; applies unchanged after rejected calls")
