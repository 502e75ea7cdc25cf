"""Pins of the oracle's large-size machinery (CPU only): the C far sums, GMRES and the whole-system
class that writes the large solution fixtures.

* C far sums (``oracle/far.c``) against the NumPy rows on a variable-coefficient ellipsoid (an
  independent implementation of the same formula, in another language) and against the
  unit-sphere closed form: with a = 1, n = x and H = 1 every remainder value is -1/(4 pi)
  (eq:explicit_remainderLB on a sphere), so a row is -(1/(4 pi)) sum_{j != i} w_j sigma_j.
* GMRES (CGS2) against dense LU on small surfaces.
* Near blocks from worker processes equal the serial ones, and the whole-system apply, solve and
  representation equal the dense operator's.
"""
import math
import os

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import ellipsoid_problem, sphere_problem, random_density
from oracle import cfar
from oracle.gmres import gmres
from oracle.operator import OracleOperator
from oracle.system import FullSystem, blocks_parallel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RAGGED = ("paper_2401_12501_amd.inputs", "ellipsoid_problem", {"k": 1, "q": 7})


@pytest.fixture(scope="module")
def ragged():
    p = ellipsoid_problem(k=1, q=7)
    orc = OracleOperator.from_problem(p)
    blocks = orc.blocks(np.arange(p.n), kernels=("R", "K"))
    return p, orc, blocks, orc.dense_matrix(blocks)


def test_c_far_rows_match_numpy(ragged):
    cfar.build()
    p, orc, _, _ = ragged
    sig = random_density(p.n, 3, seed=61)
    tg = np.arange(p.n)
    for kernel in ("R", "K"):
        a = orc.far_rows(tg, sig, kernel)
        b = cfar.far_rows(orc, tg, sig, kernel)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max(), kernel
    assert cfar.threads() >= 1


def test_c_far_rows_sphere_closed_form():
    p = sphere_problem(k=2, q=8, const_a=True)
    orc = OracleOperator.from_problem(p)
    sig = random_density(p.n, 2, seed=62)
    tg = np.arange(0, p.n, 7)
    got = cfar.far_rows(orc, tg, sig, "R")
    ws = orc.w @ sig
    ref = -(ws[None, :] - orc.w[tg, None] * sig[tg]) / (4 * math.pi)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_gmres_matches_dense_lu(ragged):
    p, orc, _, A = ragged
    f, _ = orc.project_mean_zero(p.f)
    x_lu = np.linalg.solve(A, f[:, 0])
    x, res, its = gmres(lambda v: A @ v, f[:, 0], tol=1e-13)
    assert res <= 1e-13 and its < 60
    assert np.abs(x - x_lu).max() <= 1e-12 * np.abs(x_lu).max()


def test_gmres_sphere_variable_a():
    p = sphere_problem(k=2, q=8)
    orc = OracleOperator.from_problem(p)
    A = orc.dense_matrix()
    f, _ = orc.project_mean_zero(p.f)
    x_lu = np.linalg.solve(A, f[:, 0])
    x, res, its = gmres(lambda v: A @ v, f[:, 0], tol=1e-13)
    assert res <= 1e-13
    assert np.abs(x - x_lu).max() <= 1e-12 * np.abs(x_lu).max()


def test_blocks_parallel_equal_serial(ragged):
    p, orc, blocks, _ = ragged
    tg = np.arange(0, p.n, 5)
    par = blocks_parallel(RAGGED, ROOT, tg, kernels=("R", "K"), workers=2, chunk=16)
    for i, (plist, blk) in zip(tg, par):
        ref_plist, ref_blk = blocks[i]
        assert np.array_equal(plist, ref_plist)
        for k in ("R", "K"):
            assert np.array_equal(blk[k], ref_blk[k])


def test_full_system_matches_dense(ragged):
    p, orc, _, A = ragged
    fs = FullSystem(p, RAGGED, ROOT, workers=2, kernels=("R", "K"))
    sig = random_density(p.n, 2, seed=63)
    ref = A @ sig
    assert np.abs(fs.apply(sig) - ref).max() <= 1e-13 * np.abs(ref).max()
    s, res, its = fs.solve(p.f)
    s_lu = orc.solve(p.f, A)
    assert max(res) <= 1e-13
    assert np.abs(s - s_lu).max() <= 1e-12 * np.abs(s_lu).max()
    u = fs.represent(s)
    u_ref = orc.represent(s)
    assert np.abs(u - u_ref).max() <= 1e-13 * np.abs(u_ref).max()
