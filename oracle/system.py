"""The oracle's whole Nystrom system at sizes beyond row-by-row Python (oracle, FP64).

TEST INFRASTRUCTURE ONLY.  Same discrete operator as ``OracleOperator`` (Section 6.1,
eq:IEsum with the rank-one term of Section 3):

  (A sigma)_i = sigma_i + sum_{j != i} w_j R(x_i, x_j) sigma_j
              + sum_{P in near(i)} C_{i,P,:} . sigma_P + sum_j w_j sigma_j,

assembled from the same pieces: the near/self correction blocks of every target come from
``OracleOperator.blocks`` (computed once, in worker processes that each rebuild the same seeded
problem), the smooth-rule sums from the C oracle (``cfar``, all host cores), and the block sums
through a sparse matrix whose row i holds target i's blocks at their patches' columns (a library
sparse product).  ``solve`` runs the oracle's GMRES on it (Section 6 and Section 7 solve the
system with GMRES); ``represent`` is eq:representation with the parametrix blocks, mean removed.
"""
from __future__ import annotations

import importlib
import multiprocessing as mp
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import cfar
from .gmres import gmres
from .operator import OracleOperator

_W = {}


def _worker_init(root: str, factory: tuple, opts: dict, one_thread: bool = True):
    if one_thread:   # the workers already use every core
        from threadpoolctl import threadpool_limits
        _W["limits"] = threadpool_limits(limits=1)
    if root not in sys.path:
        sys.path.insert(0, root)
    if one_thread:
        import torch
        torch.set_num_threads(1)
    mod, fn, kw = factory
    prob = getattr(importlib.import_module(mod), fn)(**kw)
    _W["orc"] = OracleOperator.from_problem(prob, **opts)


def _worker_blocks(targets, kernels):
    return _W["orc"].blocks(np.asarray(targets), kernels=kernels)


class BlockPool:
    """Worker processes (spawned, so that a parent that has touched a GPU is never forked), each
    holding an ``OracleOperator`` of the same seeded problem: factory = (module, function,
    kwargs) of the problem builder.  ``blocks`` returns ``OracleOperator.blocks`` in target order."""

    def __init__(self, factory: tuple, root: str, workers: int | None = None, opts: dict | None = None):
        self.workers = workers or os.cpu_count() or 1
        self.ex = None
        if self.workers == 1:
            _worker_init(root, factory, opts or {}, one_thread=False)
        else:
            self.ex = ProcessPoolExecutor(max_workers=self.workers, mp_context=mp.get_context("spawn"),
                                          initializer=_worker_init, initargs=(root, factory, opts or {}))

    def blocks(self, targets, kernels=("R",), chunk: int = 64):
        targets = np.asarray(targets)
        parts = [targets[k:k + chunk] for k in range(0, len(targets), chunk)]
        if self.ex is None:
            out = [_worker_blocks(p, kernels) for p in parts]
        else:
            out = list(self.ex.map(_worker_blocks, parts, [kernels] * len(parts)))
        return [b for part in out for b in part]

    def close(self):
        if self.ex is not None:
            self.ex.shutdown()
            self.ex = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def blocks_parallel(factory: tuple, root: str, targets, kernels=("R",), workers: int | None = None,
                    chunk: int = 64, opts: dict | None = None):
    """``OracleOperator.blocks`` for the targets, split over the worker processes of a ``BlockPool``."""
    with BlockPool(factory, root, workers, opts) as pool:
        return pool.blocks(targets, kernels, chunk)


def rows_from_blocks(orc: OracleOperator, blocks, targets, sigma: np.ndarray, kernel: str = "R") -> np.ndarray:
    """Rows of A sigma (kernel "R") or of K[sigma] before its mean is removed (kernel "K") from the
    targets' correction blocks, with the smooth-rule sums over all sources from the C oracle."""
    sigma = np.asarray(sigma, dtype=np.float64).reshape(orc.N, -1)
    targets = np.asarray(targets)
    q2 = orc.q * orc.q
    y = cfar.far_rows(orc, targets, sigma, kernel)
    for t, (plist, blk) in enumerate(blocks):
        for P, b in zip(plist, blk[kernel]):
            y[t] += b @ sigma[P * q2:(P + 1) * q2]
    if kernel == "R":
        y += sigma[targets] + (orc.w @ sigma)[None, :]
    return y


def rows(orc: OracleOperator, factory: tuple, root: str, targets, sigma: np.ndarray, kernel: str = "R",
         workers: int | None = None) -> np.ndarray:
    """``rows_from_blocks`` with the targets' blocks from a fresh worker pool.  Rows are
    independent, so this equals the same rows of the whole operator."""
    blocks = blocks_parallel(factory, root, targets, kernels=(kernel,), workers=workers, chunk=16)
    return rows_from_blocks(orc, blocks, targets, sigma, kernel)


def near_matrix(orc: OracleOperator, blocks, kernel: str = "R"):
    """Sparse N x N matrix holding every target's correction blocks at its near patches' columns."""
    import scipy.sparse as sp
    q2 = orc.q * orc.q
    rows, cols, vals = [], [], []
    for i, (plist, blk) in enumerate(blocks):
        for P, b in zip(plist, blk[kernel]):
            rows.append(np.full(q2, i, dtype=np.int64))
            cols.append(np.arange(P * q2, (P + 1) * q2, dtype=np.int64))
            vals.append(b)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(orc.N, orc.N))


class FullSystem:
    """A sigma, the solve and the representation over all N nodes of one problem."""

    def __init__(self, prob, factory: tuple, root: str, workers: int | None = None, kernels=("R",), log=None):
        self.orc = OracleOperator.from_problem(prob)
        self.N = self.orc.N
        self.log = log or (lambda *a: None)
        self.log(f"[oracle] near blocks of {self.N} targets ({', '.join(kernels)}) on {workers or os.cpu_count()} "
                 f"processes")
        blocks = blocks_parallel(factory, root, np.arange(self.N), kernels, workers)
        self.S = {k: near_matrix(self.orc, blocks, k) for k in kernels}

    def apply(self, sigma: np.ndarray) -> np.ndarray:
        sigma = np.asarray(sigma, dtype=np.float64).reshape(self.N, -1)
        far = cfar.far_rows(self.orc, np.arange(self.N), sigma, "R")
        return sigma + far + self.S["R"] @ sigma + (self.orc.w @ sigma)[None, :]

    def solve(self, f: np.ndarray, tol: float = 1e-13, max_iter: int = 300):
        """sigma (N, n_rhs) for f projected to mean zero; GMRES per column.  Also returns the
        recomputed relative residuals and iteration counts."""
        fz, _ = self.orc.project_mean_zero(f)
        cols, res, its = [], [], []
        for r in range(fz.shape[1]):
            x, rr, k = gmres(lambda v: self.apply(v)[:, 0], fz[:, r], tol=tol, max_iter=max_iter,
                             callback=lambda k, e: self.log(f"[oracle] gmres rhs {r} iter {k}: {e:.2e}"))
            cols.append(x)
            res.append(rr)
            its.append(k)
        return np.stack(cols, axis=1), res, its

    def represent(self, sigma: np.ndarray) -> np.ndarray:
        sigma = np.asarray(sigma, dtype=np.float64).reshape(self.N, -1)
        u = cfar.far_rows(self.orc, np.arange(self.N), sigma, "K") + self.S["K"] @ sigma
        return u - ((self.orc.w @ u) / self.orc.w.sum())[None, :]
