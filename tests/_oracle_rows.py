"""Oracle rows of the operator at full workload sizes, and the choice of rows to sample.

Rows of the discrete operator are independent, so large applies and solutions are checked on
samples: near/self correction blocks of the sampled targets from the oracle in worker processes,
smooth-rule sums over all sources from the oracle's C sums on every host core.
"""
from __future__ import annotations

import os

import numpy as np

from oracle.system import rows

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INPUTS = "paper_2401_12501_amd.inputs"


def workers() -> int:
    return max(1, min(8, os.cpu_count() or 1))   # the test process plus these stay well under 16 GPU-visible processes


def apply_rows(orc, factory: tuple, targets, sigma: np.ndarray, kernel: str = "R") -> np.ndarray:
    """Oracle rows (``oracle.system.rows``); factory = (function name in the inputs module, kwargs)
    of orc's problem."""
    fn, kw = factory
    return rows(orc, (INPUTS, fn, kw), ROOT, targets, sigma, kernel, workers())


def stratified_targets(n_nodes: int, q: int, ptr: np.ndarray, n: int = 1024, seed: int = 0) -> np.ndarray:
    """At least n distinct rows (sorted): the first and last node of seeded patches, the targets with the most
    near patches (ptr: CSR offsets of the near lists), the first and last nodes overall, and seeded
    random nodes for the rest."""
    rng = np.random.default_rng(seed)
    q2 = q * q
    M = n_nodes // q2
    pick = set([0, n_nodes - 1])
    patches = rng.choice(M, size=min(M, n // 8), replace=False)
    pick.update((patches * q2).tolist())
    pick.update((patches * q2 + q2 - 1).tolist())
    counts = np.diff(ptr)
    pick.update(np.argsort(-counts, kind="stable")[: n // 8].tolist())
    while len(pick) < n:
        pick.update(rng.choice(n_nodes, size=n - len(pick), replace=False).tolist())
    return np.array(sorted(pick))
