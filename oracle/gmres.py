"""GMRES for the oracle's Nystrom system when dense LU is out of reach (oracle, FP64).

TEST INFRASTRUCTURE ONLY.  The paper solves its discretized integral equation with GMRES
(Section 6 and Section 7).  This is the textbook method (Saad and Schultz): from x_0 = 0 the
Arnoldi process builds an orthonormal basis of the Krylov space of A and f, orthogonalizing each
new vector against the basis with classical Gram-Schmidt applied twice (CGS2); the iterate
minimizes the residual norm over that space, found from the small Hessenberg least-squares
problem with a library least-squares routine.  No restarts; one right-hand side at a time.
Pinned in ``tests/test_oracle_large.py`` against dense LU (``numpy.linalg.solve``) on small
surfaces.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, f: np.ndarray, tol: float = 1e-13, max_iter: int = 300, callback=None):
    """x with ||f - A x||_2 <= tol ||f||_2 (or max_iter reached).  Returns (x, relative residual
    of the final iterate recomputed from a fresh apply, iterations)."""
    f = np.asarray(f, dtype=np.float64).ravel()
    beta = np.linalg.norm(f)
    if beta == 0.0:
        return np.zeros_like(f), 0.0, 0
    V = [f / beta]
    H = np.zeros((max_iter + 1, max_iter))
    k = 0
    y = np.zeros(0)
    for k in range(1, max_iter + 1):
        w = matvec(V[-1])
        Vm = np.stack(V, axis=1)
        h = Vm.T @ w                       # classical Gram-Schmidt ...
        w = w - Vm @ h
        h2 = Vm.T @ w                      # ... applied twice
        w = w - Vm @ h2
        H[:k, k - 1] = h + h2
        H[k, k - 1] = np.linalg.norm(w)
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
        est = np.linalg.norm(H[:k + 1, :k] @ y - e1) / beta
        if callback is not None:
            callback(k, est)
        if est <= tol or H[k, k - 1] == 0.0:
            break
        V.append(w / H[k, k - 1])
    x = np.stack(V[:k], axis=1) @ y
    res = np.linalg.norm(f - matvec(x)) / beta
    return x, float(res), k
