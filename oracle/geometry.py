"""Node geometry, patch centroids/radii and near lists (oracle, FP64).

Surface calculus of Section 2.2: metric g from the parameter derivatives, unit
normal n, mean curvature H = (1/2) div_G n with n outward, so that H = +1 on the
unit sphere.  Nystrom weights of Section 6.1: w = w_a w_b sqrt(det g) with
tensor Gauss-Legendre weights on the reference square.  Near criterion of
Section 6.1.2: a target is near a patch when it is within 1.5 patch radii of
the patch centroid, where the centroid is the mean of the patch corners and
the radius the largest centroid-corner distance.
"""
from __future__ import annotations

import numpy as np


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1] (library routine)."""
    return np.polynomial.legendre.leggauss(n)


def lagrange_basis(nodes: np.ndarray, t: np.ndarray) -> np.ndarray:
    """l_j(t) for the interpolating polynomial through ``nodes``: (len(t), len(nodes)).

    Product form prod_{k != j} (t - t_k) / (t_j - t_k); no division by t - t_j.
    """
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    q = len(nodes)
    num = t[:, None, None] - nodes[None, None, :]          # (K, 1, q): t - t_k
    den = nodes[:, None] - nodes[None, :]                  # (q, q):    t_j - t_k
    off = ~np.eye(q, dtype=bool)
    fac = np.where(off[None], num / np.where(off, den, 1.0)[None], 1.0)   # (K, q_j, q_k)
    return fac.prod(axis=2)


def node_geometry(x, xu, xv, xuu, xuv, xvv, q: int):
    """Per-node normal, area element J = sqrt(det g), weight w and mean curvature H."""
    cr = np.cross(xu, xv)
    J = np.linalg.norm(cr, axis=1)
    n = cr / J[:, None]
    E = np.einsum("ij,ij->i", xu, xu)
    Fm = np.einsum("ij,ij->i", xu, xv)
    G = np.einsum("ij,ij->i", xv, xv)
    e = np.einsum("ij,ij->i", xuu, n)
    f = np.einsum("ij,ij->i", xuv, n)
    g = np.einsum("ij,ij->i", xvv, n)
    # (1/2) div_G n for the outward normal: minus half the trace of the shape operator.
    H = -(e * G - 2 * f * Fm + g * E) / (2 * (E * G - Fm * Fm))
    _, wgl = gauss_legendre(q)
    wq = np.outer(wgl, wgl).ravel()                     # node order iu*q + iv
    n_patches = x.shape[0] // (q * q)
    w = np.tile(wq, n_patches) * J
    return {"n": n, "J": J, "w": w, "H": H}


def surface_gradient(grad_a: np.ndarray, n: np.ndarray) -> np.ndarray:
    """Tangential part (I - n n^T) grad a of an ambient gradient."""
    return grad_a - n * np.einsum("ij,ij->i", grad_a, n)[:, None]


def patch_nodes(arr: np.ndarray, q: int) -> np.ndarray:
    """(N, c) node array -> (M, q, q, c) indexed [patch, iu, iv]."""
    return arr.reshape(-1, q, q, arr.shape[-1])


def interpolate_patch(Xp: np.ndarray, tnodes: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Tensor Lagrange interpolant of node data Xp (q, q, c) at points (u, v): (K, c)."""
    return tensor_interp(lagrange_basis(tnodes, u), lagrange_basis(tnodes, v), Xp)


def tensor_interp(Lu: np.ndarray, Lv: np.ndarray, Xp: np.ndarray) -> np.ndarray:
    """sum_ab Lu[k, a] Lv[k, b] Xp[a, b, c] for every point k: (K, c)."""
    q, _, c = Xp.shape
    T = (Lu @ Xp.reshape(q, q * c)).reshape(-1, q, c)     # sum over a
    return np.einsum("kbc,kb->kc", T, Lv)


def patch_corners(x: np.ndarray, q: int) -> np.ndarray:
    """Images of the four corners (-1,-1), (1,-1), (1,1), (-1,1) of every patch: (M, 4, 3)."""
    t, _ = gauss_legendre(q)
    X = patch_nodes(x, q)
    cu = np.array([-1.0, 1.0, 1.0, -1.0])
    cv = np.array([-1.0, -1.0, 1.0, 1.0])
    Lu = lagrange_basis(t, cu)
    Lv = lagrange_basis(t, cv)
    return np.einsum("ka,kb,mabc->mkc", Lu, Lv, X)


def centroid_radius(corners: np.ndarray):
    """Centroid (mean of corners) and radius (largest centroid-corner distance)."""
    c = corners.mean(axis=-2)
    rad = np.linalg.norm(corners - c[..., None, :], axis=-1).max(axis=-1)
    return c, rad


def near_lists(x_targets: np.ndarray, target_ids: np.ndarray, q: int, centroids: np.ndarray,
               radii: np.ndarray, eta: float = 1.5):
    """For each target: sorted patch ids P with |x - c_P| < eta * rho_P, plus its own patch."""
    out = []
    for xi, i in zip(x_targets, target_ids):
        d = np.linalg.norm(centroids - xi, axis=1)
        near = set(np.nonzero(d < eta * radii)[0].tolist())
        near.add(int(i) // (q * q))
        out.append(np.array(sorted(near), dtype=np.int64))
    return out
