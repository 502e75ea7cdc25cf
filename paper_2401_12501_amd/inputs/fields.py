"""Seeded coefficient fields a(x) > 0 with ambient gradients, and right-hand sides.

Pure input data: each field is a smooth closed-form function of the ambient
position, evaluated at the nodes together with its ambient gradient (by
reverse-mode differentiation).  The library and the oracle project the gradient
onto the tangent plane themselves and remove the weighted mean of f
themselves; none of that happens here.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .surfaces import real_sph_harm_cartesian

__all__ = [
    "eval_field", "a_const", "a_sphere_cfg", "a_exp_xy", "a_seed_field", "a_tanh_sin", "a_linear_z", "c_exp_x",
    "solid_harmonic_rhs", "harmonic_basis_lm",
]


def eval_field(fn, x: np.ndarray):
    """Evaluate a torch field fn(X) -> (N,) at x (N, 3); return (values, ambient gradient)."""
    X = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    val = fn(X)
    (grad,) = torch.autograd.grad(val.sum(), X)
    return val.detach().numpy().copy(), grad.detach().numpy().copy()


def a_const(a0: float = 1.0):
    return lambda X: a0 + 0.0 * X[:, 0]


def a_sphere_cfg(X):
    """a(x) = 1 + 0.5 sin(2 x1) cos(x2)."""
    return 1.0 + 0.5 * torch.sin(2 * X[:, 0]) * torch.cos(X[:, 1])


def a_exp_xy(X):
    """a(x) = exp(0.3 x1 x2)."""
    return torch.exp(0.3 * X[:, 0] * X[:, 1])


def a_tanh_sin(X):
    """a(x) = 1 + 0.5 tanh(sin(3 x1))."""
    return 1.0 + 0.5 * torch.tanh(torch.sin(3 * X[:, 0]))


def a_linear_z(X):
    """a(x) = 2 + x3: linear in z, a factor of three over the unit sphere."""
    return 2.0 + X[:, 2]


def c_exp_x(X):
    """c(x) = -4 - exp(x1 / 2) (negative everywhere: the modified Helmholtz type)."""
    return -4.0 - torch.exp(0.5 * X[:, 0])


def c_pos_y(X):
    """c(x) = 2 (1 + 0.2 x2) (positive on the unit sphere and the test ellipsoids: the Helmholtz
    type).  The real part of the form c0 (1 + 0.2 y + 0.2 i sin x) of the variable-coefficient
    experiment, with c0 = 2 so that c stays between the first two eigenvalue bands of
    -div_G(a grad_G) for a = 2 + x3 on the unit sphere (about 0 and 4)."""
    return 2.0 * (1.0 + 0.2 * X[:, 1])


def b_rotation_z(x: np.ndarray, omega: float) -> np.ndarray:
    """Advection field omega e3 x x = omega (-x2, x1, 0): the rotation about the x3 axis, tangent
    to every surface of revolution about that axis (so b . grad u = omega du/dphi there)."""
    x = np.asarray(x, dtype=np.float64)
    return omega * np.stack([-x[:, 1], x[:, 0], np.zeros(len(x))], axis=1)


def b_swirl(x: np.ndarray) -> np.ndarray:
    """A smooth ambient field, not tangent to any of the surfaces here (the operator uses its
    tangential part): (0.6 - x2, x1 + 0.4 x3, 0.5 x1 x2)."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([0.6 - x[:, 1], x[:, 0] + 0.4 * x[:, 2], 0.5 * x[:, 0] * x[:, 1]], axis=1)


def a_seed_field(seed: int, n_modes: int = 8):
    """Smooth field with values in [0.5, 2]: a = 2^tanh(s), s = sum_k alpha_k cos(w_k . x + phi_k).

    alpha_k ~ U(-1, 1), w_k ~ N(0, 2^2 I_3), phi_k ~ U(0, 2 pi), all from ``seed``.
    """
    rng = np.random.default_rng(seed)
    alpha = torch.tensor(rng.uniform(-1, 1, n_modes))
    omega = torch.tensor(rng.normal(0.0, 2.0, (n_modes, 3)))
    phase = torch.tensor(rng.uniform(0, 2 * math.pi, n_modes))

    def fn(X):
        s = (alpha[None, :] * torch.cos(X @ omega.T + phase[None, :])).sum(dim=1)
        return torch.pow(2.0, torch.tanh(s))

    return fn


def harmonic_basis_lm(n_terms: int = 20):
    """The first ``n_terms`` real (l, m) pairs with l >= 1, in (l, m) order."""
    out = []
    l = 1
    while len(out) < n_terms:
        for m in range(-l, l + 1):
            out.append((l, m))
            if len(out) == n_terms:
                break
        l += 1
    return out


def solid_harmonic_rhs(x: np.ndarray, seed: int, n_terms: int = 20) -> np.ndarray:
    """f(x) = sum_k c_k |x|^l Y_lm(x/|x|) over the first 20 (l, m), c_k ~ N(0, 1) from ``seed``."""
    rng = np.random.default_rng(seed)
    c = rng.normal(0.0, 1.0, n_terms)
    X = torch.tensor(x, dtype=torch.float64)
    f = torch.zeros(X.shape[0], dtype=torch.float64)
    for ck, (l, m) in zip(c, harmonic_basis_lm(n_terms)):
        f = f + float(ck) * real_sph_harm_cartesian(l, m, X, homogeneous=True)
    return f.numpy().copy()
