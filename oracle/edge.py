"""Edge operators of the open-surface problems (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU leg use this module.

Section 5 (the Neumann system eq:NeuBVPsystem, the Dirichlet system eq:DirBVPsystem and their
representations) applies four operators whose sources lie on the boundary gamma of an open surface
Gamma and whose targets x are points of Gamma:

    K_gamma[mu](x) = int_gamma K(x, x') mu(x') ds(x')                       (eq:BC_rep)
    N_gamma[mu](x) = int_gamma nu(x') . grad'_G K(x, x') mu(x') ds(x')       (eq:DirichletRep)
    R_gamma[mu](x) = int_gamma R(x, x') mu(x') ds(x')                       (Lemma lem:surf_term)
    T_gamma[mu](x) = int_gamma nu(x') . grad'_G R(x, x') mu(x') ds(x')       (Lemma lem:Dirichlet_surf_term)

nu(x') is the unit conormal of gamma: tangent to Gamma, normal to gamma, pointing out of Gamma.  The
primed gradient acts on the source point x', which enters both through r = x - x' and through the
coefficient a(x') of the parametrix K(x, x') = G(|x - x'|; a(x')).  Since nu is tangent to Gamma, the
surface gradient along nu equals the ambient one, so nu . grad'_G a = nu . grad a for any extension of a.

Only c = 0 is taken here (K = log r / (2 pi a(x')), the Laplace-Beltrami type and its variable-a
generalization, as in the paper's boundary-value tests).

Two edge-to-edge operators of the systems' boundary rows are here too, with targets on gamma, smooth
kernels and the trapezoid rule on the samples: K'_gamma, the conormal derivative at the target
(``kprime_gamma``), and D_gamma, the double layer (``dlayer_gamma``, for nu . grad a = 0 on gamma).

Discretization (Section 6.1.4, edge quadrature): each boundary curve has a smooth periodic
parameterization gamma(t), t in [0, 2 pi), sampled at n equispaced t.  Every sampled quantity (the
position, dgamma/dt, the across-curve direction d, a, grad a and mu) is Fourier-interpolated to m n
equispaced points, and the trapezoid rule with weights (2 pi / (m n)) |dgamma/dt| runs on those fine
points.  The interpolation is the trigonometric interpolant of the samples: the discrete Fourier
transform zero-padded to m n coefficients, for even n with the Nyquist coefficient split evenly
between the frequencies +n/2 and -n/2 (so the interpolant of real samples is real).
"""
from __future__ import annotations

import numpy as np

from .kernels import parametrix, remainder

KINDS = ("K", "N", "R", "T")


def fourier_upsample(f: np.ndarray, m: int) -> np.ndarray:
    """Trigonometric interpolant of the n samples f[j] = f(2 pi j / n) (axis 0), evaluated at the m n
    points 2 pi k / (m n): FFT, zero padding, inverse FFT (library routines)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    if m == 1:
        return f.copy()
    F = np.fft.fft(f, axis=0)
    G = np.zeros((m * n,) + f.shape[1:], dtype=np.complex128)
    h = (n + 1) // 2                    # frequencies 0 .. h-1 and -(h-1) .. -1 (odd n: all of them)
    G[:h] = F[:h]
    if h > 1:
        G[m * n - (h - 1):] = F[n - (h - 1):]
    if n % 2 == 0:                      # the Nyquist coefficient, split between +n/2 and -n/2
        G[n // 2] = F[n // 2] / 2
        G[m * n - n // 2] = F[n // 2] / 2
    return (np.fft.ifft(G, axis=0) * m).real


def conormal(xt: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Unit conormal: the part of d normal to the curve's tangent dgamma/dt, normalized (d is tangent
    to the surface and points out of it, so the result is tangent to the surface, normal to the
    curve and outward)."""
    tau = xt / np.linalg.norm(xt, axis=-1, keepdims=True)
    v = d - np.sum(d * tau, axis=-1, keepdims=True) * tau
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def edge_points(edge, m: int) -> dict:
    """Fine quadrature points of all curves: position y, conormal nu, weight w, coefficient a and
    nu . grad a, curve after curve (m n_k points for a curve of n_k samples)."""
    out = {k: [] for k in ("y", "nu", "w", "a", "nu_ga")}
    off = np.asarray(edge.offsets)
    for k in range(len(off) - 1):
        s = slice(int(off[k]), int(off[k + 1]))
        n = off[k + 1] - off[k]
        y = fourier_upsample(edge.x[s], m)
        xt = fourier_upsample(edge.xt[s], m)
        d = fourier_upsample(edge.d[s], m)
        a = fourier_upsample(edge.a[s], m)
        ga = fourier_upsample(edge.grad_a[s], m)
        nu = conormal(xt, d)
        out["y"].append(y)
        out["nu"].append(nu)
        out["w"].append(2 * np.pi / (m * n) * np.linalg.norm(xt, axis=1))
        out["a"].append(a)
        out["nu_ga"].append(np.sum(nu * ga, axis=1))
    return {k: np.concatenate(v) for k, v in out.items()}


def upsample_density(mu: np.ndarray, offsets, m: int) -> np.ndarray:
    """mu (M, n_rhs) on the samples -> its interpolant on the fine points, curve by curve."""
    off = np.asarray(offsets)
    return np.concatenate([fourier_upsample(mu[int(off[k]):int(off[k + 1])], m) for k in range(len(off) - 1)])


def n_kernel(x, y, nu, a_s, nu_ga_s):
    """nu(x') . grad' K(x, x') for K = log|x - x'| / (2 pi a(x')): the derivative of log|x - x'| along
    nu is -(nu . r) / r^2 (r = x - x'), and that of 1 / a(x') is -(nu . grad a) / a^2."""
    r = x - y
    r2 = np.sum(r * r, axis=-1)
    K = np.log(np.sqrt(r2)) / (2 * np.pi * a_s)
    return -np.sum(nu * r, axis=-1) / (2 * np.pi * a_s * r2) - K * nu_ga_s / a_s


def t_kernel(x, n, H, a_t, gs_t, y, nu, a_s, nu_ga_s):
    """nu(x') . grad' R(x, x') for c = 0.  With r = x - x' the remainder (eq:explicit_remainder, with
    G' = 1 / (2 pi a' r) and G'' = -1 / (2 pi a' r^2)) is R = P(r) / a(x') where
        P(r) = (1 / 2 pi) [ gs . r / r^2 + 2 a (n.r)^2 / r^4 - 2 a H (n.r) / r^2 ]
    depends on the source through r only.  Since dr/dx' = -I,
        nu . grad' R = -(nu . grad_r P) / a' - R (nu . grad a') / a',
        2 pi nu . grad_r P = gs.nu / r^2 - 2 (gs.r)(nu.r) / r^4 + 4 a (n.r)(n.nu) / r^4
                             - 8 a (n.r)^2 (nu.r) / r^6 - 2 a H (n.nu) / r^2 + 4 a H (n.r)(nu.r) / r^4."""
    r = x - y
    r2 = np.sum(r * r, axis=-1)
    nr = np.sum(n * r, axis=-1)
    vr = np.sum(nu * r, axis=-1)
    gr = np.sum(gs_t * r, axis=-1)
    gv = np.sum(gs_t * nu, axis=-1)
    nv = np.sum(n * nu, axis=-1)
    dP = (gv / r2 - 2 * gr * vr / r2 ** 2 + 4 * a_t * nr * nv / r2 ** 2 - 8 * a_t * nr ** 2 * vr / r2 ** 3
          - 2 * a_t * H * nv / r2 + 4 * a_t * H * nr * vr / r2 ** 2) / (2 * np.pi)
    R = remainder(x, n, H, a_t, gs_t, y, a_s)
    return -dP / a_s - R * nu_ga_s / a_s


def edge_kernel(kind: str, tgt: dict, i, pts: dict, p=slice(None)):
    """Kernel values of one operator for targets i (index array) against fine points p: (len(i), P).
    tgt: x, n, H, a, gs (node arrays of the surface); pts: from ``edge_points``."""
    x = tgt["x"][i][:, None, :]
    y, nu = pts["y"][p][None], pts["nu"][p][None]
    a_s, nu_ga = pts["a"][p][None], pts["nu_ga"][p][None]
    if kind == "K":
        return parametrix(x, y, a_s)
    if kind == "N":
        return n_kernel(x, y, nu, a_s, nu_ga)
    n, H, a_t, gs = tgt["n"][i][:, None, :], tgt["H"][i][:, None], tgt["a"][i][:, None], tgt["gs"][i][:, None, :]
    if kind == "R":
        return remainder(x, n, H, a_t, gs, y, a_s)
    if kind == "T":
        return t_kernel(x, n, H, a_t, gs, y, nu, a_s, nu_ga)
    raise ValueError(f"unknown edge operator {kind!r}")


def edge_apply(kind: str, tgt: dict, edge, mu: np.ndarray, m: int, targets=None, chunk: int = 256) -> np.ndarray:
    """The operator ``kind`` (K, N, R or T) applied to mu (M, n_rhs) on the samples of ``edge``, at
    the surface nodes ``targets`` (all when None): the trapezoid sum over the m-fold Fourier
    oversampled curves.  Returns (len(targets), n_rhs)."""
    pts = edge_points(edge, m)
    muf = upsample_density(np.asarray(mu, dtype=np.float64).reshape(edge.x.shape[0], -1), edge.offsets, m)
    wm = pts["w"][:, None] * muf
    idx = np.arange(tgt["x"].shape[0]) if targets is None else np.asarray(targets)
    out = np.empty((len(idx), wm.shape[1]))
    for s in range(0, len(idx), chunk):
        i = idx[s:s + chunk]
        out[s:s + chunk] = edge_kernel(kind, tgt, i, pts) @ wm
    return out


def fourier_derivative(f: np.ndarray) -> np.ndarray:
    """d/dt of the trigonometric interpolant of the n samples f[j] = f(2 pi j / n) (axis 0), at the
    samples: FFT, multiplication by i k, inverse FFT (for even n the Nyquist mode, split evenly, has a
    derivative that vanishes at the samples)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    k = np.fft.fftfreq(n, d=1.0 / n)
    if n % 2 == 0:
        k[n // 2] = 0.0
    shape = (n,) + (1,) * (f.ndim - 1)
    return np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=0), axis=0).real


def kprime_gamma(edge, mu: np.ndarray) -> np.ndarray:
    """K'_gamma[mu] at the samples of every curve (Theorem thm:NeumannBCsrep, eq:neumann):
        K'_gamma[mu](x) = int_gamma nu(x) . grad_G K(x, x') mu(x') ds(x'),   x in gamma,
    the conormal derivative at the target of K = log|x - x'| / (2 pi a(x')), i.e.
    nu(x) . (x - x') / (2 pi a(x') |x - x'|^2).  The kernel is smooth (Theorem thm:kern_smth), so the
    trapezoid rule runs on the samples themselves (weights (2 pi / n) |dgamma/dt|).  At x' = x it takes
    its limit: with x' = gamma(t + h), nu . (x - x') = -(nu . gamma'') h^2 / 2 + O(h^3) and
    |x - x'|^2 = |gamma'|^2 h^2 + O(h^3), so the kernel tends to -(nu . gamma'') / (4 pi a |gamma'|^2);
    gamma'' is the derivative of the interpolant of the sampled dgamma/dt.  Returns (M, n_rhs)."""
    off = np.asarray(edge.offsets)
    mu = np.asarray(mu, dtype=np.float64).reshape(edge.x.shape[0], -1)
    nu = conormal(edge.xt, edge.d)
    w = np.empty(edge.x.shape[0])
    lim = np.empty(edge.x.shape[0])
    for k in range(len(off) - 1):
        s = slice(int(off[k]), int(off[k + 1]))
        n = off[k + 1] - off[k]
        xtt = fourier_derivative(edge.xt[s])
        L2 = np.sum(edge.xt[s] ** 2, axis=1)
        w[s] = 2 * np.pi / n * np.sqrt(L2)
        lim[s] = -np.sum(nu[s] * xtt, axis=1) / (4 * np.pi * edge.a[s] * L2)
    r = edge.x[:, None, :] - edge.x[None, :, :]
    r2 = np.sum(r * r, axis=-1)
    np.fill_diagonal(r2, 1.0)
    Kp = np.sum(nu[:, None, :] * r, axis=-1) / (2 * np.pi * edge.a[None, :] * r2)
    np.fill_diagonal(Kp, lim)
    return Kp @ (w[:, None] * mu)


def dlayer_gamma(edge, mu: np.ndarray) -> np.ndarray:
    """D_gamma[mu] at the samples of every curve: the limit on gamma of N_gamma[mu] less its jump,
        D_gamma[mu](x) = int_gamma nu(x') . grad' K(x, x') mu(x') ds(x'),   x in gamma,
    the source-conormal (double-layer) kernel nu(x') . (x' - x) / (2 pi a(x') |x - x'|^2) when
    nu . grad a = 0 along gamma (otherwise the kernel has a log|x - x'| term, not taken here: ValueError).
    The kernel is smooth, so the trapezoid rule runs on the samples; at x' = x it takes its limit: with
    x' = gamma(t + h), nu(x') . (x' - x) = -(nu . gamma'') h^2 / 2 + O(h^3), the same limit as K'_gamma,
    -(nu . gamma'') / (4 pi a |gamma'|^2).  Returns (M, n_rhs)."""
    nu = conormal(edge.xt, edge.d)
    nga = np.sum(nu * edge.grad_a, axis=1)
    if np.abs(nga).max() > 1e-14 * np.abs(edge.grad_a).max(initial=1.0):
        raise ValueError("the on-curve double layer is taken for nu . grad a = 0 along the curve only")
    off = np.asarray(edge.offsets)
    mu = np.asarray(mu, dtype=np.float64).reshape(edge.x.shape[0], -1)
    w = np.empty(edge.x.shape[0])
    lim = np.empty(edge.x.shape[0])
    for k in range(len(off) - 1):
        s = slice(int(off[k]), int(off[k + 1]))
        n = off[k + 1] - off[k]
        xtt = fourier_derivative(edge.xt[s])
        L2 = np.sum(edge.xt[s] ** 2, axis=1)
        w[s] = 2 * np.pi / n * np.sqrt(L2)
        lim[s] = -np.sum(nu[s] * xtt, axis=1) / (4 * np.pi * edge.a[s] * L2)
    r = edge.x[None, :, :] - edge.x[:, None, :]          # x' - x (source j, target i)
    r2 = np.sum(r * r, axis=-1)
    np.fill_diagonal(r2, 1.0)
    Dk = np.sum(nu[None, :, :] * r, axis=-1) / (2 * np.pi * edge.a[None, :] * r2)
    np.fill_diagonal(Dk, lim)
    return Dk @ (w[:, None] * mu)


def edge_abs_sum(kind: str, tgt: dict, edge, m: int, targets=None, chunk: int = 256) -> np.ndarray:
    """sum_p |k(x_i, y_p)| w_p over the fine points for each target: the scale of the rounding error of
    the trapezoid sum (used for tolerances, not part of the operator)."""
    pts = edge_points(edge, m)
    idx = np.arange(tgt["x"].shape[0]) if targets is None else np.asarray(targets)
    out = np.empty(len(idx))
    for s in range(0, len(idx), chunk):
        i = idx[s:s + chunk]
        out[s:s + chunk] = np.abs(edge_kernel(kind, tgt, i, pts)) @ pts["w"]
    return out


def targets_of(orc) -> dict:
    """Target node arrays of an OracleOperator."""
    return {"x": orc.x, "n": orc.n, "H": orc.H, "a": orc.a, "gs": orc.gs}
