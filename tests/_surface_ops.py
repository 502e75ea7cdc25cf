"""Test helper: the surface operator div_G(a grad_G u) of nodal values on quad patches by spectral
differentiation (the Lagrange interpolant of the q x q Gauss-Legendre values of each patch, its
derivatives at the nodes), with the metric from the map's first derivatives:
    div_G(a grad_G u) = (1 / sqrt g) d_i (sqrt g a g^ij d_j u),  g_ij = x_i . x_j  (i, j in u, v).
Used to check Lemma lem:surf_term and Lemma lem:Dirichlet_surf_term: the operator applied to the edge
potentials K_gamma[mu] and N_gamma[mu] gives R_gamma[mu] and T_gamma[mu] away from the boundary."""
import numpy as np


def diff_matrix(t: np.ndarray) -> np.ndarray:
    """D[i, j] = l_j'(t_i) for the Lagrange basis on the nodes t (barycentric form)."""
    q = len(t)
    w = np.array([1.0 / np.prod([t[j] - t[k] for k in range(q) if k != j]) for j in range(q)])
    D = np.zeros((q, q))
    for i in range(q):
        for j in range(q):
            if i != j:
                D[i, j] = (w[j] / w[i]) / (t[i] - t[j])
        D[i, i] = -D[i].sum()
    return D


def surface_operator(u, a, xu, xv, q: int) -> np.ndarray:
    """div_G(a grad_G u) at the nodes of every whole patch in u (node order iu * q + iv per patch)."""
    t, _ = np.polynomial.legendre.leggauss(q)
    D = diff_matrix(t)
    out = np.empty_like(u)
    for p in range(u.shape[0] // (q * q)):
        s = slice(p * q * q, (p + 1) * q * q)
        U, A = u[s].reshape(q, q), a[s].reshape(q, q)
        Xu, Xv = xu[s].reshape(q, q, 3), xv[s].reshape(q, q, 3)
        E, F, G = (Xu * Xu).sum(-1), (Xu * Xv).sum(-1), (Xv * Xv).sum(-1)
        g = E * G - F * F
        sg = np.sqrt(g)
        Uu, Uv = D @ U, U @ D.T
        fu = sg * A * (G * Uu - F * Uv) / g
        fv = sg * A * (-F * Uu + E * Uv) / g
        out[s] = ((D @ fu + fv @ D.T) / sg).ravel()
    return out


def advection_term(u, b, xu, xv, q: int) -> np.ndarray:
    """b . grad_G u at the nodes (grad_G u = g^ij d_j u x_i, tangent; b ambient, so only its tangential
    part counts)."""
    t, _ = np.polynomial.legendre.leggauss(q)
    D = diff_matrix(t)
    out = np.empty_like(u)
    for p in range(u.shape[0] // (q * q)):
        s = slice(p * q * q, (p + 1) * q * q)
        U = u[s].reshape(q, q)
        Xu, Xv, B = xu[s].reshape(q, q, 3), xv[s].reshape(q, q, 3), b[s].reshape(q, q, 3)
        E, F, G = (Xu * Xu).sum(-1), (Xu * Xv).sum(-1), (Xv * Xv).sum(-1)
        g = E * G - F * F
        Uu, Uv = D @ U, U @ D.T
        cu = (G * Uu - F * Uv) / g          # contravariant components g^uj d_j u, g^vj d_j u
        cv = (-F * Uu + E * Uv) / g
        out[s] = ((B * Xu).sum(-1) * cu + (B * Xv).sum(-1) * cv).ravel()
    return out


def middle_row_nodes(n_u: int, n_v: int, q: int, cols=(0, 3, 6, 9)) -> np.ndarray:
    """Node indices of a few patches of the band's middle row of patches (farthest from its edges)."""
    row = n_u // 2
    return np.concatenate([np.arange((row * n_v + c) * q * q, (row * n_v + c + 1) * q * q) for c in cols])


def lagrange_at(t: np.ndarray, x: float) -> np.ndarray:
    """l_j(x) for the Lagrange basis on the nodes t."""
    q = len(t)
    return np.array([np.prod([(x - t[k]) / (t[j] - t[k]) for k in range(q) if k != j]) for j in range(q)])


def trig_eval(f: np.ndarray, tq: np.ndarray) -> np.ndarray:
    """The trigonometric interpolant of n equispaced samples f (t_j = 2 pi j / n) at the points tq (for even
    n the Nyquist coefficient split between +n/2 and -n/2)."""
    n = len(f)
    F = np.fft.fft(f) / n
    k = np.fft.fftfreq(n, d=1.0 / n)
    if n % 2 == 0:
        F = np.append(F, F[n // 2] / 2)
        F[n // 2] /= 2
        k = np.append(k, n // 2)
    return np.real(np.exp(1j * np.outer(tq, k)) @ F)


def conormal_derivative_at_edge(u, xu, xv, x, q: int, patches, n_v: int):
    """nu . grad_G u at the points u = +1 of the given patches (the edge of a band's last row), from the
    nodal values by the Lagrange interpolant in u (extrapolated to the edge) and in v; nu is the part of
    x_u normal to x_v, normalized.  Returns (values, poloidal parameters of the points, positions)."""
    t, _ = np.polynomial.legendre.leggauss(q)
    D = diff_matrix(t)
    l1 = lagrange_at(t, 1.0)
    dl1 = D.T @ l1                       # l_a'(1) = sum_i l_i(1) D[i, a]
    vals, ts, xs = [], [], []
    for ci, P in enumerate(patches):
        s = slice(ci * q * q, (ci + 1) * q * q)
        U = u[s].reshape(q, q)
        Xu, Xv, X = xu[s].reshape(q, q, 3), xv[s].reshape(q, q, 3), x[s].reshape(q, q, 3)
        Ue, Uu = l1 @ U, dl1 @ U
        Uv = D @ Ue
        Xu_e = np.einsum("a,avk->vk", l1, Xu)
        Xv_e = np.einsum("a,avk->vk", l1, Xv)
        E, F, G = (Xu_e * Xu_e).sum(-1), (Xu_e * Xv_e).sum(-1), (Xv_e * Xv_e).sum(-1)
        g = E * G - F * F
        grad = ((G * Uu - F * Uv) / g)[:, None] * Xu_e + ((-F * Uu + E * Uv) / g)[:, None] * Xv_e
        tau = Xv_e / np.linalg.norm(Xv_e, axis=1)[:, None]
        nu = Xu_e - (Xu_e * tau).sum(1)[:, None] * tau
        nu /= np.linalg.norm(nu, axis=1)[:, None]
        vals.append((grad * nu).sum(1))
        ts.append(2 * np.pi * ((P % n_v) + (t + 1) / 2) / n_v)
        xs.append(np.einsum("a,avk->vk", l1, X))
    return np.concatenate(vals), np.concatenate(ts), np.concatenate(xs)


def values_at_edge(u, q: int, patches, n_v: int):
    """u extrapolated to u = +1 of the given patches by the Lagrange interpolant in u (nodal values of
    whole patches, in patch order), and the poloidal parameters of those points."""
    t, _ = np.polynomial.legendre.leggauss(q)
    l1 = lagrange_at(t, 1.0)
    vals = [l1 @ u[ci * q * q:(ci + 1) * q * q].reshape(q, q) for ci in range(len(patches))]
    ts = [2 * np.pi * ((P % n_v) + (t + 1) / 2) / n_v for P in patches]
    return np.concatenate(vals), np.concatenate(ts)

