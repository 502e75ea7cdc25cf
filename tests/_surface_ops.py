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
