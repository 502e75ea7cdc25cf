"""The discrete remainder operator, its solve and the representation (oracle, FP64).

Nystrom system (Section 6.1, eq:IEsum with the quadrature regimes of Sections
6.1.1-6.1.3), for every node i:

  (A sigma)_i = sigma_i
              + sum_{j != i} w_j R(x_i, x_j) sigma_j                      (smooth rule)
              + sum_{P in near(i)} sum_{j in P} C_{i,P,j} sigma_j          (near / self correction)
              + sum_j w_j sigma_j                                          (rank-one term)

with C_{i,P,j} = W_{i,P,j} - [j != i] w_j R(x_i, x_j) and
W_{i,P,j} = int_P R(x_i, y) l_j(y) dA(y) by the self rule (i in P) or the
near rule.  Off-node values on a patch (position, parameter derivatives, a)
are tensor Lagrange interpolants of the node data, as the paper interpolates
sigma to the quadrature grid (Remark in Section 6.1.1 and Section 6.1.2).

The rank-one term is Section 3's "adding the term int_G sigma", taken
unscaled.  The representation u = K[sigma] (eq:representation) uses the same
rules with the parametrix, then the weighted mean is removed so that u is the
mean-zero solution.

With c != 0 (c < 0 at every node, the modified Helmholtz type, or c > 0 at every node, the
Helmholtz type with its complex kernel) the problem has no null space: the system is sigma + R[sigma] = f (Theorem thm:second_kind), f is taken as
given and u = K[sigma] is not shifted.  R and K then carry the c-dependent Green's
function (``kernels``), c is interpolated on a patch like a, and the self rule integrates R
on dyadically graded radial panels, since R then has r^m log r parts.

With c > 0 the blocks, the matrix, sigma and u are complex (numpy complex128); real data f
gives a complex sigma whose u = K[sigma] is real up to the discretization error.

An advection field b (eq:surf_PDE's first-order term, Section 4's theorem
thm:advectionparametrix) is taken with c != 0 only: the remainder becomes R_b of
eq:adv_remainder, the system sigma + R_b[sigma] = f (eq:IE_adv) and u = K[sigma] as before.
b is given as ambient vectors at the nodes and projected onto each node's tangent plane.
With c = 0 constants still solve the homogeneous problem but the data's solvability
condition is no longer a zero mean, which the paper does not treat.
"""
from __future__ import annotations

import numpy as np

from .geometry import (gauss_legendre, lagrange_basis, tensor_interp, node_geometry, surface_gradient, patch_nodes,
                       patch_corners, centroid_radius, near_lists)
from .kernels import remainder, parametrix
from .rules import self_rule, near_rule


class OracleOperator:
    """Plain FP64 discretization of eq:IE on a quad-patch surface."""

    def __init__(self, q, x, xu, xv, xuu, xuv, xvv, a, grad_a, eta: float = 1.5, n_gl: int = 16,
                 split: float = 2.0, c=None, b=None):
        self.q = q
        self.N = x.shape[0]
        self.M = self.N // (q * q)
        self.x, self.xu, self.xv = x, xu, xv
        self.a = np.asarray(a, dtype=np.float64)
        geo = node_geometry(x, xu, xv, xuu, xuv, xvv, q)
        self.n, self.J, self.w, self.H = geo["n"], geo["J"], geo["w"], geo["H"]
        self.gs = surface_gradient(np.asarray(grad_a, dtype=np.float64), self.n)
        self.eta, self.n_gl, self.split = eta, n_gl, split
        self.tnodes, _ = gauss_legendre(q)
        self.corners = patch_corners(x, q)
        self.centroids, self.radii = centroid_radius(self.corners)
        self._P_x = patch_nodes(x, q)
        self._P_xu = patch_nodes(xu, q)
        self._P_xv = patch_nodes(xv, q)
        self._P_a = patch_nodes(self.a[:, None], q)
        self.c = None if c is None else np.asarray(c, dtype=np.float64)
        if self.c is not None and not (np.all(self.c < 0) or np.all(self.c > 0)):
            raise ValueError("c must be negative at every node or positive at every node (or None for c = 0)")
        self.complex = self.c is not None and bool(self.c[0] > 0)
        self.dtype = np.complex128 if self.complex else np.float64
        self._P_c = None if self.c is None else patch_nodes(self.c[:, None], q)
        self.b = None
        if b is not None:
            if self.c is None:
                raise ValueError("an advection field b needs c != 0")
            b = np.asarray(b, dtype=np.float64).reshape(self.N, 3)
            self.b = b - np.sum(b * self.n, axis=1)[:, None] * self.n
        self._self_cache = {}

    @classmethod
    def from_problem(cls, prob, **kw):
        s = prob.surface
        if getattr(prob, "c", None) is not None and "c" not in kw:
            kw["c"] = prob.c
        if getattr(prob, "b", None) is not None and "b" not in kw:
            kw["b"] = prob.b
        return cls(s.q, s.x, s.xu, s.xv, s.xuu, s.xuv, s.xvv, prob.a, prob.grad_a, **kw)

    def _c(self, idx):
        return None if self.c is None else self.c[idx]

    def _b(self, idx):
        return None if self.b is None else self.b[idx]

    # ----------------------------------------------------------------- kernels at nodes
    def R_row(self, i: int, js) -> np.ndarray:
        """R(x_i, x_j) for node indices js (all must differ from i)."""
        return remainder(self.x[i], self.n[i], self.H[i], self.a[i], self.gs[i], self.x[js], self.a[js],
                         self._c(i), self._c(js), self._b(i))

    def K_row(self, i: int, js) -> np.ndarray:
        return parametrix(self.x[i], self.x[js], self.a[js], self._c(js))

    # ----------------------------------------------------------------- near lists
    def near(self, targets) -> list:
        targets = np.asarray(targets)
        return near_lists(self.x[targets], targets, self.q, self.centroids, self.radii, self.eta)

    # ----------------------------------------------------------------- local rules
    def rule_points(self, i: int, P: int, radial: str = "plain"):
        """Parameter-plane rule for target node i over patch P (self or near)."""
        q = self.q
        if i // (q * q) == P:
            loc = i % (q * q)
            key = (loc // q, loc % q, radial)
            if key not in self._self_cache:
                self._self_cache[key] = self_rule(self.tnodes[key[0]], self.tnodes[key[1]], self.n_gl, self.split,
                                                  radial)
            return self._self_cache[key]
        return near_rule(self.x[i], self._P_x[P], self.tnodes, self.n_gl, self.eta)

    def pair_weights(self, i: int, P: int, kernels=("R",)) -> dict:
        """W_{i,P,j} for j in P (q*q values, node order) for each kernel in "R", "K", "one"."""
        q = self.q
        if i // (q * q) == P and len(kernels) > 1:
            out = {}
            for k in kernels:
                out.update(self.pair_weights(i, P, (k,)))
            return out
        radial = "log" if kernels == ("K",) else ("dyadic" if self.c is not None else "plain")
        u, v, wq = self.rule_points(i, P, radial)
        Lu = lagrange_basis(self.tnodes, u)
        Lv = lagrange_basis(self.tnodes, v)
        interp = lambda Xp: tensor_interp(Lu, Lv, Xp)
        y = interp(self._P_x[P])
        Jt = np.linalg.norm(np.cross(interp(self._P_xu[P]), interp(self._P_xv[P])), axis=1)
        a_s = interp(self._P_a[P])[:, 0]
        c_s = None if self.c is None else interp(self._P_c[P])[:, 0]
        out = {}
        for kernel in kernels:
            if kernel == "R":
                F = remainder(self.x[i], self.n[i], self.H[i], self.a[i], self.gs[i], y, a_s, self._c(i), c_s,
                              self._b(i))
            elif kernel == "K":
                F = parametrix(self.x[i], y, a_s, c_s)
            elif kernel == "one":
                F = np.ones_like(a_s)
            else:
                raise ValueError(kernel)
            c = wq * F * Jt
            out[kernel] = (Lu.T @ (c[:, None] * Lv)).ravel()
        return out

    def correction_blocks(self, i: int, P: int, kernels=("R",)) -> dict:
        """C_{i,P,:} = W_{i,P,:} - [j != i] w_j F(x_i, x_j) for F = R (and D for F = K)."""
        W = self.pair_weights(i, P, kernels)
        q2 = self.q * self.q
        js = np.arange(P * q2, (P + 1) * q2)
        mask = js != i
        for kernel in kernels:
            smooth = self.R_row(i, js[mask]) if kernel == "R" else self.K_row(i, js[mask])
            W[kernel][mask] -= self.w[js[mask]] * smooth
        return W

    def blocks(self, targets, kernels=("R",)):
        """Near lists and correction blocks for the given targets.

        Returns a list (one entry per target) of (patch ids, {kernel: blocks[n_near, q*q]}).
        """
        out = []
        for i, plist in zip(targets, self.near(targets)):
            per = [self.correction_blocks(int(i), int(P), kernels) for P in plist]
            out.append((plist, {k: np.stack([b[k] for b in per]) for k in kernels}))
        return out

    # ----------------------------------------------------------------- apply
    def far_rows(self, targets, sigma: np.ndarray, kernel: str = "R") -> np.ndarray:
        """sum_{j != i} w_j F(x_i, x_j) sigma_j for the given targets; sigma (N, n_rhs)."""
        sigma = sigma.reshape(self.N, -1)
        out = np.zeros((len(targets), sigma.shape[1]), dtype=np.result_type(self.dtype, sigma.dtype))
        alls = np.arange(self.N)
        for t, i in enumerate(targets):
            js = alls[alls != i]
            row = self.R_row(i, js) if kernel == "R" else self.K_row(i, js)
            out[t] = (self.w[js] * row) @ sigma[js]
        return out

    def apply_rows(self, targets, sigma: np.ndarray, blocks=None) -> np.ndarray:
        """(A sigma)_i for the given targets (rows are independent)."""
        sigma = sigma.reshape(self.N, -1)
        targets = np.asarray(targets)
        if blocks is None:
            blocks = self.blocks(targets)
        q2 = self.q * self.q
        y = sigma[targets] + self.far_rows(targets, sigma)
        if self.c is None:
            y += (self.w @ sigma)[None, :]
        for t, (plist, C) in enumerate(blocks):
            for P, Cb in zip(plist, C["R"]):
                y[t] += Cb @ sigma[P * q2:(P + 1) * q2]
        return y

    def dense_matrix(self, blocks=None) -> np.ndarray:
        """The full N x N Nystrom matrix (small N only)."""
        N, q2 = self.N, self.q * self.q
        if blocks is None:
            blocks = self.blocks(np.arange(N))
        A = np.zeros((N, N), dtype=self.dtype)
        for i in range(N):
            js = np.arange(N)
            js = js[js != i]
            A[i, js] = self.w[js] * self.R_row(i, js)
        A += np.eye(N)
        if self.c is None:
            A += self.w[None, :]
        for i, (plist, C) in zip(range(N), blocks):
            for P, Cb in zip(plist, C["R"]):
                A[i, P * q2:(P + 1) * q2] += Cb
        return A

    def apply(self, sigma: np.ndarray, A: np.ndarray | None = None) -> np.ndarray:
        if A is None:
            return self.apply_rows(np.arange(self.N), sigma)
        return A @ sigma.reshape(self.N, -1)

    # ----------------------------------------------------------------- solve
    def project_mean_zero(self, f: np.ndarray):
        """f - (sum w f)/(sum w): the c = 0 problem needs mean-zero data (Section 2.3).
        With c != 0 f is used as given (mean reported as 0)."""
        f = f.reshape(self.N, -1)
        if self.c is not None:
            return f.copy(), np.zeros(f.shape[1])
        mean = (self.w @ f) / self.w.sum()
        return f - mean[None, :], mean

    def solve(self, f: np.ndarray, A: np.ndarray | None = None) -> np.ndarray:
        """sigma with A sigma = f (f projected to mean zero first); dense LU (library routine)."""
        if A is None:
            A = self.dense_matrix()
        fz, _ = self.project_mean_zero(f)
        return np.linalg.solve(A, fz)

    # ----------------------------------------------------------------- representation
    def represent_rows(self, targets, sigma: np.ndarray, blocks=None) -> np.ndarray:
        """K[sigma] at the given targets, before the mean is removed."""
        sigma = sigma.reshape(self.N, -1)
        targets = np.asarray(targets)
        if blocks is None:
            blocks = self.blocks(targets, kernels=("K",))
        q2 = self.q * self.q
        u = self.far_rows(targets, sigma, kernel="K")
        for t, (plist, D) in enumerate(blocks):
            for P, Db in zip(plist, D["K"]):
                u[t] += Db @ sigma[P * q2:(P + 1) * q2]
        return u

    def represent(self, sigma: np.ndarray, blocks=None) -> np.ndarray:
        """u = K[sigma] with the same rules, then minus its weighted mean."""
        sigma = sigma.reshape(self.N, -1)
        targets = np.arange(self.N)
        if blocks is None:
            blocks = self.blocks(targets, kernels=("K",))
        q2 = self.q * self.q
        u = self.far_rows(targets, sigma, kernel="K")
        for t, (plist, D) in enumerate(blocks):
            for P, Db in zip(plist, D["K"]):
                u[t] += Db @ sigma[P * q2:(P + 1) * q2]
        if self.c is None:
            u -= ((self.w @ u) / self.w.sum())[None, :]
        return u
