"""ctypes binding of libpmx.so (the C ABI declared in include/pmx.h).

Argument marshalling only: every step of the method runs in the HIP library.
The module-level functions carry the C names; ``Context``, ``Surface`` and
``Operator`` are small owning wrappers.  Host arrays are numpy float64; device
arrays are torch CUDA tensors (their memory and the current stream are handed
to the library as plain pointers).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmx.so")

PMX_OK, PMX_PENDING = 0, 1
PMX_ERR_INVALID, PMX_ERR_OOM, PMX_ERR_TOO_LARGE, PMX_ERR_NOT_CONVERGED = -1, -2, -3, -4
PMX_ERR_ORIENTATION, PMX_ERR_DEVICE, PMX_ERR_CANCELLED = -5, -6, -7
PMX_MEM_HOST, PMX_MEM_DEVICE = 0, 1
PMX_PREC_FP64_DIRECT, PMX_PREC_MIXED_FMM, PMX_PREC_FP32_DIRECT = 0, 1, 2

_ERRNAMES = {-1: "INVALID", -2: "OOM", -3: "TOO_LARGE", -4: "NOT_CONVERGED", -5: "ORIENTATION", -6: "DEVICE",
             -7: "CANCELLED"}


class PmxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pmx error {code} ({_ERRNAMES.get(code, '?')}): {msg}")
        self.code = code


class pmx_options(C.Structure):
    _fields_ = [("eta_near", C.c_double), ("n_gl", C.c_int), ("fmm_order", C.c_int), ("fmm_leaf", C.c_int),
                ("gmres_tol", C.c_double), ("gmres_restart", C.c_int), ("max_iter", C.c_int),
                ("ir_tol", C.c_double), ("inner_tol", C.c_double), ("max_ir", C.c_int), ("precision", C.c_int),
                ("overlap", C.c_int)]


class pmx_info(C.Structure):
    _fields_ = [("iters_total", C.c_int), ("ir_steps", C.c_int), ("applies_fp64", C.c_int),
                ("applies_low", C.c_int), ("rel_residual", C.c_double), ("removed_mean", C.c_double),
                ("t_setup", C.c_double), ("t_solve", C.c_double)]


class pmx_operator_stats(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_patches", C.c_int64), ("q", C.c_int32), ("fmm_levels", C.c_int32),
                ("near_pairs", C.c_int64), ("fmm_boxes", C.c_int64), ("fmm_m2l_pairs", C.c_int64),
                ("fmm_p2p_pairs", C.c_int64), ("device_bytes", C.c_uint64)]


_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_SIGS = {
    "pmx_ctx_create": (C.c_int32, [C.c_int, C.c_uint64, C.POINTER(_vp)]),
    "pmx_ctx_destroy": (None, [_vp]),
    "pmx_last_error": (C.c_char_p, []),
    "pmx_default_options": (None, [C.POINTER(pmx_options)]),
    "pmx_surface_create": (C.c_int32, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int, _vp,
                                        C.POINTER(_vp)]),
    "pmx_surface_destroy": (None, [_vp]),
    "pmx_operator_create": (C.c_int32, [_vp, _vp, _vp, C.POINTER(pmx_options), C.c_int, _vp, C.POINTER(_vp)]),
    "pmx_operator_create_c": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, C.POINTER(pmx_options), C.c_int, _vp,
                                          C.POINTER(_vp)]),
    "pmx_operator_destroy": (None, [_vp]),
    "pmx_operator_get_stats": (C.c_int32, [_vp, C.POINTER(pmx_operator_stats)]),
    "pmx_apply": (C.c_int32, [_vp, C.c_int, C.c_int, _vp, _vp, C.c_int, _vp]),
    "pmx_apply_noalloc": (C.c_int32, [_vp, C.c_int, _vp, _vp, _vp]),
    "pmx_solve": (C.c_int32, [_vp, C.POINTER(pmx_options), C.c_int, _vp, _vp, C.c_int, _vp, C.c_int, _vp,
                              C.POINTER(pmx_info)]),
    "pmx_represent": (C.c_int32, [_vp, C.c_int, _vp, _vp, C.c_int, _vp]),
    "pmx_operator_export_geometry": (C.c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "pmx_operator_export_near": (C.c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "pmx_operator_export_near_imag": (C.c_int32, [_vp, _vp, _vp]),
    "pmx_operator_is_complex": (C.c_int32, [_vp, C.POINTER(C.c_int)]),
    "pmx_server_create": (C.c_int32, [_vp, C.POINTER(pmx_options), C.c_int, C.POINTER(_vp)]),
    "pmx_server_submit": (C.c_int32, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int,
                                      C.POINTER(C.c_uint64)]),
    "pmx_server_step": (C.c_int32, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "pmx_server_poll": (C.c_int32, [_vp, C.c_uint64, _vp, _vp, C.POINTER(pmx_info), _vp]),
    "pmx_server_cancel": (C.c_int32, [_vp, C.c_uint64]),
    "pmx_server_destroy": (None, [_vp]),
    "pmx_server_get_stats": (C.c_int32, [_vp] + [C.POINTER(C.c_uint64)] * 5),
    "pmx_profile_enable": (C.c_int32, [_vp, C.c_int]),
    "pmx_edge_create": (C.c_int32, [_vp, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, _vp,
                                    C.POINTER(_vp)]),
    "pmx_edge_destroy": (None, [_vp]),
    "pmx_edge_size": (C.c_int32, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "pmx_edge_export_points": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "pmx_edge_apply": (C.c_int32, [_vp, _vp, C.c_int, C.c_int, _vp, _vp, C.c_int, _vp]),
    "pmx_edge_apply_kprime": (C.c_int32, [_vp, C.c_int, _vp, _vp, C.c_int, _vp]),
    "pmx_edge_apply_dlayer": (C.c_int32, [_vp, C.c_int, _vp, _vp, C.c_int, _vp]),
    "pmx_profile_read": (C.c_int32, [_vp, _vp, _vp]),
}

PHASES = ["prep", "direct64", "direct32", "near", "fmm_p2m", "fmm_m2m", "fmm_m2l", "fmm_l2l", "fmm_l2p",
          "fmm_p2p", "log", "fmm_m2l_sum", "edge"]

_lib = None


def lib():
    """Load libpmx.so (raises if it has not been built: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2401_12501_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code not in (PMX_OK, PMX_PENDING):
        raise PmxError(code, lib().pmx_last_error().decode())
    return code


# ------------------------------------------------------------------ C names
def pmx_default_options() -> pmx_options:
    o = pmx_options()
    lib().pmx_default_options(C.byref(o))
    return o


def pmx_last_error() -> str:
    return lib().pmx_last_error().decode()


def pmx_ctx_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = _vp()
    _check(lib().pmx_ctx_create(device, hbm_budget_bytes, C.byref(h)))
    return h


def pmx_ctx_destroy(h):
    lib().pmx_ctx_destroy(h)


# ------------------------------------------------------------------ array marshalling
def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _stream_ptr(arrs):
    import torch
    for a in arrs:
        if _is_torch(a) and a.is_cuda:
            return torch.cuda.current_stream(a.device).cuda_stream
    return None


def _host(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _marshal(*arrs):
    """(pointers, mem_kind, stream, keepalive) for numpy (host) or torch CUDA (device) arrays."""
    dev = [_is_torch(a) and a.is_cuda for a in arrs if a is not None]
    if any(dev) and not all(dev):
        raise ValueError("mix of host and device arrays")
    kind = PMX_MEM_DEVICE if dev and all(dev) else PMX_MEM_HOST
    ptrs, keep = [], []
    for a in arrs:
        if a is None:
            ptrs.append(None)
            continue
        if kind == PMX_MEM_DEVICE:
            import torch
            if a.dtype != torch.float64 or not a.is_contiguous():
                raise ValueError("device arrays must be contiguous float64 tensors")
            ptrs.append(a.data_ptr())
        else:
            if _is_torch(a):
                a = a.detach().cpu().numpy()
            a = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(a)
            ptrs.append(a.ctypes.data)
    stream = _stream_ptr(arrs) if kind == PMX_MEM_DEVICE else None
    return ptrs, kind, stream, keep


class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.h = pmx_ctx_create(device, hbm_budget_bytes)

    def close(self):
        if self.h:
            pmx_ctx_destroy(self.h)
            self.h = None

    __del__ = close


class Surface:
    """pmx_surface_create: node positions and parameter derivatives (N x 3 each)."""

    def __init__(self, ctx: Context, n_patches: int, q: int, x, xu, xv, xuu, xuv, xvv):
        self.ctx = ctx
        self.n_patches, self.q = n_patches, q
        self.N = n_patches * q * q
        ptrs, kind, stream, keep = _marshal(x, xu, xv, xuu, xuv, xvv)
        h = _vp()
        _check(lib().pmx_surface_create(ctx.h, n_patches, q, *ptrs, kind, stream, C.byref(h)))
        self.h = h

    @classmethod
    def from_inputs(cls, ctx, s):
        return cls(ctx, s.n_patches, s.q, s.x, s.xu, s.xv, s.xuu, s.xuv, s.xvv)

    def close(self):
        if getattr(self, "h", None):
            lib().pmx_surface_destroy(self.h)
            self.h = None

    __del__ = close


class Operator:
    """pmx_operator_create and the calls on an operator."""

    def __init__(self, surface: Surface, a, grad_a, opts: pmx_options | None = None, c=None, b=None):
        """pmx_operator_create, or pmx_operator_create_c when c (N values of one sign) is given,
        with the advection field b ((N, 3) ambient vectors) or without (b None).  With c > 0 the
        operator is complex: apply, solve and represent take and return complex arrays (n_rhs, N),
        passed to the library as 2N reals per vector (real parts, then imaginary parts)."""
        self.surface = surface
        self.N = surface.N
        self.q = surface.q
        self.opts = opts if opts is not None else pmx_default_options()
        ptrs, kind, stream, keep = _marshal(a, grad_a, c, b)
        h = _vp()
        if c is None:
            if b is not None:
                raise PmxError(PMX_ERR_INVALID, "an advection field b needs c != 0 (pmx_operator_create_c)")
            _check(lib().pmx_operator_create(surface.h, ptrs[0], ptrs[1], C.byref(self.opts), kind, stream,
                                             C.byref(h)))
        else:
            _check(lib().pmx_operator_create_c(surface.h, ptrs[0], ptrs[1], ptrs[2], ptrs[3], C.byref(self.opts),
                                               kind, stream, C.byref(h)))
        self.h = h
        flag = C.c_int(0)
        _check(lib().pmx_operator_is_complex(h, C.byref(flag)))
        self.complex = bool(flag.value)

    def close(self):
        if getattr(self, "h", None):
            lib().pmx_operator_destroy(self.h)
            self.h = None

    __del__ = close

    def stats(self) -> pmx_operator_stats:
        s = pmx_operator_stats()
        _check(lib().pmx_operator_get_stats(self.h, C.byref(s)))
        return s

    def _rhs(self, a):
        n_rhs = (a.numel() if _is_torch(a) else np.size(a)) // self.N
        if n_rhs * self.N != (a.numel() if _is_torch(a) else np.size(a)):
            raise ValueError("array size is not a multiple of N")
        return n_rhs

    def _planar(self, a):
        """A complex operator's layout: complex (n, N) values as real (n, 2, N), real parts first."""
        if a is None:
            return None
        if _is_torch(a):
            import torch
            a = a.reshape(-1, self.N)
            if not a.is_complex():
                a = a.to(torch.complex128)
            return torch.stack([a.real, a.imag], dim=1).contiguous()
        a = np.asarray(a).reshape(-1, self.N).astype(np.complex128)
        return np.ascontiguousarray(np.stack([a.real, a.imag], axis=1))

    @staticmethod
    def _unplanar(p):
        if p is None:
            return None
        if _is_torch(p):
            import torch
            return torch.complex(p[:, 0].contiguous(), p[:, 1].contiguous())
        return p[:, 0] + 1j * p[:, 1]

    def apply(self, sigma, precision: int = PMX_PREC_FP64_DIRECT, out=None):
        """y = A sigma; sigma is (n_rhs, N) (host numpy or device tensor; complex for a complex operator)."""
        if self.complex:
            sp = self._planar(sigma)
            y = np.empty(sp.shape) if not _is_torch(sp) else sp.new_empty(sp.shape)
            ptrs, kind, stream, keep = _marshal(sp, y)
            _check(lib().pmx_apply(self.h, precision, sp.shape[0], ptrs[0], ptrs[1], kind, stream))
            return self._unplanar(y)
        n_rhs = self._rhs(sigma)
        if out is None:
            out = np.empty((n_rhs, self.N)) if not _is_torch(sigma) else sigma.new_empty(sigma.shape)
        ptrs, kind, stream, keep = _marshal(sigma, out)
        _check(lib().pmx_apply(self.h, precision, n_rhs, ptrs[0], ptrs[1], kind, stream))
        return out

    def apply_planar(self, sp, precision: int = PMX_PREC_FP64_DIRECT, out=None):
        """pmx_apply on a complex operator in the library's own layout: sp is (n_rhs, 2, N) float64
        (real parts, then imaginary parts), out likewise; nothing is converted."""
        if out is None:
            out = np.empty(sp.shape) if not _is_torch(sp) else sp.new_empty(sp.shape)
        ptrs, kind, stream, keep = _marshal(sp, out)
        _check(lib().pmx_apply(self.h, precision, sp.shape[0], ptrs[0], ptrs[1], kind, stream))
        return out

    def apply_noalloc(self, sigma, out=None, check: bool = True):
        """pmx_apply_noalloc: y = A sigma (FP64 direct far field) with the library's static scratch;
        sigma and out are device tensors of shape (n_rhs, N), or for a complex operator float64 tensors
        of shape (n_rhs, 2, N) in the library's layout (real parts, then imaginary parts: nothing is
        converted, so nothing is allocated).  Returns out (check=True) or the status."""
        n_rhs = sigma.shape[0] if self.complex else self._rhs(sigma)
        if out is None:
            out = sigma.new_empty(sigma.shape)
        ptrs, kind, stream, keep = _marshal(sigma, out)
        code = lib().pmx_apply_noalloc(self.h, n_rhs, ptrs[0], ptrs[1], stream)
        if not check:
            return code
        _check(code)
        return out

    def solve(self, f, opts: pmx_options | None = None, sigma0=None, want_u: bool = False, check: bool = True):
        """(sigma, u or None, [pmx_info]) for f of shape (n_rhs, N) (complex results for a complex operator)."""
        if self.complex:
            fp = self._planar(f)
            sig, u, infos = self._solve_real(fp, fp.shape[0], opts, self._planar(sigma0), want_u, check)
            return self._unplanar(sig), self._unplanar(u), infos
        return self._solve_real(f, self._rhs(f), opts, sigma0, want_u, check)

    def _solve_real(self, f, n_rhs, opts, sigma0, want_u, check):
        torch_in = _is_torch(f)
        shape = np.shape(f) if np.ndim(f) == 3 else (n_rhs, self.N)   # 3-d: a complex operator's (n, 2, N)
        mk = (lambda: f.new_empty(f.shape)) if torch_in else (lambda: np.empty(shape))
        sigma = mk() if sigma0 is None else (sigma0.clone() if torch_in else np.array(sigma0, dtype=np.float64))
        u = mk() if want_u else None
        ptrs, kind, stream, keep = _marshal(f, sigma, u)
        if kind == PMX_MEM_HOST:        # outputs must be the arrays the library writes
            sigma, u = keep[1], (keep[2] if want_u else None)
        infos = (pmx_info * n_rhs)()
        code = lib().pmx_solve(self.h, C.byref(opts) if opts is not None else None, n_rhs, ptrs[0], ptrs[1],
                               1 if sigma0 is not None else 0, ptrs[2], kind, stream, infos)
        if check:
            _check(code)
        return sigma, u, list(infos)

    def represent(self, sigma, out=None):
        if self.complex:
            sp = self._planar(sigma)
            u = np.empty(sp.shape) if not _is_torch(sp) else sp.new_empty(sp.shape)
            ptrs, kind, stream, keep = _marshal(sp, u)
            _check(lib().pmx_represent(self.h, sp.shape[0], ptrs[0], ptrs[1], kind, stream))
            return self._unplanar(u)
        n_rhs = self._rhs(sigma)
        if out is None:
            out = np.empty((n_rhs, self.N)) if not _is_torch(sigma) else sigma.new_empty(sigma.shape)
        ptrs, kind, stream, keep = _marshal(sigma, out)
        _check(lib().pmx_represent(self.h, n_rhs, ptrs[0], ptrs[1], kind, stream))
        return out

    def profile(self, enable: bool = True):
        _check(lib().pmx_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{phase: (total ms, launches)} since the last read."""
        ms = np.zeros(len(PHASES))
        cnt = np.zeros(len(PHASES), dtype=np.int64)
        _check(lib().pmx_profile_read(self.h, ms.ctypes.data, cnt.ctypes.data))
        return {p: (float(m), int(c)) for p, m, c in zip(PHASES, ms, cnt)}

    def export_geometry(self):
        N = self.N
        n, H, w, gs = np.empty((N, 3)), np.empty(N), np.empty(N), np.empty((N, 3))
        _check(lib().pmx_operator_export_geometry(self.h, n.ctypes.data, H.ctypes.data, w.ctypes.data,
                                                   gs.ctypes.data))
        return {"n": n, "H": H, "w": w, "gs": gs}

    def export_near(self, with_D: bool = False):
        st = self.stats()
        N, nnz, q2 = self.N, st.near_pairs, self.q * self.q
        ptr = np.empty(N + 1, dtype=np.int64)
        patch = np.empty(nnz, dtype=np.int32)
        Cb = np.empty((nnz, q2))
        Db = np.empty((nnz, q2)) if with_D else None
        _check(lib().pmx_operator_export_near(self.h, ptr.ctypes.data, patch.ctypes.data, Cb.ctypes.data,
                                               Db.ctypes.data if with_D else None))
        return ptr, patch, Cb, Db

    def export_near_imag(self, with_D: bool = False):
        """Imaginary parts of the blocks C (and D) of a complex operator, in export_near's layout."""
        nnz, q2 = self.stats().near_pairs, self.q * self.q
        Ci = np.empty((nnz, q2))
        Di = np.empty((nnz, q2)) if with_D else None
        _check(lib().pmx_operator_export_near_imag(self.h, Ci.ctypes.data, Di.ctypes.data if with_D else None))
        return Ci, Di


EDGE_KINDS = {"K": 0, "N": 1, "R": 2, "T": 3}   # PMX_EDGE_K, _N, _R, _T


class Edge:
    """pmx_edge_create: boundary curves of an open surface, sampled at equispaced parameter values,
    Fourier-oversampled ``oversample`` times for the edge quadrature.  ``counts`` gives the samples of
    each curve (stored curve after curve); x, xt, d, grad_a are (M, 3), a is (M,)."""

    def __init__(self, ctx: Context, counts, x, xt, d, a, grad_a, oversample: int = 1):
        self.ctx = ctx
        cnt = np.ascontiguousarray(counts, dtype=np.int64)
        self.counts = cnt
        ptrs, kind, stream, keep = _marshal(x, xt, d, a, grad_a)
        h = _vp()
        _check(lib().pmx_edge_create(ctx.h, len(cnt), cnt.ctypes.data, *ptrs, int(oversample), kind, stream,
                                     C.byref(h)))
        self.h = h
        m, f = C.c_int64(0), C.c_int64(0)
        _check(lib().pmx_edge_size(h, C.byref(m), C.byref(f)))
        self.M, self.n_fine = m.value, f.value

    @classmethod
    def from_inputs(cls, ctx, edge, oversample: int = 1):
        """From an ``inputs.EdgeSamples``."""
        return cls(ctx, np.diff(edge.offsets), edge.x, edge.xt, edge.d, edge.a, edge.grad_a, oversample)

    def close(self):
        if getattr(self, "h", None):
            lib().pmx_edge_destroy(self.h)
            self.h = None

    __del__ = close

    def _n_rhs(self, mu) -> int:
        size = mu.numel() if _is_torch(mu) else np.size(mu)
        if size == 0 or size % self.M:
            raise ValueError(f"mu must hold n_rhs rows of {self.M} values (got {size})")
        return size // self.M

    @staticmethod
    def _check_out(out, size: int):
        got = out.numel() if _is_torch(out) else np.size(out)
        if got != size:
            raise ValueError(f"out must hold {size} values (got {got})")

    def points(self) -> dict:
        """pmx_edge_export_points: the fine quadrature points (y, nu, w, a, nu . grad a)."""
        F = self.n_fine
        out = {"y": np.empty((F, 3)), "nu": np.empty((F, 3)), "w": np.empty(F), "a": np.empty(F),
               "nu_ga": np.empty(F)}
        _check(lib().pmx_edge_export_points(self.h, *(out[k].ctypes.data for k in ("y", "nu", "w", "a", "nu_ga"))))
        return out

    def apply(self, op: "Operator", kind: str, mu, out=None):
        """pmx_edge_apply: the edge operator ``kind`` (K, N, R or T) of mu (n_rhs, M) at the operator's
        nodes, (n_rhs, N); numpy arrays (host) or float64 CUDA tensors (device)."""
        n_rhs = self._n_rhs(mu)
        if out is None:
            out = np.empty((n_rhs, op.N)) if not _is_torch(mu) else mu.new_empty((n_rhs, op.N))
        self._check_out(out, n_rhs * op.N)
        ptrs, kind_mem, stream, keep = _marshal(mu, out)
        _check(lib().pmx_edge_apply(op.h, self.h, EDGE_KINDS[kind], n_rhs, ptrs[0], ptrs[1], kind_mem, stream))
        return out

    def kprime(self, mu, out=None):
        """pmx_edge_apply_kprime: K'_gamma of mu (n_rhs, M) at the samples, (n_rhs, M)."""
        n_rhs = self._n_rhs(mu)
        if out is None:
            out = np.empty((n_rhs, self.M)) if not _is_torch(mu) else mu.new_empty((n_rhs, self.M))
        self._check_out(out, n_rhs * self.M)
        ptrs, kind_mem, stream, keep = _marshal(mu, out)
        _check(lib().pmx_edge_apply_kprime(self.h, n_rhs, ptrs[0], ptrs[1], kind_mem, stream))
        return out

    def dlayer(self, mu, out=None):
        """pmx_edge_apply_dlayer: D_gamma of mu (n_rhs, M) at the samples, (n_rhs, M)."""
        n_rhs = self._n_rhs(mu)
        if out is None:
            out = np.empty((n_rhs, self.M)) if not _is_torch(mu) else mu.new_empty((n_rhs, self.M))
        self._check_out(out, n_rhs * self.M)
        ptrs, kind_mem, stream, keep = _marshal(mu, out)
        _check(lib().pmx_edge_apply_dlayer(self.h, n_rhs, ptrs[0], ptrs[1], kind_mem, stream))
        return out


class Server:
    """pmx_server_*: continuous-batching solve server (host arrays, copied on submit)."""

    def __init__(self, ctx: Context, opts: pmx_options | None = None, max_active: int = 4):
        self.ctx = ctx
        h = _vp()
        _check(lib().pmx_server_create(ctx.h, C.byref(opts) if opts is not None else None, max_active, C.byref(h)))
        self.h = h
        self.n = {}

    def close(self):
        if getattr(self, "h", None):
            lib().pmx_server_destroy(self.h)
            self.h = None

    __del__ = close

    def submit(self, surface, a, grad_a, f, want_u: bool = False) -> int:
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in
                (surface.x, surface.xu, surface.xv, surface.xuu, surface.xuv, surface.xvv, a, grad_a, f)]
        t = C.c_uint64()
        _check(lib().pmx_server_submit(self.h, surface.n_patches, surface.q, *[v.ctypes.data for v in arrs],
                                       1 if want_u else 0, C.byref(t)))
        self.n[t.value] = (surface.n, want_u)
        return t.value

    def step(self):
        na, nq = C.c_int(), C.c_int()
        _check(lib().pmx_server_step(self.h, C.byref(na), C.byref(nq)))
        return na.value, nq.value

    def poll(self, ticket: int):
        """None while pending; else (status, sigma, u, info, times)."""
        N, want_u = self.n[ticket]
        sig = np.empty(N)
        u = np.empty(N) if want_u else None
        info = pmx_info()
        times = np.zeros(3)
        code = lib().pmx_server_poll(self.h, ticket, sig.ctypes.data, u.ctypes.data if want_u else None,
                                     C.byref(info), times.ctypes.data)
        if code == PMX_PENDING:
            return None
        del self.n[ticket]
        return code, sig, u, info, times

    def cancel(self, ticket: int):
        _check(lib().pmx_server_cancel(self.h, ticket))

    def stats(self) -> dict:
        """Counters: shared launches of the apply path, applies carried, largest batch, requests held
        back for memory, largest estimated footprint admitted at once (bytes)."""
        v = [C.c_uint64() for _ in range(5)]
        _check(lib().pmx_server_get_stats(self.h, *[C.byref(x) for x in v]))
        return dict(zip(("batches", "applies", "max_batch", "held_for_memory", "peak_reserved_bytes"),
                        (x.value for x in v)))
