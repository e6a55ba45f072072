"""ctypes binding of libphmg.so (the C ABI in include/phmg.h).

Argument marshalling only: host arrays are passed as pointers to
``phmg_hierarchy_create``; device vectors are torch float64 CUDA tensors whose
``data_ptr()`` is handed to the library, and the library's stream is torch's
current stream.  Every step of the solve runs in the library's HIP kernels;
there is no fallback: if the library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphmg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2407_07253_amd.build` "
                      "(or __graft_entry__.build()); there is no CPU fallback")

_lib = C.CDLL(LIB_PATH)

PHMG_OK, PHMG_EINVAL, PHMG_ENOMEM, PHMG_ESINGULAR, PHMG_ENOCONV, PHMG_EHIP, PHMG_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ESINGULAR", -4: "ENOCONV", -5: "EHIP", -6: "ESTATE"}
PREC = {"f64": 0, "f32": 1, "bf16": 2}
KERNELS = {"patch_apply": 0, "scatter": 1, "spmv": 2, "extract": 3, "factor": 4}
MAX_PATCH = 1024


class PhmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"phmg {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class CsrT(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class PatchesT(C.Structure):
    _fields_ = [("npatch", C.c_int32), ("ptr", C.c_void_p), ("dofs", C.c_void_p), ("weight", C.c_void_p)]


class OptsT(C.Structure):
    _fields_ = [("nu_p", C.c_int32), ("nu_h", C.c_int32), ("n_v", C.c_int32), ("n_plevels", C.c_int32),
                ("omega", C.c_double), ("smoother", C.c_int32), ("eig_iters", C.c_int32),
                ("cheb_lo", C.c_double), ("cheb_hi", C.c_double)]


SMOOTHERS = {"richardson": 0, "chebyshev": 1}


class DescT(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("K", C.POINTER(CsrT)), ("P", C.POINTER(CsrT)),
                ("patches", C.POINTER(PatchesT)), ("coarse_null", C.c_void_p)]


class LevelInfoT(C.Structure):
    _fields_ = [("n", C.c_int32), ("npatch", C.c_int32), ("max_m", C.c_int32), ("precision", C.c_int32),
                ("nnz", C.c_int64), ("sum_m", C.c_int64), ("sum_m2", C.c_int64), ("lambda_max", C.c_double),
                ("apply_variant", C.c_int32), ("apply_variants", C.c_int32),
                ("symmetric_storage", C.c_int32), ("spmv_variant", C.c_int32), ("stored_elements", C.c_int64),
                ("block_variant", C.c_int32), ("block_variants", C.c_int32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_create = _sig("phmg_hierarchy_create", C.c_int, [C.POINTER(DescT), C.POINTER(OptsT), C.c_void_p, C.POINTER(C.c_void_p)])
_destroy = _sig("phmg_hierarchy_destroy", C.c_int, [C.c_void_p])
_setup = _sig("phmg_relax_setup", C.c_int, [C.c_void_p, C.c_int])
_set_prec = _sig("phmg_set_precision", C.c_int, [C.c_void_p, C.c_int, C.c_int])
_apply = _sig("phmg_relax_apply", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int])
_apply_na = _sig("phmg_relax_apply_noalloc", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int])
_vcycle = _sig("phmg_vcycle", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p])
_fgmres = _sig("phmg_fgmres_solve", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_int,
                                              C.POINTER(C.c_int), C.POINTER(C.c_double)])
_residual = _sig("phmg_residual", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p])
_set_kernel = _sig("phmg_set_kernel_vector", C.c_int, [C.c_void_p, C.c_void_p])
_project = _sig("phmg_project_kernel", C.c_int, [C.c_void_p, C.c_int, C.c_void_p])
_info = _sig("phmg_get_level_info", C.c_int, [C.c_void_p, C.c_int, C.POINTER(LevelInfoT)])
_prof_on = _sig("phmg_profile_enable", C.c_int, [C.c_void_p, C.c_uint])
_prof_read = _sig("phmg_profile_read", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)])
_prof_reset = _sig("phmg_profile_reset", C.c_int, [C.c_void_p])
_last_error = _sig("phmg_last_error", C.c_char_p, [])
_ritz = _sig("phmg_ritz_max_real", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double)])
_graphs = _sig("phmg_set_graphs", C.c_int, [C.c_void_p, C.c_int])
_apply_b = _sig("phmg_relax_apply_batched", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int])
_vcycle_b = _sig("phmg_vcycle_batched", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p])
_FGMRES_B_ARGS = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int32),
                  C.POINTER(C.c_double)]
_fgmres_b = _sig("phmg_fgmres_solve_batched", C.c_int, _FGMRES_B_ARGS)
_fgmres_bt = _sig("phmg_fgmres_solve_batched_transposed", C.c_int, _FGMRES_B_ARGS)
_vcycle_bt = _sig("phmg_vcycle_batched_transposed", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p])
_apply_t = _sig("phmg_relax_apply_transposed", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int])
_vcycle_t = _sig("phmg_vcycle_transposed", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p])
_fgmres_t = _sig("phmg_fgmres_solve_transposed", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                                           C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)])
_set_sens = _sig("phmg_set_sensitivities", C.c_int, [C.c_void_p, C.POINTER(CsrT), C.POINTER(CsrT)])
_forcing_rhs = _sig("phmg_forcing_rhs", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p])
_gradients = _sig("phmg_gradients", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p])
_fbf_create = _sig("phmg_fbf_create", C.c_int, [C.c_void_p, C.POINTER(CsrT), C.POINTER(CsrT), C.POINTER(CsrT),
                                                 C.POINTER(C.c_void_p)])
_fbf_apply = _sig("phmg_fbf_apply", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p])
_fbf_fgmres = _sig("phmg_fbf_fgmres_solve", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                                      C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)])
_fbf_destroy = _sig("phmg_fbf_destroy", C.c_int, [C.c_void_p])
_set_variant = _sig("phmg_set_apply_variant", C.c_int, [C.c_void_p, C.c_int, C.c_int])
_set_storage = _sig("phmg_set_patch_storage", C.c_int, [C.c_void_p, C.c_int, C.c_int])
_set_spmv = _sig("phmg_set_spmv_variant", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int])
_set_spmm = _sig("phmg_set_spmm_variant", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int])
_set_block = _sig("phmg_set_block_variant", C.c_int, [C.c_void_p, C.c_int, C.c_int])
SPMV_VARIANTS = 20
STORAGE = {"auto": 0, "general": 1}
MAX_RHS = 16

EXPORTED = ["phmg_hierarchy_create", "phmg_hierarchy_destroy", "phmg_relax_setup", "phmg_set_precision",
            "phmg_relax_apply", "phmg_vcycle", "phmg_fgmres_solve", "phmg_residual", "phmg_get_level_info",
            "phmg_profile_enable", "phmg_profile_read", "phmg_profile_reset", "phmg_ritz_max_real",
            "phmg_set_graphs", "phmg_relax_apply_batched", "phmg_vcycle_batched", "phmg_fgmres_solve_batched",
            "phmg_relax_apply_transposed", "phmg_vcycle_transposed", "phmg_fgmres_solve_transposed",
            "phmg_set_sensitivities", "phmg_forcing_rhs", "phmg_gradients",
            "phmg_fbf_create", "phmg_fbf_apply", "phmg_fbf_fgmres_solve", "phmg_fbf_destroy",
            "phmg_set_apply_variant", "phmg_set_patch_storage", "phmg_set_spmv_variant", "phmg_set_spmm_variant",
            "phmg_set_block_variant",
            "phmg_vcycle_batched_transposed", "phmg_fgmres_solve_batched_transposed",
            "phmg_relax_apply_noalloc", "phmg_set_kernel_vector", "phmg_project_kernel", "phmg_last_error"]
NOALLOC_MAX_DOUBLES = 4 << 20


def ritz_max_real(H: np.ndarray, k: int) -> float:
    """Largest real eigenvalue part of H[:k, :k] computed by the library's host QR."""
    Hf = np.asfortranarray(H, dtype=np.float64)
    out = C.c_double(0.0)
    _check(_ritz(Hf.ctypes.data, Hf.shape[0], k, C.byref(out)))
    return float(out.value)


def last_error() -> str:
    return _last_error().decode()


def _check(st: int, allow=()):
    if st != PHMG_OK and st not in allow:
        raise PhmgError(st, last_error())
    return st


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _block_ptr(t, n: int, name: str) -> (int, int):
    """(pointer, nrhs) of a contiguous float64 CUDA tensor of shape (nrhs, n)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.dim() != 2 or t.shape[1] != n or not 1 <= t.shape[0] <= MAX_RHS:
        raise ValueError(f"{name} must have shape (nrhs, {n}) with 1 <= nrhs <= {MAX_RHS}, got {tuple(t.shape)}")
    return t.data_ptr(), int(t.shape[0])


def _vec_ptr(t, n: int, name: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} entries, the level needs {n}")
    return t.data_ptr()


class Hierarchy:
    """A validated hierarchy living in device memory (phmg_hierarchy_create)."""

    def __init__(self, K: Sequence, P: Sequence, patches: Sequence, coarse_null: Optional[np.ndarray],
                 nu_p: int = 2, nu_h: int = 2, n_v: int = 1, n_plevels: int = 1, omega: float = 0.5,
                 smoother: str = "richardson", cheb_lo: float = 0.1, cheb_hi: float = 1.1, eig_iters: int = 20,
                 stream: Optional[int] = None):
        """K: list of (rowptr, col, val, nrows, ncols); P: list of the same (len-1);
        patches: list of (ptr int64, dofs int32, weight float64 or None)."""
        import torch
        keep = []

        def csr(item):
            rowptr, col, val, nrows, ncols = item
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
            col = np.ascontiguousarray(col, dtype=np.int32)
            val = np.ascontiguousarray(val, dtype=np.float64)
            keep.extend([rowptr, col, val])
            return CsrT(int(nrows), int(ncols), int(col.size), _ptr(rowptr), _ptr(col), _ptr(val))

        nl = len(K)
        Ks = (CsrT * nl)(*[csr(k) for k in K])
        Ps = (CsrT * max(nl - 1, 1))(*[csr(p) for p in P])
        pts = []
        for (ptr, dofs, w) in patches:
            ptr = np.ascontiguousarray(ptr, dtype=np.int64)
            dofs = np.ascontiguousarray(dofs, dtype=np.int32)
            w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
            keep.extend([ptr, dofs, w])
            pts.append(PatchesT(int(ptr.size - 1), _ptr(ptr), _ptr(dofs), _ptr(w)))
        Pt = (PatchesT * max(nl - 1, 1))(*pts)
        z = None if coarse_null is None else np.ascontiguousarray(coarse_null, dtype=np.float64)
        desc = DescT(nl, Ks, Ps, Pt, _ptr(z))
        opts = OptsT(nu_p, nu_h, n_v, n_plevels, omega, SMOOTHERS[smoother], eig_iters, cheb_lo, cheb_hi)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        _check(_create(C.byref(desc), C.byref(opts), C.c_void_p(stream), C.byref(h)))
        self._h = h
        self.nlevels = nl
        self.n = [int(k[3]) for k in K]
        self.opts = dict(nu_p=nu_p, nu_h=nu_h, n_v=n_v, n_plevels=n_plevels, omega=omega, smoother=smoother,
                         cheb_lo=cheb_lo, cheb_hi=cheb_hi, eig_iters=eig_iters)

    @classmethod
    def from_frontend(cls, fh, weights: Optional[bool] = None, stream=None, **overrides) -> "Hierarchy":
        """Build from a frontend.Hierarchy (host arrays in the canonical numbering).

        weights: pass the partition-of-unity W_i (default: the workload's choice)."""
        levels = fh.levels
        if weights is None:
            weights = fh.weights
        K = [(l.K.rowptr, l.K.col, l.K.val, l.K.nrows, l.K.ncols) for l in levels]
        P = [(l.P.rowptr, l.P.col, l.P.val, l.P.nrows, l.P.ncols) for l in levels[1:]]
        pts = [(l.patch_ptr, l.patch_dofs, l.patch_weight if weights else None) for l in levels[:-1]]
        opts = dict(fh.opts)
        opts.update(overrides)
        H = cls(K, P, pts, levels[-1].null_vector(), stream=stream, **opts)
        H.set_kernel_vector(levels[0].null_vector())
        if levels[0].visc_sens is not None and levels[0].forcing_map is not None:
            H.set_sensitivities(levels[0].visc_sens, levels[0].forcing_map)
        return H

    def set_apply_variant(self, level: int, variant: int):
        """Override the autotuned patch-solve kernel shape of a level (results are identical)."""
        _check(_set_variant(self._h, level, variant))

    def set_block_variant(self, level: int, variant: int):
        """Override the autotuned multi-right-hand-side patch-solve shape of a level (identical results)."""
        _check(_set_block(self._h, level, variant))

    # -- adjoint gradients
    def set_sensitivities(self, S, G):
        """S: dK/dtheta over K_0's nonzeros (n_theta x nnz), G: forcing map (n_0 x n_f); frontend Csr."""
        keep = []

        def csr(A):
            rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int32)
            col = np.ascontiguousarray(A.col, dtype=np.int32)
            val = np.ascontiguousarray(A.val, dtype=np.float64)
            keep.extend([rowptr, col, val])
            return CsrT(int(A.nrows), int(A.ncols), int(col.size), _ptr(rowptr), _ptr(col), _ptr(val))

        cs, cg = csr(S), csr(G)
        _check(_set_sens(self._h, C.byref(cs), C.byref(cg)))
        self.n_theta, self.n_f = int(S.nrows), int(G.ncols)

    def forcing_rhs(self, F, B):
        """B[c] = G F[c]; F (nrhs, n_f), B (nrhs, n_0) contiguous float64 CUDA tensors."""
        k = F.shape[0]
        if B.shape[0] != k:
            raise ValueError("F and B must hold the same number of systems")
        _check(_forcing_rhs(self._h, k, _vec_ptr(F, k * self.n_f, "F"), _vec_ptr(B, k * self.n[0], "B")))

    def gradients(self, X, Lam, grad_theta, grad_f=None):
        """grad_theta = -sum_c S (Lam_c o X_c on K's nonzeros); grad_f[c] = G^T Lam[c]."""
        k = X.shape[0]
        if Lam.shape[0] != k:
            raise ValueError("X and Lam must hold the same number of systems")
        pf = None if grad_f is None else _vec_ptr(grad_f, k * self.n_f, "grad_f")
        _check(_gradients(self._h, k, _vec_ptr(X, k * self.n[0], "X"), _vec_ptr(Lam, k * self.n[0], "Lam"),
                          _vec_ptr(grad_theta, self.n_theta, "grad_theta"), pf))

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls
    def setup(self, level: int = -1):
        _check(_setup(self._h, level))

    def set_graphs(self, on: bool):
        """Replay the V-cycle as a captured HIP graph (default) or launch it eagerly."""
        _check(_graphs(self._h, 1 if on else 0))

    def set_precision(self, level: int, prec: str):
        _check(_set_prec(self._h, level, PREC[prec]))

    def set_spmv_variant(self, level: int, matrix: str, variant: int):
        """Override the autotuned SpMV kernel of K / P / R on a level, or with "RK" the restricted
        residual's form (0 two-step, 1-6 fused with 2..64 lanes); results differ only in rounding."""
        _check(_set_spmv(self._h, level, {"K": 0, "P": 1, "R": 2, "RK": 3}[matrix], variant))

    def set_spmm_variant(self, level: int, matrix: str, variant: int):
        """Override the autotuned block SpMM shape of K / P / R on a level (0-9, see the header)."""
        _check(_set_spmm(self._h, level, {"K": 0, "P": 1, "R": 2}[matrix], variant))

    def set_patch_storage(self, level: int, storage: str):
        """"auto" (symmetric strip layout when K_l is symmetric to rounding) or "general"."""
        _check(_set_storage(self._h, level, STORAGE[storage]))

    def relax_apply(self, level: int, b, x, nu: int = 1):
        n = self.n[level]
        _check(_apply(self._h, level, _vec_ptr(b, n, "b"), _vec_ptr(x, n, "x"), nu))

    def relax_apply_noalloc(self, level: int, b, x, nu: int = 1):
        """relax_apply with the sweep's work buffers in the library's fixed device array (no allocation)."""
        n = self.n[level]
        _check(_apply_na(self._h, level, _vec_ptr(b, n, "b"), _vec_ptr(x, n, "x"), nu))

    def vcycle(self, b, x):
        _check(_vcycle(self._h, _vec_ptr(b, self.n[0], "b"), _vec_ptr(x, self.n[0], "x")))

    def set_kernel_vector(self, z: Optional[np.ndarray]):
        """Kernel vector of K_0 (host array of n_0 values; None removes it)."""
        zz = None if z is None else np.ascontiguousarray(z, dtype=np.float64)
        if zz is not None and zz.shape != (self.n[0],):
            raise ValueError(f"kernel vector must have {self.n[0]} entries")
        _check(_set_kernel(self._h, _ptr(zz)))

    def project_kernel(self, X):
        """X[c] <- X[c] - (z . X[c] / z . z) z for every row of X (nrhs, n_0), in place on the device."""
        px, k = _block_ptr(X, self.n[0], "X")
        _check(_project(self._h, k, px))

    def residual(self, level: int, b, x, r):
        n = self.n[level]
        _check(_residual(self._h, level, _vec_ptr(b, n, "b"), _vec_ptr(x, n, "x"), _vec_ptr(r, n, "r")))

    def fgmres(self, b, x, rtol: float = 1e-8, restart: int = 30, maxit: int = 1000):
        it = C.c_int(0)
        rr = C.c_double(0.0)
        st = _check(_fgmres(self._h, _vec_ptr(b, self.n[0], "b"), _vec_ptr(x, self.n[0], "x"), rtol, restart, maxit,
                            C.byref(it), C.byref(rr)), allow=(PHMG_ENOCONV,))
        return int(it.value), float(rr.value), st == PHMG_OK

    # ---- adjoint (transposed) operators ----
    def relax_apply_transposed(self, level: int, b, x, nu: int = 1):
        n = self.n[level]
        _check(_apply_t(self._h, level, _vec_ptr(b, n, "b"), _vec_ptr(x, n, "x"), nu))

    def vcycle_transposed(self, b, x):
        _check(_vcycle_t(self._h, _vec_ptr(b, self.n[0], "b"), _vec_ptr(x, self.n[0], "x")))

    def fgmres_transposed(self, b, x, rtol: float = 1e-8, restart: int = 30, maxit: int = 1000):
        it = C.c_int(0)
        rr = C.c_double(0.0)
        st = _check(_fgmres_t(self._h, _vec_ptr(b, self.n[0], "b"), _vec_ptr(x, self.n[0], "x"), rtol, restart,
                              maxit, C.byref(it), C.byref(rr)), allow=(PHMG_ENOCONV,))
        return int(it.value), float(rr.value), st == PHMG_OK

    # ---- several right-hand sides at once: tensors of shape (nrhs, n), nrhs <= 16 ----
    def relax_apply_batched(self, level: int, B, X, nu: int = 1):
        n = self.n[level]
        pb, k = _block_ptr(B, n, "B")
        px, kx = _block_ptr(X, n, "X")
        if k != kx:
            raise ValueError("B and X must hold the same number of right-hand sides")
        _check(_apply_b(self._h, level, k, pb, px, nu))

    def vcycle_batched(self, B, X):
        pb, k = _block_ptr(B, self.n[0], "B")
        px, kx = _block_ptr(X, self.n[0], "X")
        if k != kx:
            raise ValueError("B and X must hold the same number of right-hand sides")
        _check(_vcycle_b(self._h, k, pb, px))

    def fgmres_batched(self, B, X, rtol: float = 1e-8, restart: int = 30, maxit: int = 1000):
        """Solve K x_c = b_c for every row c of B (X in/out); returns (iters[], relres[], all_converged)."""
        return self._fgmres_b(_fgmres_b, B, X, rtol, restart, maxit)

    def fgmres_batched_transposed(self, B, X, rtol: float = 1e-8, restart: int = 30, maxit: int = 1000):
        """Solve K^T x_c = b_c for every row c of B (adjoint cycle; symmetric levels only)."""
        return self._fgmres_b(_fgmres_bt, B, X, rtol, restart, maxit)

    def vcycle_batched_transposed(self, B, X):
        pb, k = _block_ptr(B, self.n[0], "B")
        px, kx = _block_ptr(X, self.n[0], "X")
        if k != kx:
            raise ValueError("B and X must hold the same number of right-hand sides")
        _check(_vcycle_bt(self._h, k, pb, px))

    def _fgmres_b(self, fn, B, X, rtol, restart, maxit):
        pb, k = _block_ptr(B, self.n[0], "B")
        px, kx = _block_ptr(X, self.n[0], "X")
        if k != kx:
            raise ValueError("B and X must hold the same number of right-hand sides")
        it = (C.c_int32 * k)()
        rr = (C.c_double * k)()
        st = _check(fn(self._h, k, pb, px, rtol, restart, maxit, it, rr), allow=(PHMG_ENOCONV,))
        return [int(v) for v in it], [float(v) for v in rr], st == PHMG_OK

    def level_info(self, level: int) -> dict:
        i = LevelInfoT()
        _check(_info(self._h, level, C.byref(i)))
        return dict(n=i.n, npatch=i.npatch, max_m=i.max_m, precision=i.precision, nnz=i.nnz, sum_m=i.sum_m,
                    sum_m2=i.sum_m2, lambda_max=i.lambda_max, apply_variant=i.apply_variant,
                    apply_variants=i.apply_variants, symmetric_storage=bool(i.symmetric_storage), spmv_variant=i.spmv_variant,
                    stored_elements=i.stored_elements, block_variant=i.block_variant,
                    block_variants=i.block_variants)

    def profile(self, kernels=("patch_apply",)):
        """Enable HIP-event timing of the named kernels (empty = off)."""
        mask = 0
        for k in kernels:
            mask |= 1 << KERNELS[k]
        _check(_prof_on(self._h, mask))

    def profile_reset(self):
        _check(_prof_reset(self._h))

    def profile_read(self, kernel: str, level: int = -1):
        """(summed milliseconds, launches) of one kernel on one level (-1 = all levels)."""
        ms = C.c_double(0.0)
        cnt = C.c_int64(0)
        _check(_prof_read(self._h, KERNELS[kernel], level, C.byref(ms), C.byref(cnt)))
        return float(ms.value), int(cnt.value)


def _csr_struct(A, keep):
    rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int32)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    keep.extend([rowptr, col, val])
    return CsrT(int(A.nrows), int(A.ncols), int(col.size), _ptr(rowptr), _ptr(col), _ptr(val))


class Fbf:
    """Full-block-factorisation preconditioner and its FGMRES (phmg_fbf_*).

    velocity: a set-up Hierarchy on the velocity block; K, B, S_inv: frontend Csr objects."""

    def __init__(self, velocity: Hierarchy, K, B, S_inv):
        keep = []
        ck, cb, cs = _csr_struct(K, keep), _csr_struct(B, keep), _csr_struct(S_inv, keep)
        h = C.c_void_p()
        _check(_fbf_create(velocity._h, C.byref(ck), C.byref(cb), C.byref(cs), C.byref(h)))
        self._h = h
        self.velocity = velocity          # keeps the velocity context alive
        self.n = int(K.nrows)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _fbf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, r, z):
        _check(_fbf_apply(self._h, _vec_ptr(r, self.n, "r"), _vec_ptr(z, self.n, "z")))

    def fgmres(self, b, x, rtol: float = 1e-8, restart: int = 30, maxit: int = 1000):
        it = C.c_int(0)
        rr = C.c_double(0.0)
        st = _check(_fbf_fgmres(self._h, _vec_ptr(b, self.n, "b"), _vec_ptr(x, self.n, "x"), rtol, restart, maxit,
                                C.byref(it), C.byref(rr)), allow=(PHMG_ENOCONV,))
        return int(it.value), float(rr.value), st == PHMG_OK
