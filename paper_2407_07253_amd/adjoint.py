"""Differentiable Stokes solve: torch.autograd.Function with a hand-written adjoint.

Forward: x_c = K(l)^{-1} G f_c for a batch of nodal forcings f_c, where l is
the nodal log-viscosity on the finest mesh's vertices (the velocity block is
int nu_h grad u : grad v with nu_h the P1 interpolant of exp(l)) and G maps
nodal forcing values to the free right-hand side.  The host front-end
assembles the hierarchy for l; the library solves with FGMRES right-
preconditioned by the phMG / hMG cycle (batched over the forcings).

Backward (adjoint method): K^T lam_c = dJ/dx_c, solved by FGMRES on K^T
right-preconditioned by the transposed cycle (the library's transposed patch
solves reuse the forward factors), then
    dJ/dl = - sum_c lam_c^T (dK/dl) x_c,   dJ/df_c = G^T lam_c,
both contracted on the GPU (phmg_gradients).

The constant pressure spans the kernel of K when the whole boundary is
Dirichlet: the forward output has its pressure mean removed (the l2
projection off that kernel, phmg_project_kernel), and the backward applies
the same projection to the incoming gradient, so the adjoint systems are
consistent.  Every arithmetic step runs in the library; this module only
marshals tensors.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

import synth

from . import frontend
from ._lib import MAX_RHS, Hierarchy


class StokesProblem:
    """A workload's hierarchy with viscosity and forcing as inputs (homogeneous Dirichlet data)."""

    def __init__(self, name: str, k: Optional[int] = None, rtol: float = 1e-10, restart: int = 30,
                 maxit: int = 1000, precision: str = "f64", batched_adjoint: bool = True):
        self.name, self.k = name, k
        self.rtol, self.restart, self.maxit = rtol, restart, maxit
        self.precision = precision
        self.batched_adjoint = batched_adjoint     # adjoint solves through the block path (symmetric levels)
        self.mesh = synth.config_mesh_hierarchy(name)[-1]
        self.nv = self.mesh.verts.shape[0]
        self._key = None
        self._H = None
        self._fh = None
        self.last_iters = None

    def hierarchy(self, log_visc: np.ndarray):
        """(front-end hierarchy, set-up library hierarchy) for this log-viscosity (cached)."""
        lv = np.ascontiguousarray(log_visc, dtype=np.float64)
        if lv.shape != (self.nv,):
            raise ValueError(f"log_visc must have shape ({self.nv},), got {lv.shape}")
        key = lv.tobytes()
        if key != self._key:
            fh = frontend.build_hierarchy(self.name, self.k, forcing=None, log_visc=lv, sensitivities=True)
            H = Hierarchy.from_frontend(fh)
            for lev in range(len(fh.levels) - 1):
                H.set_precision(lev, self.precision)
            H.setup()
            self._key, self._fh, self._H = key, fh, H
        return self._fh, self._H

    @property
    def sizes(self):
        """(n_0, first pressure index, number of forcing parameters)."""
        fh, _ = self._fh, self._H
        if fh is None:
            raise RuntimeError("no hierarchy built yet")
        L0 = fh.levels[0]
        return L0.n, L0.dim * L0.nfu, L0.forcing_map.ncols

    def solve(self, f, log_visc):
        """x (nrhs, n_0) for nodal forcings f (nrhs, 2 nV) and log-viscosity (nv,), differentiable in both."""
        return _StokesSolve.apply(f, log_visc, self)


def _project_pressure(H, X):
    """X[c] <- X[c] minus its component along the constant pressure (phmg_project_kernel), in blocks
    of at most MAX_RHS rows."""
    for c0 in range(0, X.shape[0], MAX_RHS):
        c1 = min(X.shape[0], c0 + MAX_RHS)
        Xc = X[c0:c1].contiguous()
        H.project_kernel(Xc)
        X[c0:c1] = Xc


def _autograd():
    import torch

    class StokesSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, f, log_visc, problem):
            fh, H = problem.hierarchy(log_visc.detach().cpu().numpy())
            n0, p0, nf = problem.sizes
            F = f.detach().to(device="cuda", dtype=torch.float64).contiguous()
            if F.dim() != 2 or F.shape[1] != nf:
                raise ValueError(f"f must have shape (nrhs, {nf})")
            nrhs = F.shape[0]
            B = torch.empty(nrhs, n0, dtype=torch.float64, device="cuda")
            H.forcing_rhs(F, B)
            X = torch.zeros_like(B)
            iters = []
            for c0 in range(0, nrhs, MAX_RHS):
                c1 = min(nrhs, c0 + MAX_RHS)
                Xc = X[c0:c1].contiguous()
                its, rr, ok = H.fgmres_batched(B[c0:c1].contiguous(), Xc, rtol=problem.rtol,
                                               restart=problem.restart, maxit=problem.maxit)
                if not ok:
                    raise RuntimeError(f"forward solve did not converge (relres {max(rr):.3e})")
                X[c0:c1] = Xc
                iters += its
            problem.last_iters = iters
            ctx.problem, ctx.H, ctx.p0 = problem, H, p0
            ctx.devices = (f.device, log_visc.device)
            ctx.save_for_backward(X.clone())
            _project_pressure(H, X)
            return X

        @staticmethod
        def backward(ctx, gX):
            (X,) = ctx.saved_tensors
            problem, H, p0 = ctx.problem, ctx.H, ctx.p0
            G = gX.detach().to(torch.float64).contiguous().clone()
            _project_pressure(H, G)
            Lam = torch.zeros_like(G)
            adj_iters = []
            infos = [H.level_info(l) for l in range(H.nlevels - 1)]
            block_ok = problem.batched_adjoint and all(i["symmetric_storage"] or i["npatch"] == 0 for i in infos)
            if block_ok:
                # all adjoint systems together through the block adjoint cycle (needs symmetric levels)
                for c0 in range(0, G.shape[0], MAX_RHS):
                    c1 = min(G.shape[0], c0 + MAX_RHS)
                    Lc = Lam[c0:c1].contiguous()
                    its, rr, ok = H.fgmres_batched_transposed(G[c0:c1].contiguous(), Lc, rtol=problem.rtol,
                                                              restart=problem.restart, maxit=problem.maxit)
                    if not ok:
                        raise RuntimeError(f"adjoint solve did not converge (relres {max(rr):.3e})")
                    Lam[c0:c1] = Lc
                    adj_iters += its
            else:
                for c in range(G.shape[0]):
                    lc = torch.zeros(G.shape[1], dtype=torch.float64, device="cuda")
                    its, rr, ok = H.fgmres_transposed(G[c].contiguous(), lc, rtol=problem.rtol,
                                                      restart=problem.restart, maxit=problem.maxit)
                    if not ok:
                        raise RuntimeError(f"adjoint solve did not converge (relres {rr:.3e})")
                    Lam[c] = lc
                    adj_iters.append(its)
            problem.last_adjoint_iters = adj_iters
            n_theta = H.n_theta
            grad_l = torch.empty(n_theta, dtype=torch.float64, device="cuda")
            grad_f = torch.empty(G.shape[0], H.n_f, dtype=torch.float64, device="cuda")
            H.gradients(X, Lam, grad_l, grad_f)
            dev_f, dev_l = ctx.devices
            return grad_f.to(dev_f), grad_l.to(dev_l), None

    return StokesSolve


class _Lazy:
    fn = None

    @classmethod
    def apply(cls, *args):
        if cls.fn is None:
            cls.fn = _autograd()
        return cls.fn.apply(*args)


_StokesSolve = _Lazy
