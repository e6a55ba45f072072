"""Gradients through the preconditioned Stokes solve by the adjoint method (oracle).

This is test infrastructure: it checks the GPU path's adjoint.

Objective (batched over right-hand sides b = 0..B-1):
    J = 1/2 sum_b || u_b - t_b ||^2,
u_b the velocity part of the solution x_b of K(l) x_b = F f_b, t_b a target.
The paper has no adjoint; the method is the standard one for a linear
constraint: K^T lam_b = dJ/dx_b (the velocity misfit, zero pressure rows),
solved with FGMRES preconditioned by the transposed cycle, then
    dJ/dl_v = - sum_b lam_b^T (dK/dl_v) x_b,      dJ/df_b = F^T lam_b.
With nu_h = sum_v exp(l_v) lambda_v (oracle/discretization.py), dK/dl_v is
exp(l_v) times the velocity-block stiffness weighted by the hat function of
vertex v; it is applied here cell by cell (element matrices), with the full
nodal velocity so that a Dirichlet lift is differentiated as well.  F maps
the nodal forcing values (both components, every velocity node) to the free
right-hand side: F = M[free, :] per component, M the velocity mass matrix.

Readings (the paper is silent): the misfit is the Euclidean norm of the
free velocity DoFs; the log-viscosity is a nodal (P1) field on the finest
mesh, injected to the vertices of the coarser nested meshes.

Pins: tests/test_oracle_adjoint.py -- central finite differences of J with
a sparse direct solve (no multigrid, no Krylov) on small meshes, for the
viscosity and the forcing gradients; J is quadratic in f, so there the
difference quotient is exact up to rounding.
"""
from __future__ import annotations

from typing import List

import numpy as np

from . import element
from .discretization import Stokes, cell_geometry, full_velocity, p1_weights
from .fgmres import fgmres
from .multigrid import vcycle


def objective(X: np.ndarray, T: np.ndarray, nfu: int, dim: int = 2) -> float:
    d = X[:, : dim * nfu] - T[:, : dim * nfu]
    return 0.5 * float(np.sum(d * d))


def objective_gradient(X: np.ndarray, T: np.ndarray, nfu: int, dim: int = 2) -> np.ndarray:
    G = np.zeros_like(X)
    G[:, : dim * nfu] = X[:, : dim * nfu] - T[:, : dim * nfu]
    return G


def adjoint_solve(levels, opts, G: np.ndarray, rtol: float = 1e-12, restart: int = 30, maxit: int = 1000):
    """lam_b from K^T lam_b = G_b, FGMRES right-preconditioned by the transposed cycle."""
    KT = levels[0].K.T.tocsr()
    out = []
    for g in G:
        res = fgmres(lambda v: KT @ v, lambda v: vcycle(levels, opts, v, transpose=True), g, rtol=rtol,
                     restart=restart, maxit=maxit)
        out.append(res.x)
    return np.stack(out)


def _free_local(disc: Stokes, vd: np.ndarray, comp: int, vec: np.ndarray) -> np.ndarray:
    """Values of one velocity component of a free-DoF vector at the cell's nodes (0 at fixed nodes)."""
    idx = disc.u_index(comp, vd)
    out = np.zeros(len(vd))
    m = idx >= 0
    out[m] = vec[idx[m]]
    return out


def viscosity_gradient(disc: Stokes, X: np.ndarray, Lam: np.ndarray) -> np.ndarray:
    """- sum_b lam_b^T (dK/dl_v) x_b for every vertex v (the partial derivative in the adjoint formula)."""
    if getattr(disc, "dim", 2) == 3:
        from . import stokes3d
        return stokes3d.viscosity_gradient(disc, X, Lam)
    verts, cells = disc.mesh.verts, disc.mesh.cells
    lv = disc.log_visc if disc.log_visc is not None else np.zeros(verts.shape[0])
    k = disc.k
    qpts, qw = element.quadrature(2 * k)
    _, dphi = element.eval_basis(k, qpts)
    lam = p1_weights(qpts)
    grad = np.zeros(verts.shape[0])
    U = [full_velocity(disc, x) for x in X]                  # (2, nV) with Dirichlet values
    for c in range(cells.shape[0]):
        _, _, adet, JinvT = cell_geometry(verts, cells[c])
        g = np.einsum("ij,qnj->qni", JinvT, dphi)
        vd = disc.V.cell_dofs[c]
        for t in range(3):
            v = int(cells[c, t])
            At = np.exp(lv[v]) * np.einsum("q,qai,qbi->ab", qw * adet * lam[:, t], g, g)
            s = 0.0
            for b in range(X.shape[0]):
                for comp in range(2):
                    s += _free_local(disc, vd, comp, Lam[b]) @ (At @ U[b][comp, vd])
            grad[v] -= s
    return grad


def forcing_gradient(disc: Stokes, Lam: np.ndarray) -> np.ndarray:
    """F^T lam_b: (B, d, nV), the gradient with respect to the nodal forcing values."""
    if getattr(disc, "dim", 2) == 3:
        from . import stokes3d
        return stokes3d.forcing_gradient(disc, Lam)
    verts, cells = disc.mesh.verts, disc.mesh.cells
    k = disc.k
    qpts, qw = element.quadrature(2 * k)
    phi, _ = element.eval_basis(k, qpts)
    out = np.zeros((Lam.shape[0], 2, disc.V.ndofs))
    for c in range(cells.shape[0]):
        _, _, adet, _ = cell_geometry(verts, cells[c])
        Mc = np.einsum("q,qa,qb->ab", qw * adet, phi, phi)
        vd = disc.V.cell_dofs[c]
        for b in range(Lam.shape[0]):
            for comp in range(2):
                out[b, comp, vd] += Mc.T @ _free_local(disc, vd, comp, Lam[b])
    return out


def forcing_rhs(disc: Stokes, f_nodal: np.ndarray) -> np.ndarray:
    """Free right-hand sides of nodal forcings f_nodal (B, d, nV): F f_b (homogeneous Dirichlet data)."""
    if getattr(disc, "dim", 2) == 3:
        from . import stokes3d
        return stokes3d.forcing_rhs(disc, f_nodal)
    verts, cells = disc.mesh.verts, disc.mesh.cells
    k = disc.k
    qpts, qw = element.quadrature(2 * k)
    phi, _ = element.eval_basis(k, qpts)
    out = np.zeros((f_nodal.shape[0], disc.n))
    full = np.zeros((f_nodal.shape[0], 2, disc.V.ndofs))
    for c in range(cells.shape[0]):
        _, _, adet, _ = cell_geometry(verts, cells[c])
        Mc = np.einsum("q,qa,qb->ab", qw * adet, phi, phi)
        vd = disc.V.cell_dofs[c]
        for b in range(f_nodal.shape[0]):
            for comp in range(2):
                full[b, comp, vd] += Mc @ f_nodal[b, comp, vd]
    for comp in range(2):
        out[:, comp * disc.nfu: (comp + 1) * disc.nfu] = full[:, comp, disc.free_u]
    return out


def gradients(levels: List, opts, disc: Stokes, X: np.ndarray, T: np.ndarray, rtol: float = 1e-12):
    """(J, dJ/dl (nvert,), dJ/df (B, 2, nV), lam) at the solutions X of the batch."""
    dim = getattr(disc, "dim", 2)
    G = objective_gradient(X, T, disc.nfu, dim)
    Lam = adjoint_solve(levels, opts, G, rtol=rtol)
    return objective(X, T, disc.nfu, dim), viscosity_gradient(disc, X, Lam), forcing_gradient(disc, Lam), Lam
