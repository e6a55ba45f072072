"""Taylor-Hood / Scott-Vogelius discretisation of Stokes (oracle).

Follows Section 2: the weak form a(u,v) = int grad u : grad v,
b(p,v) = -int p div v, F(v) = int f.v (eq. "eq:stokes-disc"), giving the
saddle-point matrix K = [A B^T; B 0] (eq. "eq:saddle") with A the vector
Laplacian and B the negative divergence.  Section 2.1: Taylor-Hood uses
continuous P_k / P_{k-1}, Scott-Vogelius continuous P_k / discontinuous
P_{k-1} on an Alfeld-split mesh.

Readings where the paper is silent:
  * Dirichlet data are imposed strongly by eliminating the boundary velocity
    DoFs (their values lifted into the right-hand side).
  * Canonical global numbering, shared *as a convention* with the GPU path's
    front-end so that two independent codes produce comparable vectors:
    [u_x | u_y | p], free DoFs only.  Within a continuous scalar field:
    vertex DoFs by vertex id, then edge DoFs by edge id (edges are the sorted
    vertex pairs in lexicographic order; interior edge nodes run from the
    lower-id to the higher-id vertex), then cell-interior DoFs by cell id,
    each cell's interior nodes in ascending lexicographic barycentric order
    relative to the cell's vertex order.  Discontinuous pressure: cell by
    cell, all local nodes in ascending lexicographic barycentric order.
  * Only structural nonzeros are stored: no u_x - u_y coupling block.
  * The forcing is interpolated into the velocity space before it is
    integrated, F(v) = int (I_h f).v, so the discrete right-hand side is an
    exact polynomial integral (the interpolation error is O(h^{k+1}), below
    the discretisation error measured in L2).

Pins: tests/test_oracle_discretization.py -- K symmetric, A SPD, K z = 0 for
the constant pressure z, B annihilates interpolated curls of polynomials,
manufactured-solution L2 rates k+1 (velocity) and k (pressure), and for SV
the direct pointwise divergence equals the projected one (-M_T^{-1} B u) on
arbitrary velocity fields while for TH it does not.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

from . import element


def _edge_ids(cells: np.ndarray):
    pairs = set()
    for c in cells:
        for t in range(3):
            a, b = int(c[t]), int(c[(t + 1) % 3])
            pairs.add((min(a, b), max(a, b)))
    ordered = sorted(pairs)
    return {e: i for i, e in enumerate(ordered)}, ordered


class ScalarSpace:
    """Lagrange space of degree k on a triangle mesh, continuous or not."""

    def __init__(self, verts: np.ndarray, cells: np.ndarray, k: int, continuous: bool):
        self.verts, self.cells, self.k, self.continuous = verts, cells, k, continuous
        nv, nc = verts.shape[0], cells.shape[0]
        mi = element.multi_indices(k)
        self.nloc = len(mi)
        ref = element.node_points(k)
        cell_dofs = np.zeros((nc, self.nloc), dtype=np.int64)
        if continuous:
            assert k >= 1
            edge_id, edges = _edge_ids(cells)
            self.edges = edges
            ne = len(edges)
            interior = [a for a in mi if min(a) >= 1]
            nint = len(interior)
            self.ndofs = nv + ne * (k - 1) + nc * nint
            for c in range(nc):
                cv = [int(v) for v in cells[c]]
                for n, a in enumerate(mi):
                    nz = [t for t in range(3) if a[t] > 0]
                    if len(nz) == 1:
                        gid = cv[nz[0]]
                    elif len(nz) == 2:
                        t1, t2 = nz
                        g1, g2 = cv[t1], cv[t2]
                        lo, hi = (t1, t2) if g1 < g2 else (t2, t1)
                        e = edge_id[(cv[lo], cv[hi])]
                        gid = nv + e * (k - 1) + (a[hi] - 1)
                    else:
                        gid = nv + ne * (k - 1) + c * nint + interior.index(a)
                    cell_dofs[c, n] = gid
            # boundary: edges that belong to exactly one cell
            count = {}
            for c in cells:
                for t in range(3):
                    a, b = int(c[t]), int(c[(t + 1) % 3])
                    key = (min(a, b), max(a, b))
                    count[key] = count.get(key, 0) + 1
            bnd = np.zeros(self.ndofs, dtype=bool)
            for (a, b), cnt in count.items():
                if cnt == 1:
                    bnd[a] = True
                    bnd[b] = True
                    e = edge_id[(a, b)]
                    bnd[nv + e * (k - 1): nv + (e + 1) * (k - 1)] = True
            self.boundary = bnd
        else:
            self.ndofs = nc * self.nloc
            for c in range(nc):
                cell_dofs[c] = c * self.nloc + np.arange(self.nloc)
            self.boundary = np.zeros(self.ndofs, dtype=bool)
        self.cell_dofs = cell_dofs
        coords = np.zeros((self.ndofs, 2))
        for c in range(nc):
            x0 = verts[cells[c, 0]]
            J = np.stack([verts[cells[c, 1]] - x0, verts[cells[c, 2]] - x0], axis=1)
            coords[cell_dofs[c]] = x0 + ref @ J.T
        self.coords = coords


def cell_geometry(verts: np.ndarray, cell: np.ndarray):
    """Affine map x = x0 + J xi of one triangle: (x0, J, |det J|, J^{-T})."""
    x0 = verts[cell[0]]
    J = np.stack([verts[cell[1]] - x0, verts[cell[2]] - x0], axis=1)
    det = J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
    return x0, J, abs(det), np.linalg.inv(J).T


@dataclass
class Stokes:
    """Assembled Stokes system on free DoFs in the canonical numbering."""
    mesh: object
    k: int
    kind: str                     # "TH" or "SV"
    V: ScalarSpace
    Q: ScalarSpace
    free_u: np.ndarray            # scalar velocity node ids that are free, ascending
    nfu: int
    nq: int
    K: sp.csr_matrix
    b: np.ndarray
    L_full: sp.csr_matrix         # scalar Laplacian on all velocity nodes
    Bx_full: sp.csr_matrix
    By_full: sp.csr_matrix
    g: Optional[np.ndarray] = None  # Dirichlet values at all velocity nodes (2, nV)
    log_visc: Optional[np.ndarray] = None   # nodal log-viscosity at the mesh vertices (None: nu = 1)

    @property
    def n(self) -> int:
        return 2 * self.nfu + self.nq

    def u_index(self, comp: int, scalar_ids: np.ndarray) -> np.ndarray:
        """Free global index of (component, scalar node); -1 where the node is fixed."""
        pos = np.full(self.V.ndofs, -1, dtype=np.int64)
        pos[self.free_u] = np.arange(self.nfu)
        out = pos[scalar_ids]
        return np.where(out >= 0, out + comp * self.nfu, -1)

    def p_index(self, q_ids: np.ndarray) -> np.ndarray:
        return 2 * self.nfu + np.asarray(q_ids, dtype=np.int64)

    def null_vector(self) -> np.ndarray:
        """Constant pressure, zero velocity: spans ker K when all of the boundary is Dirichlet."""
        z = np.zeros(self.n)
        z[2 * self.nfu:] = 1.0
        return z


def p1_weights(qpts: np.ndarray) -> np.ndarray:
    """Barycentric (P1 hat) values of the three cell vertices at reference points, (nq, 3)."""
    return np.stack([1.0 - qpts[:, 0] - qpts[:, 1], qpts[:, 0], qpts[:, 1]], axis=1)


def assemble_stokes(mesh, k: int, kind: str,
                    forcing: Optional[Callable] = None,
                    dirichlet: Optional[Callable] = None,
                    log_visc: Optional[np.ndarray] = None) -> Stokes:
    """Assemble K and b on free DoFs (eq. "eq:stokes-disc", "eq:saddle").

    forcing(x, y) -> (fx, fy); dirichlet(x, y) -> (gx, gy) on boundary nodes.
    log_visc: values l_v at the mesh vertices; the viscosity is the piecewise
    linear interpolant of exp(l), nu_h = sum_v exp(l_v) lambda_v, and the
    velocity block becomes int nu_h grad u : grad v (the paper takes nu = 1;
    the variable field serves the gradient workload).  The rule of degree 2k
    integrates nu_h grad phi_a . grad phi_b (degree 2k - 1) exactly.
    """
    verts, cells = mesh.verts, mesh.cells
    V = ScalarSpace(verts, cells, k, continuous=True)
    Q = ScalarSpace(verts, cells, k - 1, continuous=(kind == "TH"))
    qpts, qw = element.quadrature(2 * k)
    phi, dphi = element.eval_basis(k, qpts)
    psi, _ = element.eval_basis(k - 1, qpts) if k - 1 >= 1 else (np.ones((len(qw), 1)), None)
    lam = p1_weights(qpts)

    rows_L, cols_L, vals_L = [], [], []
    rows_B, cols_B, vals_Bx, vals_By = [], [], [], []
    Fx = np.zeros(V.ndofs)
    Fy = np.zeros(V.ndofs)
    for c in range(cells.shape[0]):
        x0, J, adet, JinvT = cell_geometry(verts, cells[c])
        grad = np.einsum("ij,qnj->qni", JinvT, dphi)          # physical gradients
        w = qw * adet
        if log_visc is None:
            Lc = np.einsum("q,qai,qbi->ab", w, grad, grad)
        else:
            nu_q = lam @ np.exp(log_visc[cells[c]])
            Lc = np.einsum("q,qai,qbi->ab", w * nu_q, grad, grad)
        Bxc = -np.einsum("q,qi,qa->ia", w, psi, grad[:, :, 0])
        Byc = -np.einsum("q,qi,qa->ia", w, psi, grad[:, :, 1])
        vd = V.cell_dofs[c]
        qd = Q.cell_dofs[c]
        rows_L.append(np.repeat(vd, len(vd)))
        cols_L.append(np.tile(vd, len(vd)))
        vals_L.append(Lc.ravel())
        rows_B.append(np.repeat(qd, len(vd)))
        cols_B.append(np.tile(vd, len(qd)))
        vals_Bx.append(Bxc.ravel())
        vals_By.append(Byc.ravel())
        if forcing is not None:
            # F(v) = int (I_h f) . v: the forcing is interpolated at the velocity
            # nodes, then integrated exactly with the element mass matrix
            Mc = np.einsum("q,qa,qb->ab", qw * adet, phi, phi)
            fx, fy = forcing(V.coords[vd, 0], V.coords[vd, 1])
            Fx[vd] += Mc @ fx
            Fy[vd] += Mc @ fy

    nV, nQ = V.ndofs, Q.ndofs
    L = sp.csr_matrix((np.concatenate(vals_L), (np.concatenate(rows_L), np.concatenate(cols_L))), shape=(nV, nV))
    rB, cB = np.concatenate(rows_B), np.concatenate(cols_B)
    Bx = sp.csr_matrix((np.concatenate(vals_Bx), (rB, cB)), shape=(nQ, nV))
    By = sp.csr_matrix((np.concatenate(vals_By), (rB, cB)), shape=(nQ, nV))
    for M in (L, Bx, By):
        M.sum_duplicates()
        M.sort_indices()

    free = np.flatnonzero(~V.boundary)
    bnd = np.flatnonzero(V.boundary)
    nfu = len(free)
    Lff = L[free][:, free]
    Bxf = Bx[:, free]
    Byf = By[:, free]
    Z = sp.csr_matrix((nfu, nfu))
    Zq = sp.csr_matrix((nQ, nQ))
    K = sp.bmat([[Lff, Z, Bxf.T], [Z, Lff, Byf.T], [Bxf, Byf, Zq]], format="csr")
    # bmat drops empty blocks' entries only; keep the structural pattern of the three blocks
    K.sort_indices()

    g = np.zeros((2, nV))
    if dirichlet is not None and len(bnd):
        gx, gy = dirichlet(V.coords[bnd, 0], V.coords[bnd, 1])
        g[0, bnd], g[1, bnd] = gx, gy
    bu_x = Fx[free] - L[free][:, bnd] @ g[0, bnd]
    bu_y = Fy[free] - L[free][:, bnd] @ g[1, bnd]
    bp = -(Bx[:, bnd] @ g[0, bnd] + By[:, bnd] @ g[1, bnd])
    b = np.concatenate([bu_x, bu_y, bp])
    return Stokes(mesh, k, kind, V, Q, free, nfu, nQ, K, b, L, Bx, By, g,
                  None if log_visc is None else np.array(log_visc, dtype=np.float64))


def load_vector(disc: Stokes, forcing: Callable) -> np.ndarray:
    """Right-hand side of another forcing on an assembled system (eq. "eq:stokes-disc").

    Same reading as assemble_stokes: F(v) = int (I_h f).v with the exact
    element mass matrix, minus the lift of the system's Dirichlet data.
    """
    V, k = disc.V, disc.k
    qpts, qw = element.quadrature(2 * k)
    phi, _ = element.eval_basis(k, qpts)
    Fx = np.zeros(V.ndofs)
    Fy = np.zeros(V.ndofs)
    for c in range(disc.mesh.cells.shape[0]):
        _, _, adet, _ = cell_geometry(disc.mesh.verts, disc.mesh.cells[c])
        Mc = np.einsum("q,qa,qb->ab", qw * adet, phi, phi)
        vd = V.cell_dofs[c]
        fx, fy = forcing(V.coords[vd, 0], V.coords[vd, 1])
        Fx[vd] += Mc @ fx
        Fy[vd] += Mc @ fy
    free, bnd = disc.free_u, np.flatnonzero(V.boundary)
    L = disc.L_full
    bu_x = Fx[free] - L[free][:, bnd] @ disc.g[0, bnd]
    bu_y = Fy[free] - L[free][:, bnd] @ disc.g[1, bnd]
    bp = -(disc.Bx_full[:, bnd] @ disc.g[0, bnd] + disc.By_full[:, bnd] @ disc.g[1, bnd])
    return np.concatenate([bu_x, bu_y, bp])


def interpolate(disc: Stokes, u: Callable, p: Optional[Callable] = None) -> np.ndarray:
    """Nodal interpolant on the free DoFs (velocity), and pressure if given."""
    x = np.zeros(disc.n)
    cu = disc.V.coords[disc.free_u]
    ux, uy = u(cu[:, 0], cu[:, 1])
    x[: disc.nfu] = ux
    x[disc.nfu: 2 * disc.nfu] = uy
    if p is not None:
        x[2 * disc.nfu:] = p(disc.Q.coords[:, 0], disc.Q.coords[:, 1])
    return x


def full_velocity(disc: Stokes, x: np.ndarray) -> np.ndarray:
    """(2, nV) nodal velocity with the Dirichlet values put back."""
    U = disc.g.copy()
    U[0, disc.free_u] = x[: disc.nfu]
    U[1, disc.free_u] = x[disc.nfu: 2 * disc.nfu]
    return U


def l2_errors(disc: Stokes, x: np.ndarray, u_exact: Callable, p_exact: Callable):
    """L2 errors of velocity and of pressure (both means removed from the pressure error)."""
    k = disc.k
    qp, qw = element.quadrature(2 * k + 4)
    phi, _ = element.eval_basis(k, qp)
    psi, _ = element.eval_basis(k - 1, qp) if k - 1 >= 1 else (np.ones((len(qw), 1)), None)
    U = full_velocity(disc, x)
    P = x[2 * disc.nfu:]
    verts, cells = disc.mesh.verts, disc.mesh.cells
    eu2 = 0.0
    ep_int, ep2, area = 0.0, 0.0, 0.0
    for c in range(cells.shape[0]):
        x0, J, adet, _ = cell_geometry(verts, cells[c])
        xq = x0 + qp @ J.T
        w = qw * adet
        vd = disc.V.cell_dofs[c]
        uhx, uhy = phi @ U[0, vd], phi @ U[1, vd]
        ux, uy = u_exact(xq[:, 0], xq[:, 1])
        eu2 += np.sum(w * ((uhx - ux) ** 2 + (uhy - uy) ** 2))
        ph = psi @ P[disc.Q.cell_dofs[c]]
        e = ph - p_exact(xq[:, 0], xq[:, 1])
        ep_int += np.sum(w * e)
        ep2 += np.sum(w * e * e)
        area += np.sum(w)
    mean = ep_int / area
    return np.sqrt(eu2), np.sqrt(max(ep2 - 2 * mean * ep_int + mean * mean * area, 0.0))


def divergence_at_quadrature(disc: Stokes, x: np.ndarray, degree: int = None) -> np.ndarray:
    """div u_h at the quadrature points of every cell (Scott-Vogelius check, Section 2.1)."""
    k = disc.k
    qp, _ = element.quadrature(degree or 2 * k)
    _, dphi = element.eval_basis(k, qp)
    U = full_velocity(disc, x)
    verts, cells = disc.mesh.verts, disc.mesh.cells
    out = []
    for c in range(cells.shape[0]):
        _, _, _, JinvT = cell_geometry(verts, cells[c])
        grad = np.einsum("ij,qnj->qni", JinvT, dphi)
        vd = disc.V.cell_dofs[c]
        out.append(grad[:, :, 0] @ U[0, vd] + grad[:, :, 1] @ U[1, vd])
    return np.concatenate(out)


def divergence_projected(disc: Stokes, x: np.ndarray, degree: int = None) -> np.ndarray:
    """div u_h at the quadrature points through the discrete identity div u_h = -M_T^{-1} (B u_h)_T.

    For Scott-Vogelius div V_h is contained in the discontinuous pressure
    space (Section 2.1), so on every cell T the divergence equals its own L2
    projection onto P_{k-1}(T): coefficients c_T = M_T^{-1} (-B u_h)_T with the
    cell pressure mass matrix M_T.  This evaluation avoids the cancellation of
    summing u_a grad(phi_a) directly.  Only meaningful for "SV".
    """
    if disc.kind != "SV":
        raise ValueError("the projection identity holds for Scott-Vogelius only")
    k = disc.k
    qp, qw = element.quadrature(degree or 2 * k)
    psi, _ = element.eval_basis(k - 1, qp) if k - 1 >= 1 else (np.ones((len(qw), 1)), None)
    U = full_velocity(disc, x)
    Bu = disc.Bx_full @ U[0] + disc.By_full @ U[1]
    verts, cells = disc.mesh.verts, disc.mesh.cells
    out = []
    for c in range(cells.shape[0]):
        _, _, adet, _ = cell_geometry(verts, cells[c])
        M = np.einsum("q,qi,qj->ij", qw * adet, psi, psi)
        coef = np.linalg.solve(M, -Bu[disc.Q.cell_dofs[c]])
        out.append(psi @ coef)
    return np.concatenate(out)
