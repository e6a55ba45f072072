"""Taylor-Hood P2/P1 Stokes on tetrahedral meshes (oracle, 3D).

The 3D counterpart of discretization.py / patches.py / transfer.py for the
adjoint workload (unit cube, Kuhn tetrahedra): the weak form of Section 2
(eq. "eq:stokes-disc", "eq:saddle") with continuous P_k / P_{k-1} (k = 2),
K = [A B^T; B 0], A = diag(L, L, L); the Vanka-star patches of Section 3.4
(velocity DoFs of closure(star v), pressure DoFs of star v — for P1 pressure
only the vertex v itself); finite-element interpolation transfers (Section
3.1).  Plain per-cell loops; test infrastructure only.

Readings: the same as in 2D (eliminated Dirichlet DoFs, F(v) = int (I_h f).v,
structural nonzeros only, nu_h = P1 interpolant of exp(l) for a variable
viscosity).  Canonical numbering [u_x | u_y | u_z | p] over free DoFs,
vertices by id, then edges by id (sorted vertex pairs in lexicographic
order); P1 pressure on the vertices.

Pins: tests/test_oracle_stokes3d.py -- K symmetric, A SPD, K z = 0; B
annihilates interpolated curls of cubic vector potentials; a polynomial
solution (u in P2, p in P1) is reproduced exactly; interior Vanka patch size
196; P reproduces P2 / P1 fields and R K_f P = K_c.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import combinations
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

DROP_TOL = 1e-10


# ---------------------------------------------------------------------------
# reference tetrahedron (0,0,0), (1,0,0), (0,1,0), (0,0,1)
# ---------------------------------------------------------------------------

def _exponents(k: int):
    return [(a, b, c) for t in range(k + 1) for a in range(t, -1, -1) for b in range(t - a, -1, -1)
            for c in [t - a - b]]


def multi_indices(k: int):
    """Barycentric multi-indices (a0, a1, a2, a3), sum k, descending lexicographic."""
    return [(a0, a1, a2, k - a0 - a1 - a2) for a0 in range(k, -1, -1) for a1 in range(k - a0, -1, -1)
            for a2 in range(k - a0 - a1, -1, -1)]


def node_points(k: int) -> np.ndarray:
    return np.array([[a[1] / k, a[2] / k, a[3] / k] for a in multi_indices(k)], dtype=np.float64)


def basis_coefficients(k: int) -> np.ndarray:
    ex = _exponents(k)
    X = node_points(k)
    V = np.stack([X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c for (a, b, c) in ex], axis=1)
    return np.linalg.inv(V)


def eval_basis(k: int, pts: np.ndarray):
    """phi[q, n] and reference gradients dphi[q, n, 0:3] of the nodal basis."""
    C = basis_coefficients(k)
    ex = _exponents(k)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]

    def mono(a, b, c, d):
        da, db, dc = d
        f = np.ones_like(x)
        for (p, e, dd) in ((x, a, da), (y, b, db), (z, c, dc)):
            if dd:
                if e == 0:
                    return np.zeros_like(x)
                f = f * e * p ** (e - 1)
            else:
                f = f * p ** e
        return f

    M = np.stack([mono(a, b, c, (0, 0, 0)) for (a, b, c) in ex], axis=1)
    Mx = np.stack([mono(a, b, c, (1, 0, 0)) for (a, b, c) in ex], axis=1)
    My = np.stack([mono(a, b, c, (0, 1, 0)) for (a, b, c) in ex], axis=1)
    Mz = np.stack([mono(a, b, c, (0, 0, 1)) for (a, b, c) in ex], axis=1)
    return M @ C, np.stack([Mx @ C, My @ C, Mz @ C], axis=2)


def quadrature(degree: int):
    """Collapsed (Duffy) Gauss-Legendre rule on the reference tetrahedron, exact to `degree`:
    x = a (1-b)(1-c), y = b (1-c), z = c, Jacobian (1-b)(1-c)^2."""
    n = degree // 2 + 2
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            for l in range(n):
                a, b, c = g[i], g[j], g[l]
                pts.append([a * (1 - b) * (1 - c), b * (1 - c), c])
                wts.append(w[i] * w[j] * w[l] * (1 - b) * (1 - c) ** 2)
    return np.array(pts), np.array(wts)


def p1_weights(qpts: np.ndarray) -> np.ndarray:
    return np.stack([1.0 - qpts.sum(axis=1), qpts[:, 0], qpts[:, 1], qpts[:, 2]], axis=1)


def cell_geometry(verts: np.ndarray, cell: np.ndarray):
    x0 = verts[cell[0]]
    J = np.stack([verts[cell[1]] - x0, verts[cell[2]] - x0, verts[cell[3]] - x0], axis=1)
    return x0, J, abs(np.linalg.det(J)), np.linalg.inv(J).T


# ---------------------------------------------------------------------------
# spaces
# ---------------------------------------------------------------------------

class Space3D:
    """Continuous Lagrange P1 or P2 on a tetrahedral mesh."""

    def __init__(self, verts: np.ndarray, cells: np.ndarray, k: int):
        assert k in (1, 2)
        self.k = k
        nv, nc = verts.shape[0], cells.shape[0]
        pairs = set()
        for c in cells:
            for a, b in combinations([int(v) for v in c], 2):
                pairs.add((min(a, b), max(a, b)))
        edges = sorted(pairs)
        eid = {e: i for i, e in enumerate(edges)}
        mi = multi_indices(k)
        self.nloc = len(mi)
        self.ndofs = nv + (len(edges) if k == 2 else 0)
        cd = np.zeros((nc, self.nloc), dtype=np.int64)
        for ci in range(nc):
            cv = [int(v) for v in cells[ci]]
            for n, a in enumerate(mi):
                nz = [t for t in range(4) if a[t] > 0]
                if len(nz) == 1:
                    cd[ci, n] = cv[nz[0]]
                else:
                    u, w = cv[nz[0]], cv[nz[1]]
                    cd[ci, n] = nv + eid[(min(u, w), max(u, w))]
        self.cell_dofs = cd
        ref = node_points(k)
        coords = np.zeros((self.ndofs, 3))
        for ci in range(nc):
            x0, J, _, _ = cell_geometry(verts, cells[ci])
            coords[cd[ci]] = x0 + ref @ J.T
        self.coords = coords
        # boundary: faces of exactly one cell
        count = {}
        for c in cells:
            for f in combinations(sorted(int(v) for v in c), 3):
                count[f] = count.get(f, 0) + 1
        bnd = np.zeros(self.ndofs, dtype=bool)
        for f, cnt in count.items():
            if cnt == 1:
                for v in f:
                    bnd[v] = True
                if k == 2:
                    for a, b in combinations(f, 2):
                        bnd[nv + eid[(a, b)]] = True
        self.boundary = bnd


@dataclass
class Stokes3D:
    mesh: object
    k: int
    kind: str
    V: Space3D
    Q: Space3D
    free_u: np.ndarray
    nfu: int
    nq: int
    K: sp.csr_matrix
    b: np.ndarray
    L_full: sp.csr_matrix
    B_full: list
    g: np.ndarray
    log_visc: Optional[np.ndarray] = None
    dim: int = 3

    @property
    def n(self) -> int:
        return 3 * self.nfu + self.nq

    def u_index(self, comp: int, scalar_ids: np.ndarray) -> np.ndarray:
        pos = np.full(self.V.ndofs, -1, dtype=np.int64)
        pos[self.free_u] = np.arange(self.nfu)
        out = pos[scalar_ids]
        return np.where(out >= 0, out + comp * self.nfu, -1)

    def p_index(self, q_ids) -> np.ndarray:
        return 3 * self.nfu + np.asarray(q_ids, dtype=np.int64)

    def null_vector(self) -> np.ndarray:
        z = np.zeros(self.n)
        z[3 * self.nfu:] = 1.0
        return z


def assemble(mesh, k: int = 2, forcing: Optional[Callable] = None, dirichlet: Optional[Callable] = None,
             log_visc: Optional[np.ndarray] = None) -> Stokes3D:
    """K and b on free DoFs; forcing(x,y,z) -> (fx,fy,fz), dirichlet(x,y,z) -> (gx,gy,gz)."""
    verts, cells = mesh.verts, mesh.cells
    V = Space3D(verts, cells, k)
    Q = Space3D(verts, cells, k - 1)
    qpts, qw = quadrature(2 * k)
    phi, dphi = eval_basis(k, qpts)
    psi, _ = eval_basis(k - 1, qpts)
    lam = p1_weights(qpts)
    rl, cl, vl = [], [], []
    rb, cb, vb = [], [], [[], [], []]
    F = np.zeros((3, V.ndofs))
    for c in range(cells.shape[0]):
        _, _, adet, JinvT = cell_geometry(verts, cells[c])
        grad = np.einsum("ij,qnj->qni", JinvT, dphi)
        w = qw * adet
        if log_visc is not None:
            w_l = w * (lam @ np.exp(log_visc[cells[c]]))
        else:
            w_l = w
        Lc = np.einsum("q,qai,qbi->ab", w_l, grad, grad)
        vd, qd = V.cell_dofs[c], Q.cell_dofs[c]
        rl.append(np.repeat(vd, len(vd)))
        cl.append(np.tile(vd, len(vd)))
        vl.append(Lc.ravel())
        rb.append(np.repeat(qd, len(vd)))
        cb.append(np.tile(vd, len(qd)))
        for d in range(3):
            vb[d].append((-np.einsum("q,qi,qa->ia", w, psi, grad[:, :, d])).ravel())
        if forcing is not None:
            Mc = np.einsum("q,qa,qb->ab", w, phi, phi)
            fv = forcing(V.coords[vd, 0], V.coords[vd, 1], V.coords[vd, 2])
            for d in range(3):
                F[d, vd] += Mc @ fv[d]
    nV, nQ = V.ndofs, Q.ndofs
    L = sp.csr_matrix((np.concatenate(vl), (np.concatenate(rl), np.concatenate(cl))), shape=(nV, nV))
    R, Cc = np.concatenate(rb), np.concatenate(cb)
    Bs = [sp.csr_matrix((np.concatenate(vb[d]), (R, Cc)), shape=(nQ, nV)) for d in range(3)]
    for M in [L] + Bs:
        M.sum_duplicates()
        M.sort_indices()
    free = np.flatnonzero(~V.boundary)
    bnd = np.flatnonzero(V.boundary)
    nfu = len(free)
    Lff = L[free][:, free]
    Bf = [B[:, free] for B in Bs]
    Z = sp.csr_matrix((nfu, nfu))
    K = sp.bmat([[Lff, Z, Z, Bf[0].T], [Z, Lff, Z, Bf[1].T], [Z, Z, Lff, Bf[2].T],
                 [Bf[0], Bf[1], Bf[2], sp.csr_matrix((nQ, nQ))]], format="csr")
    K.sort_indices()
    g = np.zeros((3, nV))
    if dirichlet is not None and len(bnd):
        gv = dirichlet(V.coords[bnd, 0], V.coords[bnd, 1], V.coords[bnd, 2])
        for d in range(3):
            g[d, bnd] = gv[d]
    bu = [F[d, free] - L[free][:, bnd] @ g[d, bnd] for d in range(3)]
    bp = -sum(Bs[d][:, bnd] @ g[d, bnd] for d in range(3))
    b = np.concatenate(bu + [bp])
    return Stokes3D(mesh, k, "TH", V, Q, free, nfu, nQ, K, b, L, Bs, g,
                    None if log_visc is None else np.array(log_visc, dtype=np.float64))


def interpolate(disc: Stokes3D, u: Callable, p: Optional[Callable] = None) -> np.ndarray:
    x = np.zeros(disc.n)
    cu = disc.V.coords[disc.free_u]
    uv = u(cu[:, 0], cu[:, 1], cu[:, 2])
    for d in range(3):
        x[d * disc.nfu: (d + 1) * disc.nfu] = uv[d]
    if p is not None:
        x[3 * disc.nfu:] = p(disc.Q.coords[:, 0], disc.Q.coords[:, 1], disc.Q.coords[:, 2])
    return x


def full_velocity(disc: Stokes3D, x: np.ndarray) -> np.ndarray:
    U = disc.g.copy()
    for d in range(3):
        U[d, disc.free_u] = x[d * disc.nfu: (d + 1) * disc.nfu]
    return U


# ---------------------------------------------------------------------------
# Vanka-star patches and transfers
# ---------------------------------------------------------------------------

def vanka_star_patches(disc: Stokes3D):
    """One patch per vertex: free velocity DoFs of all nodes of the cells around v (the
    closure of the star), and the pressure DoF of v (the only P1 node in the star)."""
    cells = disc.mesh.cells
    nv = disc.mesh.verts.shape[0]
    around = [[] for _ in range(nv)]
    for c in range(cells.shape[0]):
        for v in cells[c]:
            around[int(v)].append(c)
    patches = []
    for v in range(nv):
        nodes = np.unique(disc.V.cell_dofs[around[v]].ravel())
        vel = []
        for d in range(3):
            idx = disc.u_index(d, nodes)
            vel.append(idx[idx >= 0])
        dofs = np.concatenate(vel + [disc.p_index([v])])
        patches.append(np.sort(dofs))
    return patches


def _scalar_interp(fine_space: Space3D, coarse_space: Space3D, fmesh, cmesh, parent) -> sp.csr_matrix:
    k = coarse_space.k
    C = basis_coefficients(k)
    ex = _exponents(k)
    rows, cols, vals = [], [], []
    done = np.zeros(fine_space.ndofs, dtype=bool)
    for fc in range(fmesh.cells.shape[0]):
        cc = parent[fc]
        x0, J, _, _ = cell_geometry(cmesh.verts, cmesh.cells[cc])
        Jinv = np.linalg.inv(J)
        for node in fine_space.cell_dofs[fc]:
            if done[node]:
                continue
            done[node] = True
            r = Jinv @ (fine_space.coords[node] - x0)
            m = np.array([r[0] ** a * r[1] ** b * r[2] ** c for (a, b, c) in ex])
            val = m @ C
            for j, gid in enumerate(coarse_space.cell_dofs[cc]):
                if abs(val[j]) >= DROP_TOL:
                    rows.append(node)
                    cols.append(gid)
                    vals.append(val[j])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(fine_space.ndofs, coarse_space.ndofs))
    M.sum_duplicates()
    return M


def prolongation(fine: Stokes3D, coarse: Stokes3D, parent) -> sp.csr_matrix:
    """P = diag(P_u, P_u, P_u, P_p) on free DoFs: coarse basis functions at fine nodes."""
    fm, cm = fine.mesh, coarse.mesh
    Pu = _scalar_interp(fine.V, coarse.V, fm, cm, parent)[fine.free_u][:, coarse.free_u]
    Pp = _scalar_interp(fine.Q, coarse.Q, fm, cm, parent)
    P = sp.block_diag([Pu, Pu, Pu, Pp], format="csr")
    P.sort_indices()
    return P


# ---------------------------------------------------------------------------
# adjoint pieces (see adjoint.py for the method)
# ---------------------------------------------------------------------------

def _free_local(disc: Stokes3D, vd: np.ndarray, comp: int, vec: np.ndarray) -> np.ndarray:
    idx = disc.u_index(comp, vd)
    out = np.zeros(len(vd))
    m = idx >= 0
    out[m] = vec[idx[m]]
    return out


def viscosity_gradient(disc: Stokes3D, X: np.ndarray, Lam: np.ndarray) -> np.ndarray:
    verts, cells = disc.mesh.verts, disc.mesh.cells
    lv = disc.log_visc if disc.log_visc is not None else np.zeros(verts.shape[0])
    qpts, qw = quadrature(2 * disc.k)
    _, dphi = eval_basis(disc.k, qpts)
    lam = p1_weights(qpts)
    grad = np.zeros(verts.shape[0])
    U = [full_velocity(disc, x) for x in X]
    for c in range(cells.shape[0]):
        _, _, adet, JinvT = cell_geometry(verts, cells[c])
        g = np.einsum("ij,qnj->qni", JinvT, dphi)
        vd = disc.V.cell_dofs[c]
        for t in range(4):
            v = int(cells[c, t])
            At = np.exp(lv[v]) * np.einsum("q,qai,qbi->ab", qw * adet * lam[:, t], g, g)
            s = 0.0
            for b in range(X.shape[0]):
                for comp in range(3):
                    s += _free_local(disc, vd, comp, Lam[b]) @ (At @ U[b][comp, vd])
            grad[v] -= s
    return grad


def forcing_gradient(disc: Stokes3D, Lam: np.ndarray) -> np.ndarray:
    verts, cells = disc.mesh.verts, disc.mesh.cells
    qpts, qw = quadrature(2 * disc.k)
    phi, _ = eval_basis(disc.k, qpts)
    out = np.zeros((Lam.shape[0], 3, disc.V.ndofs))
    for c in range(cells.shape[0]):
        _, _, adet, _ = cell_geometry(verts, cells[c])
        Mc = np.einsum("q,qa,qb->ab", qw * adet, phi, phi)
        vd = disc.V.cell_dofs[c]
        for b in range(Lam.shape[0]):
            for comp in range(3):
                out[b, comp, vd] += Mc.T @ _free_local(disc, vd, comp, Lam[b])
    return out


def forcing_rhs(disc: Stokes3D, f_nodal: np.ndarray) -> np.ndarray:
    verts, cells = disc.mesh.verts, disc.mesh.cells
    qpts, qw = quadrature(2 * disc.k)
    phi, _ = eval_basis(disc.k, qpts)
    full = np.zeros((f_nodal.shape[0], 3, disc.V.ndofs))
    for c in range(cells.shape[0]):
        _, _, adet, _ = cell_geometry(verts, cells[c])
        Mc = np.einsum("q,qa,qb->ab", qw * adet, phi, phi)
        vd = disc.V.cell_dofs[c]
        for b in range(f_nodal.shape[0]):
            for comp in range(3):
                full[b, comp, vd] += Mc @ f_nodal[b, comp, vd]
    out = np.zeros((f_nodal.shape[0], disc.n))
    for comp in range(3):
        out[:, comp * disc.nfu: (comp + 1) * disc.nfu] = full[:, comp, disc.free_u]
    return out
