"""Host front-end: builds the inputs of the C ABI from a mesh hierarchy.

It discretises the Stokes problem of Section 2 (eq. "eq:stokes-disc",
"eq:saddle") with Taylor-Hood P_k/P_{k-1} or Scott-Vogelius
P_k/P_{k-1}^disc elements (Section 2.1), builds the Vanka-star patch lists
(Section 3.4, figure "fig:patches") and the finite-element interpolation
transfers (Sections 3.1-3.2), all as flat arrays in the canonical numbering:

  global order [u_x | u_y | p] over free DoFs; inside a continuous scalar
  field vertex DoFs by vertex id, edge DoFs by edge id (edges = sorted vertex
  pairs in lexicographic order, nodes from the lower to the higher vertex id),
  then cell-interior DoFs by cell, ascending lexicographic barycentric index;
  discontinuous pressure cell by cell.

This is set-up code on the host (not the timed path).  It is vectorised over
cells and uses its own route: barycentric (Silvester) Lagrange products for
the basis and Gauss-Jacobi collapsed quadrature.  Every solver step runs in
the HIP library; nothing here calls it.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp
from scipy.special import roots_jacobi

import synth

# --------------------------------------------------------------------------
# reference element
# --------------------------------------------------------------------------


@lru_cache(maxsize=None)
def lattice(k: int) -> np.ndarray:
    """Barycentric multi-indices of degree k, ascending lexicographic, shape (nloc, 3)."""
    rows = [(a, b, k - a - b) for a in range(k + 1) for b in range(k + 1 - a)]
    return np.array(rows, dtype=np.int64)


def barycentric(ref: np.ndarray) -> np.ndarray:
    return np.stack([1.0 - ref[..., 0] - ref[..., 1], ref[..., 0], ref[..., 1]], axis=-1)


_DLAM = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])   # d lambda_t / d (xi, eta)


def shape_functions(k: int, ref: np.ndarray):
    """Silvester form phi_a = prod_t prod_{s<a_t} (k lam_t - s)/(s+1); values and reference gradients.

    ref: (..., 2).  Returns phi (..., nloc) and dphi (..., nloc, 2).
    """
    lam = barycentric(ref)
    A = lattice(k)
    if k == 0:
        shp = ref.shape[:-1]
        return np.ones(shp + (1,)), np.zeros(shp + (1, 2))
    # per barycentric direction t and order a: value and derivative of the 1D factor
    fac = np.ones(lam.shape[:-1] + (3, k + 1))
    dfac = np.zeros(lam.shape[:-1] + (3, k + 1))
    for a in range(1, k + 1):
        term = (k * lam - (a - 1)) / a
        fac[..., :, a] = fac[..., :, a - 1] * term
        dfac[..., :, a] = dfac[..., :, a - 1] * term + fac[..., :, a - 1] * (k / a)
    vals = [fac[..., t, A[:, t]] for t in range(3)]                 # (..., nloc) each
    ders = [dfac[..., t, A[:, t]] for t in range(3)]
    phi = vals[0] * vals[1] * vals[2]
    dphi_dlam = np.stack([ders[0] * vals[1] * vals[2], vals[0] * ders[1] * vals[2], vals[0] * vals[1] * ders[2]], axis=-1)
    dphi = dphi_dlam @ _DLAM
    return phi, dphi


@lru_cache(maxsize=None)
def collapsed_rule(degree: int):
    """Gauss-Jacobi(1,0) x Gauss-Legendre rule on the reference triangle, exact to `degree`."""
    n = degree // 2 + 1
    xl, wl = np.polynomial.legendre.leggauss(n)
    xj, wj = roots_jacobi(n, 1.0, 0.0)
    s = 0.5 * (xl + 1.0)
    t = 0.5 * (xj + 1.0)
    S, T = np.meshgrid(s, t, indexing="ij")
    W = np.outer(wl, wj) * 0.125
    pts = np.stack([(S * (1.0 - T)).ravel(), T.ravel()], axis=1)
    return pts, W.ravel()


# --------------------------------------------------------------------------
# DoF maps
# --------------------------------------------------------------------------


@dataclass
class Space:
    k: int
    continuous: bool
    cell_dofs: np.ndarray   # (nc, nloc)
    ndofs: int
    coords: np.ndarray      # (ndofs, 2)
    boundary: np.ndarray    # bool (ndofs,)
    entity_verts: np.ndarray  # (nloc, 3) bool: local vertices spanning the node's entity


def _edges(cells: np.ndarray):
    loc = np.array([[0, 1], [1, 2], [2, 0]])
    pairs = np.sort(cells[:, loc], axis=2)                    # nc x 3 x 2
    uniq, inv, cnt = np.unique(pairs.reshape(-1, 2), axis=0, return_inverse=True, return_counts=True)
    return uniq, inv.reshape(-1, 3), cnt


def _local_edge(t1: int, t2: int) -> int:
    return {(0, 1): 0, (1, 2): 1, (0, 2): 2}[(min(t1, t2), max(t1, t2))]


def build_space(mesh, k: int, continuous: bool) -> Space:
    verts, cells = mesh.verts, mesh.cells
    nv, nc = verts.shape[0], cells.shape[0]
    A = lattice(k)
    nloc = A.shape[0]
    ent = A > 0
    x0 = verts[cells[:, 0]]
    J = np.stack([verts[cells[:, 1]] - x0, verts[cells[:, 2]] - x0], axis=2)    # nc x 2 x 2
    ref = A[:, 1:] / k if k > 0 else np.array([[1.0 / 3, 1.0 / 3]])
    node_xy = x0[:, None, :] + np.einsum("cij,nj->cni", J, ref)
    if not continuous:
        cd = np.arange(nc * nloc, dtype=np.int64).reshape(nc, nloc)
        return Space(k, False, cd, nc * nloc, node_xy.reshape(-1, 2), np.zeros(nc * nloc, bool), ent)
    edges, cell_edges, counts = _edges(cells)
    ne = edges.shape[0]
    interior = np.flatnonzero(ent.all(axis=1))
    nint = interior.size
    cd = np.zeros((nc, nloc), dtype=np.int64)
    for n in range(nloc):
        nz = np.flatnonzero(A[n])
        if nz.size == 1:
            cd[:, n] = cells[:, nz[0]]
        elif nz.size == 2:
            t1, t2 = nz
            eid = cell_edges[:, _local_edge(t1, t2)]
            a_hi = np.where(cells[:, t1] > cells[:, t2], A[n, t1], A[n, t2])
            cd[:, n] = nv + eid * (k - 1) + a_hi - 1
        else:
            q = int(np.searchsorted(interior, n))
            cd[:, n] = nv + ne * (k - 1) + np.arange(nc) * nint + q
    ndofs = nv + ne * (k - 1) + nc * nint
    coords = np.zeros((ndofs, 2))
    coords[cd.ravel()] = node_xy.reshape(-1, 2)
    bnd = np.zeros(ndofs, dtype=bool)
    be = np.flatnonzero(counts == 1)
    bnd[edges[be].ravel()] = True
    if k > 1:
        bnd[(nv + be[:, None] * (k - 1) + np.arange(k - 1)[None, :]).ravel()] = True
    return Space(k, True, cd, ndofs, coords, bnd, ent)


# --------------------------------------------------------------------------
# assembly
# --------------------------------------------------------------------------


@dataclass
class Csr:
    rowptr: np.ndarray   # int32 (nrows+1)
    col: np.ndarray      # int32 (nnz)
    val: np.ndarray      # float64 (nnz)
    nrows: int
    ncols: int

    @classmethod
    def from_scipy(cls, M) -> "Csr":
        M = sp.csr_matrix(M)
        M.sum_duplicates()
        M.sort_indices()
        if M.nnz >= 2 ** 31:
            raise ValueError("nnz exceeds int32 indexing")
        return cls(M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64),
                   M.shape[0], M.shape[1])

    def to_scipy(self):
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.nrows, self.ncols))

    @property
    def nnz(self) -> int:
        return int(self.col.size)


@dataclass
class LevelData:
    k: int
    kind: str
    V: Space
    Q: Space
    nfu: int
    nq: int
    free_u: np.ndarray
    K: Csr
    mesh_index: int
    patch_ptr: Optional[np.ndarray] = None     # int64 (npatch+1)
    patch_dofs: Optional[np.ndarray] = None    # int32 (sum m)
    patch_weight: Optional[np.ndarray] = None  # float64 (sum m)
    P: Optional[Csr] = None                    # prolongation from the next coarser level to this one
    b: Optional[np.ndarray] = None
    mesh: object = None
    log_visc: Optional[np.ndarray] = None       # nodal log-viscosity at the mesh vertices (None: nu = 1)
    visc_sens: Optional[Csr] = None             # (nv x nnz(K)): d K_e / d l_v, e over K's nonzeros
    forcing_map: Optional[Csr] = None           # (n x d nV): free right-hand side of nodal forcing values
    dim: int = 2

    @property
    def n(self) -> int:
        return self.dim * self.nfu + self.nq

    def null_vector(self) -> np.ndarray:
        z = np.zeros(self.n)
        z[self.dim * self.nfu:] = 1.0
        return z


def _geometry(mesh):
    v, c = mesh.verts, mesh.cells
    x0 = v[c[:, 0]]
    J = np.stack([v[c[:, 1]] - x0, v[c[:, 2]] - x0], axis=2)
    det = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    Jinv = np.stack([np.stack([J[:, 1, 1], -J[:, 0, 1]], 1), np.stack([-J[:, 1, 0], J[:, 0, 0]], 1)], 1) / det[:, None, None]
    return x0, J, np.abs(det), Jinv


def assemble_level(mesh, k: int, kind: str, forcings: Optional[List[Callable]] = None,
                   dirichlet: Optional[Callable] = None, mesh_index: int = 0,
                   log_visc: Optional[np.ndarray] = None, sensitivities: bool = False) -> LevelData:
    """log_visc: nodal log-viscosity l at the mesh vertices; the velocity block is then
    int nu_h grad u : grad v with nu_h = sum_v exp(l_v) lambda_v (P1 interpolant of exp(l)),
    integrated exactly (rule of degree 2k - 1).  sensitivities: also build dK/dl (as a
    vertex x nonzero matrix) and the forcing map for the adjoint gradients."""
    V = build_space(mesh, k, True)
    Q = build_space(mesh, k - 1, kind == "TH")
    x0, J, adet, Jinv = _geometry(mesh)
    if log_visc is None:
        pts, w = collapsed_rule(2 * k - 2 if k > 1 else 1)
    else:
        pts, w = collapsed_rule(2 * k - 1)
    _, dphi = shape_functions(k, pts)                      # nq x nv x 2
    psi, _ = shape_functions(k - 1, pts)                   # nq x np
    g = np.einsum("qnj,cji->cqni", dphi, Jinv)             # physical gradients, nc x nq x nloc x 2
    wc = adet[:, None] * w[None, :]
    Lt = None
    if log_visc is None:
        Le = np.einsum("cq,cqai,cqbi->cab", wc, g, g)
    else:
        # hat-weighted stiffness per cell vertex t: int lambda_t grad phi_a . grad phi_b
        Lt = np.einsum("cq,qt,cqai,cqbi->ctab", wc, barycentric(pts), g, g)
        ev = np.exp(np.asarray(log_visc, dtype=np.float64)[mesh.cells])      # nc x 3
        Le = np.einsum("ct,ctab->cab", ev, Lt)
    Bxe = -np.einsum("cq,qi,cqa->cia", wc, psi, g[..., 0])
    Bye = -np.einsum("cq,qi,cqa->cia", wc, psi, g[..., 1])
    vd, qd = V.cell_dofs, Q.cell_dofs
    nl, ql = vd.shape[1], qd.shape[1]
    L = sp.coo_matrix((Le.ravel(), (np.repeat(vd, nl, axis=1).ravel(), np.tile(vd, (1, nl)).ravel())),
                      shape=(V.ndofs, V.ndofs)).tocsr()
    ri = np.repeat(qd, nl, axis=1).ravel()
    ci = np.tile(vd, (1, ql)).ravel()
    Bx = sp.coo_matrix((Bxe.ravel(), (ri, ci)), shape=(Q.ndofs, V.ndofs)).tocsr()
    By = sp.coo_matrix((Bye.ravel(), (ri, ci)), shape=(Q.ndofs, V.ndofs)).tocsr()
    free = np.flatnonzero(~V.boundary)
    bnd = np.flatnonzero(V.boundary)
    nfu = free.size
    Lff = L[free][:, free]
    Bxf, Byf = Bx[:, free], By[:, free]
    K = sp.bmat([[Lff, None, Bxf.T], [None, Lff, Byf.T], [Bxf, Byf, sp.csr_matrix((Q.ndofs, Q.ndofs))]], format="csr")
    lev = LevelData(k, kind, V, Q, nfu, Q.ndofs, free, Csr.from_scipy(K), mesh_index, mesh=mesh,
                    log_visc=None if log_visc is None else np.asarray(log_visc, dtype=np.float64))
    if sensitivities:
        lev.visc_sens = _viscosity_sensitivity(lev, mesh, Lt)
        lev.forcing_map = _forcing_map(lev, mesh, adet)
    if forcings is not None:
        # F(v) = int (I_h f).v: nodal interpolant of f times the exact element mass matrix
        mpts, mw = collapsed_rule(2 * k)
        mphi, _ = shape_functions(k, mpts)
        Me = np.einsum("c,q,qa,qb->cab", adet, mw, mphi, mphi)
        xn = V.coords[vd]                                   # nc x nloc x 2
        gx = np.zeros(V.ndofs)
        gy = np.zeros(V.ndofs)
        if dirichlet is not None and bnd.size:
            gx[bnd], gy[bnd] = dirichlet(V.coords[bnd, 0], V.coords[bnd, 1])
        lift_x = L[free][:, bnd] @ gx[bnd]
        lift_y = L[free][:, bnd] @ gy[bnd]
        lift_p = Bx[:, bnd] @ gx[bnd] + By[:, bnd] @ gy[bnd]
        rhs = []
        for f in forcings:
            fx, fy = f(xn[..., 0], xn[..., 1])
            Fx = np.zeros(V.ndofs)
            Fy = np.zeros(V.ndofs)
            np.add.at(Fx, vd, np.einsum("cab,cb->ca", Me, fx))
            np.add.at(Fy, vd, np.einsum("cab,cb->ca", Me, fy))
            rhs.append(np.concatenate([Fx[free] - lift_x, Fy[free] - lift_y, -lift_p]))
        lev.b = np.stack(rhs, axis=0)
    return lev


def _viscosity_sensitivity(lev: LevelData, mesh, Lt) -> Csr:
    """S[v, e] = d K_e / d l_v over the nonzeros e of K (CSR order): exp(l_v) times the
    hat-weighted stiffness of vertex v, in both velocity blocks."""
    nv = mesh.verts.shape[0]
    K = lev.K
    n, nfu = K.nrows, lev.nfu
    if Lt is None:
        raise ValueError("the viscosity sensitivity needs a log-viscosity field")
    keys = np.repeat(np.arange(n, dtype=np.int64), np.diff(K.rowptr)) * n + K.col
    pos = -np.ones(lev.V.ndofs, dtype=np.int64)
    pos[lev.free_u] = np.arange(nfu)
    fi = pos[lev.V.cell_dofs]                                             # nc x nl (-1 fixed)
    ev = np.exp(lev.log_visc[mesh.cells])                                 # nc x 3
    nl = fi.shape[1]
    rows, cols, vals = [], [], []
    I = np.repeat(fi[:, :, None], nl, axis=2)
    Jc = np.repeat(fi[:, None, :], nl, axis=1)
    ok = (I >= 0) & (Jc >= 0)
    for t in range(3):
        val = (ev[:, t, None, None] * Lt[:, t])[ok]
        vtx = np.broadcast_to(mesh.cells[:, t, None, None], I.shape)[ok]
        for comp in range(2):
            key = (I[ok] + comp * nfu) * n + (Jc[ok] + comp * nfu)
            e = np.searchsorted(keys, key)
            assert np.array_equal(keys[e], key)
            rows.append(vtx)
            cols.append(e)
            vals.append(val)
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nv, K.nnz)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return Csr.from_scipy(S)


def _forcing_map(lev: LevelData, mesh, adet) -> Csr:
    """G (n x 2 nV): b = G f for nodal forcing values f = [f_x; f_y] at every velocity node
    (F(v) = int (I_h f) . v with the exact mass matrix; homogeneous Dirichlet data)."""
    k = lev.k
    mpts, mw = collapsed_rule(2 * k)
    mphi, _ = shape_functions(k, mpts)
    Me = np.einsum("c,q,qa,qb->cab", adet, mw, mphi, mphi)
    vd = lev.V.cell_dofs
    nl = vd.shape[1]
    nV = lev.V.ndofs
    M = sp.coo_matrix((Me.ravel(), (np.repeat(vd, nl, axis=1).ravel(), np.tile(vd, (1, nl)).ravel())),
                      shape=(nV, nV)).tocsr()
    Mf = M[lev.free_u]
    G = sp.bmat([[Mf, None], [None, Mf], [sp.csr_matrix((lev.nq, nV)), sp.csr_matrix((lev.nq, nV))]],
                format="csr")
    G.sum_duplicates()
    G.sort_indices()
    return Csr.from_scipy(G)


# --------------------------------------------------------------------------
# Vanka-star patches
# --------------------------------------------------------------------------


def vanka_patches(lev: LevelData):
    """One patch per vertex: velocity DoFs of closure(star v), pressure DoFs of star v."""
    mesh = lev.mesh
    cells = mesh.cells
    nv, nc = mesh.nv, mesh.nc
    order = np.argsort(cells.ravel(), kind="stable")
    cell_of = order // 3
    vptr = np.zeros(nv + 1, dtype=np.int64)
    np.add.at(vptr, cells.ravel() + 1, 1)
    vptr = np.cumsum(vptr)
    upos = np.full(lev.V.ndofs, -1, dtype=np.int64)
    upos[lev.free_u] = np.arange(lev.nfu)
    ent = lev.Q.entity_verts                    # (nlocq, 3)
    out = []
    for v in range(nv):
        cs = cell_of[vptr[v]:vptr[v + 1]]
        if cs.size == 0:
            continue
        vel = upos[np.unique(lev.V.cell_dofs[cs])]
        vel = vel[vel >= 0]
        if lev.Q.continuous:
            at_v = cells[cs] == v                                # (ncs, 3)
            inside = (at_v[:, None, :] & ent[None, :, :]).any(axis=2)   # node entity contains v
            prs = np.unique(lev.Q.cell_dofs[cs][inside])
        else:
            prs = np.unique(lev.Q.cell_dofs[cs])
        dofs = np.concatenate([vel, vel + lev.nfu, 2 * lev.nfu + prs])
        if dofs.size:
            out.append(np.sort(dofs))
    ptr = np.zeros(len(out) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([p.size for p in out])
    dofs = np.concatenate(out).astype(np.int32)
    mult = np.bincount(dofs, minlength=lev.n).astype(np.float64)
    weight = 1.0 / mult[dofs]
    return ptr, dofs, weight


# --------------------------------------------------------------------------
# transfers
# --------------------------------------------------------------------------


def _interp_entries(fine: Space, coarse: Space, fmesh, cmesh, parent):
    nc_f = fmesh.nc
    cc = np.arange(nc_f) if parent is None else parent
    x0, _, _, Jinv = _geometry(cmesh)
    fd = fine.cell_dofs
    pts = fine.coords[fd]                                   # ncf x nlf x 2
    ref = np.einsum("cij,cnj->cni", Jinv[cc], pts - x0[cc][:, None, :])
    phi, _ = shape_functions(coarse.k, ref)                 # ncf x nlf x nlc
    cdofs = coarse.cell_dofs[cc]                            # ncf x nlc
    rows = np.broadcast_to(fd[:, :, None], phi.shape).ravel()
    cols = np.broadcast_to(cdofs[:, None, :], phi.shape).ravel()
    vals = phi.ravel()
    key = rows * coarse.ndofs + cols
    _, first = np.unique(key, return_index=True)
    return rows[first], cols[first], vals[first]


# basis values at lattice points are either exact zeros (computed to ~1e-14 on
# distorted cells) or rationals of magnitude >= 1/32
ZERO_TOL = 1e-10


def prolongation(fine: LevelData, coarse: LevelData, parent) -> Csr:
    fm, cm = fine.mesh, coarse.mesh
    fpos = np.full(fine.V.ndofs, -1, dtype=np.int64)
    fpos[fine.free_u] = np.arange(fine.nfu)
    cpos = np.full(coarse.V.ndofs, -1, dtype=np.int64)
    cpos[coarse.free_u] = np.arange(coarse.nfu)
    r, c, v = _interp_entries(fine.V, coarse.V, fm, cm, parent)
    keep = (fpos[r] >= 0) & (cpos[c] >= 0) & (np.abs(v) >= ZERO_TOL)
    r, c, v = fpos[r[keep]], cpos[c[keep]], v[keep]
    rq, cq, vq = _interp_entries(fine.Q, coarse.Q, fm, cm, parent)
    keep = np.abs(vq) >= ZERO_TOL
    rq, cq, vq = rq[keep], cq[keep], vq[keep]
    rows = np.concatenate([r, r + fine.nfu, 2 * fine.nfu + rq])
    cols = np.concatenate([c, c + coarse.nfu, 2 * coarse.nfu + cq])
    vals = np.concatenate([v, v, vq])
    P = sp.csr_matrix((vals, (rows, cols)), shape=(fine.n, coarse.n))
    return Csr.from_scipy(P)


# --------------------------------------------------------------------------
# hierarchies of the benchmark workloads
# --------------------------------------------------------------------------


@dataclass
class Hierarchy:
    name: str
    levels: List[LevelData]
    opts: dict = field(default_factory=dict)
    weights: bool = True          # pass the partition-of-unity W_i (False: W_i = I)

    @property
    def b(self) -> np.ndarray:
        return self.levels[0].b


SEEDS = {"cfg1": 1, "cfg2": 2, "cfg3": 3, "cfg4": 4, "cfg5": 5, "cube": 5}


def p_schedule(k: int) -> List[int]:
    """Velocity orders of gradual p-coarsening (Section 4, figure "fig:pmg_schedule"):
    k <= 5 goes to P2 in one step, k = 6, 7 through P4, k = 8..10 through P5."""
    if k <= 2:
        return [2]
    if k <= 5:
        return [k, 2]
    if k <= 7:
        return [k, 4, 2]
    if k <= 10:
        return [k, 5, 2]
    raise ValueError(f"no schedule for order {k}")


def workload_specs(name: str, k: Optional[int] = None, schedule: str = "direct"):
    """Levels as (mesh index from the finest, order, kind), the cycle options and the weight choice.

    cfg1 names its smoother (nu = 2 damped sweeps, omega = 0.5): Richardson
    with the partition-of-unity weights.  The other workloads name none and use
    the paper's: Chebyshev acceleration (nu = 2) of the basic additive Schwarz
    operator (W_i = I) over [0.1, 1.1] * lambda_max.
    """
    cheb = dict(smoother="chebyshev", cheb_lo=0.1, cheb_hi=1.1, eig_iters=20)
    if name in ("cfg1", "tiny2", "tiny4"):
        return [(0, 2, "TH"), (1, 2, "TH")], dict(nu_p=2, nu_h=2, n_v=1, n_plevels=0, omega=0.5), True
    if name.startswith("cfg2") or name.startswith("cfg3"):
        nref = {"cfg2": 3, "cfg2_r2": 2, "cfg2_r1": 1, "cfg3": 4, "cfg3_r2": 2, "cfg3_r1": 1, "cfg3_r0": 0}[name]
        kk = 4 if k is None else k
        orders = p_schedule(kk) if schedule == "gradual" else ([kk, 2] if kk != 2 else [2])
        specs = [(0, o, "TH") for o in orders[:-1]] + [(i, 2, "TH") for i in range(nref + 1)]
        return specs, dict(nu_p=2, nu_h=2, n_v=1, n_plevels=len(orders) - 1, omega=0.5, **cheb), False
    if name in ("cfg4", "cfg4_r0", "sv_small"):
        nmac = {"cfg4": 3, "cfg4_r0": 1, "sv_small": 2}[name]
        kk = 4 if k is None else k
        specs = [(0, kk, "SV"), (0, 2, "TH")] + [(i, 2, "TH") for i in range(1, nmac + 1)]
        return specs, dict(nu_p=2, nu_h=2, n_v=1, n_plevels=1, omega=0.5, **cheb), False
    raise KeyError(name)


def build_hierarchy(name: str, k: Optional[int] = None, forcing: str = "mms", nrhs: int = 1,
                    specs=None, opts=None, log_visc: Optional[np.ndarray] = None,
                    sensitivities: bool = False, schedule: str = "direct") -> Hierarchy:
    """log_visc: nodal log-viscosity on the finest mesh's vertices, injected to the vertices
    of every coarser (nested) mesh; sensitivities: level 0 also carries dK/dl and the
    forcing map (adjoint gradients)."""
    meshes = synth.config_mesh_hierarchy(name)[::-1]       # finest first
    if meshes[0].meta.get("dim") == 3:
        from . import frontend3d
        return frontend3d.build_hierarchy(name, meshes, forcing, nrhs, log_visc, sensitivities)
    weights = True
    if specs is None:
        specs, opts, weights = workload_specs(name, k, schedule)
    seed = SEEDS.get(name.split("_")[0], 1)
    if forcing == "mms":
        A = synth.mms_amplitude(seed)
        fs = [lambda x, y: synth.mms_forcing(x, y, A)]
        g = lambda x, y: synth.mms_velocity(x, y, A)
    elif forcing == "bumps":
        C, Wd, D = synth.gaussian_bump_params(nrhs, seed)
        fs = [(lambda x, y, i=i: synth.gaussian_bump_forcing(x, y, C[i], Wd[i], D[i])) for i in range(nrhs)]
        g = None
    else:
        fs, g = None, None
    levels: List[LevelData] = []
    for li, (mi, kk, kind) in enumerate(specs):
        lv = None
        if log_visc is not None:
            nvl = meshes[mi].verts.shape[0]
            assert np.array_equal(meshes[mi].verts, meshes[0].verts[:nvl])
            lv = np.asarray(log_visc, dtype=np.float64)[:nvl]
        lev = assemble_level(meshes[mi], kk, kind, forcings=fs if li == 0 else None,
                             dirichlet=g if li == 0 else None, mesh_index=mi, log_visc=lv,
                             sensitivities=sensitivities and li == 0)
        if li < len(specs) - 1:
            lev.patch_ptr, lev.patch_dofs, lev.patch_weight = vanka_patches(lev)
        if li > 0:
            fine = levels[li - 1]
            parent = None if fine.mesh_index == mi else meshes[fine.mesh_index].parent
            lev.P = prolongation(fine, lev, parent)
        levels.append(lev)
    return Hierarchy(name, levels, dict(opts), weights)


# --------------------------------------------------------------------------
# full block factorisation (Section 3.3, eq. "eq:fbf")
# --------------------------------------------------------------------------


def star_patches(lev: LevelData):
    """Velocity-only vertex-star patches (the ASMStarPC patches of Section 3.4): the free
    velocity DoFs of the entities of star(v) -- v itself, the edges and the cells around v --
    both components; one patch per vertex with any such DoF."""
    mesh = lev.mesh
    cells = mesh.cells
    nv = mesh.nv
    order = np.argsort(cells.ravel(), kind="stable")
    cell_of = order // 3
    vptr = np.zeros(nv + 1, dtype=np.int64)
    np.add.at(vptr, cells.ravel() + 1, 1)
    vptr = np.cumsum(vptr)
    upos = np.full(lev.V.ndofs, -1, dtype=np.int64)
    upos[lev.free_u] = np.arange(lev.nfu)
    ent = lev.V.entity_verts
    out = []
    for v in range(nv):
        cs = cell_of[vptr[v]:vptr[v + 1]]
        if cs.size == 0:
            continue
        at_v = cells[cs] == v
        inside = (at_v[:, None, :] & ent[None, :, :]).any(axis=2)
        vel = upos[np.unique(lev.V.cell_dofs[cs][inside])]
        vel = vel[vel >= 0]
        if vel.size:
            out.append(np.concatenate([vel, vel + lev.nfu]))
    ptr = np.zeros(len(out) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([p.size for p in out])
    return ptr, np.concatenate(out).astype(np.int32)


def pressure_mass_inverse(lev: LevelData) -> Csr:
    """-M_p^{-1} for a discontinuous pressure space: the cell blocks of the pressure mass
    matrix inverted cell by cell, with the sign of the Schur complement -B A^{-1} B^T."""
    if lev.Q.continuous:
        raise ValueError("the block-diagonal pressure mass inverse needs a discontinuous pressure space")
    kq = lev.k - 1
    pts, w = collapsed_rule(2 * kq)
    psi, _ = shape_functions(kq, pts)
    _, _, adet, _ = _geometry(lev.mesh)
    Mref = np.einsum("q,qa,qb->ab", w, psi, psi)
    inv = -np.linalg.inv(Mref)[None, :, :] / adet[:, None, None]          # (nc, nq, nq)
    qd = lev.Q.cell_dofs
    nl = qd.shape[1]
    S = sp.coo_matrix((inv.ravel(), (np.repeat(qd, nl, axis=1).ravel(), np.tile(qd, (1, nl)).ravel())),
                      shape=(lev.nq, lev.nq)).tocsr()
    S.sort_indices()
    return Csr.from_scipy(S)


def fbf_inputs(fh: Hierarchy) -> dict:
    """Inputs of the FBF preconditioner for a Scott-Vogelius hierarchy: the velocity blocks
    A_l of every level with star patches and the velocity parts of the transfers (the phMG
    hierarchy on A), and K_0, B_0 and S~^{-1} = -M_p^{-1} of the finest level."""
    A, P, patches = [], [], []
    for li, lev in enumerate(fh.levels):
        nu = 2 * lev.nfu
        K = lev.K.to_scipy()
        A.append(Csr.from_scipy(K[:nu, :nu].tocsr()))
        if li > 0:
            nuf = 2 * fh.levels[li - 1].nfu
            P.append(Csr.from_scipy(lev.P.to_scipy()[:nuf, :nu].tocsr()))
        if li < len(fh.levels) - 1:
            ptr, dofs = star_patches(lev)
            patches.append((ptr, dofs, None))
    L0 = fh.levels[0]
    nu0 = 2 * L0.nfu
    K0 = L0.K.to_scipy()
    B = K0[nu0:, :nu0].tocsr()
    B.sort_indices()
    return dict(A=A, P=P, patches=patches, K=L0.K, B=Csr.from_scipy(B), S_inv=pressure_mass_inverse(L0),
                opts=dict(fh.opts))
