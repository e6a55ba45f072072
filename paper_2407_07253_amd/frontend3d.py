"""Host front-end for 3D Taylor-Hood P2/P1 on tetrahedral (Kuhn cube) meshes.

The 3D counterpart of frontend.py: the Stokes weak form of Section 2 with
continuous P2 velocity / P1 pressure, the Vanka-star patches of Section 3.4
(velocity DoFs of the closure of each vertex star, the vertex's pressure
DoF) and finite-element interpolation transfers (Section 3.1), flattened into
the C ABI's inputs in the canonical numbering [u_x | u_y | u_z | p] over free
DoFs (vertices by id, then edges by id, edges being the sorted vertex pairs
in lexicographic order; P1 pressure on the vertices).

Vectorised over cells with its own route: Silvester products of the four
barycentric coordinates for the basis and the Stroud conical product
(Gauss-Jacobi(2,0) x Gauss-Jacobi(1,0) x Gauss-Legendre) for quadrature.
Set-up code on the host; it never calls the library.
"""
from __future__ import annotations

from functools import lru_cache
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
from scipy.special import roots_jacobi

import synth

from .frontend import ZERO_TOL, Csr, Hierarchy, LevelData


@lru_cache(maxsize=None)
def lattice4(k: int) -> np.ndarray:
    """Barycentric multi-indices of degree k in 4 coordinates, ascending lexicographic."""
    rows = [(a, b, c, k - a - b - c) for a in range(k + 1) for b in range(k + 1 - a) for c in range(k + 1 - a - b)]
    return np.array(rows, dtype=np.int64)


def bary4(ref: np.ndarray) -> np.ndarray:
    return np.concatenate([1.0 - ref.sum(axis=-1, keepdims=True), ref], axis=-1)


_DLAM = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def shape_functions(k: int, ref: np.ndarray):
    """phi_a = prod_t prod_{s < a_t} (k lam_t - s) / (s + 1): values (nq, nloc), gradients (nq, nloc, 3)."""
    lam = bary4(ref)
    L = lattice4(k)
    nq, nloc = ref.shape[0], L.shape[0]
    val = np.ones((nq, nloc))
    grad = np.zeros((nq, nloc, 3))
    for a in range(nloc):
        factors, dfactors = [], []
        for t in range(4):
            for s_ in range(L[a, t]):
                factors.append((k * lam[:, t] - s_) / (s_ + 1))
                dfactors.append(np.outer(np.full(nq, k / (s_ + 1)), _DLAM[t]))
        for i, f in enumerate(factors):
            val[:, a] *= f
            g = dfactors[i]
            for j, f2 in enumerate(factors):
                if j != i:
                    g = g * f2[:, None]
            grad[:, a] += g
    return val, grad


@lru_cache(maxsize=None)
def conical_rule(degree: int):
    """Stroud conical product rule on the reference tetrahedron, exact to `degree`."""
    n = degree // 2 + 1
    xa, wa = roots_jacobi(n, 2.0, 0.0)
    xb, wb = roots_jacobi(n, 1.0, 0.0)
    xc, wc = np.polynomial.legendre.leggauss(n)
    a = 0.5 * (xa + 1.0)
    b = 0.5 * (xb + 1.0)
    c = 0.5 * (xc + 1.0)
    A, B, Cc = np.meshgrid(a, b, c, indexing="ij")
    W = np.einsum("i,j,l->ijl", wa / 8.0, wb / 4.0, wc / 2.0)
    z = A
    y = B * (1.0 - A)
    x = Cc * (1.0 - A) * (1.0 - B)
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1), W.ravel()


class Space3:
    """Continuous P1 / P2 on a tetrahedral mesh (vertex and edge DoFs)."""

    def __init__(self, mesh, k: int):
        verts, cells = mesh.verts, mesh.cells
        nv, nc = verts.shape[0], cells.shape[0]
        L = lattice4(k)
        self.k = k
        pairs = np.sort(cells[:, [[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]]], axis=2).reshape(-1, 2)
        edges, inv = np.unique(pairs, axis=0, return_inverse=True)
        cell_edges = inv.reshape(nc, 6)
        local_edge = {(0, 1): 0, (0, 2): 1, (0, 3): 2, (1, 2): 3, (1, 3): 4, (2, 3): 5}
        cd = np.zeros((nc, L.shape[0]), dtype=np.int64)
        for a, row in enumerate(L):
            nz = np.flatnonzero(row)
            if len(nz) == 1:
                cd[:, a] = cells[:, nz[0]]
            else:
                cd[:, a] = nv + cell_edges[:, local_edge[(nz[0], nz[1])]]
        self.cell_dofs = cd
        self.ndofs = nv + (edges.shape[0] if k == 2 else 0)
        ref = L[:, 1:] / k
        x0 = verts[cells[:, 0]]
        J = np.stack([verts[cells[:, 1]] - x0, verts[cells[:, 2]] - x0, verts[cells[:, 3]] - x0], axis=2)
        coords = np.zeros((self.ndofs, 3))
        coords[cd] = x0[:, None, :] + np.einsum("cij,aj->cai", J, ref)
        self.coords = coords
        faces = np.sort(cells[:, [[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]], axis=2).reshape(-1, 3)
        uf, cnt = np.unique(faces, axis=0, return_counts=True)
        bf = uf[cnt == 1]
        bnd = np.zeros(self.ndofs, dtype=bool)
        bnd[bf.ravel()] = True
        if k == 2:
            fe = np.sort(bf[:, [[0, 1], [0, 2], [1, 2]]], axis=2).reshape(-1, 2)
            key_all = edges[:, 0] * nv + edges[:, 1]
            idx = np.searchsorted(key_all, fe[:, 0] * nv + fe[:, 1])
            bnd[nv + idx] = True
        self.boundary = bnd


def _geometry(mesh):
    v, c = mesh.verts, mesh.cells
    x0 = v[c[:, 0]]
    J = np.stack([v[c[:, 1]] - x0, v[c[:, 2]] - x0, v[c[:, 3]] - x0], axis=2)
    det = np.linalg.det(J)
    return x0, J, np.abs(det), np.linalg.inv(J)


def assemble_level(mesh, mesh_index: int, log_visc: Optional[np.ndarray] = None, sensitivities: bool = False,
                   forcing_nodal: Optional[np.ndarray] = None) -> LevelData:
    k = 2
    V, Q = Space3(mesh, 2), Space3(mesh, 1)
    x0, J, adet, Jinv = _geometry(mesh)
    pts, w = conical_rule(2 * k - 1 if log_visc is not None else 2 * k - 2)
    _, dphi = shape_functions(k, pts)
    psi, _ = shape_functions(k - 1, pts)
    g = np.einsum("qnj,cji->cqni", dphi, Jinv)
    wc = adet[:, None] * w[None, :]
    Lt = None
    if log_visc is None:
        Le = np.einsum("cq,cqai,cqbi->cab", wc, g, g)
    else:
        Lt = np.einsum("cq,qt,cqai,cqbi->ctab", wc, bary4(pts), g, g)
        Le = np.einsum("ct,ctab->cab", np.exp(np.asarray(log_visc)[mesh.cells]), Lt)
    Be = [-np.einsum("cq,qi,cqa->cia", wc, psi, g[..., d]) for d in range(3)]
    vd, qd = V.cell_dofs, Q.cell_dofs
    nl, ql = vd.shape[1], qd.shape[1]
    Lm = sp.coo_matrix((Le.ravel(), (np.repeat(vd, nl, axis=1).ravel(), np.tile(vd, (1, nl)).ravel())),
                       shape=(V.ndofs, V.ndofs)).tocsr()
    ri = np.repeat(qd, nl, axis=1).ravel()
    ci = np.tile(vd, (1, ql)).ravel()
    Bm = [sp.coo_matrix((b.ravel(), (ri, ci)), shape=(Q.ndofs, V.ndofs)).tocsr() for b in Be]
    free = np.flatnonzero(~V.boundary)
    nfu = free.size
    Lff = Lm[free][:, free]
    Bf = [b[:, free] for b in Bm]
    K = sp.bmat([[Lff, None, None, Bf[0].T], [None, Lff, None, Bf[1].T], [None, None, Lff, Bf[2].T],
                 [Bf[0], Bf[1], Bf[2], sp.csr_matrix((Q.ndofs, Q.ndofs))]], format="csr")
    lev = LevelData(k, "TH", V, Q, nfu, Q.ndofs, free, Csr.from_scipy(K), mesh_index, mesh=mesh,
                    log_visc=None if log_visc is None else np.asarray(log_visc, dtype=np.float64), dim=3)
    G = None
    if sensitivities or forcing_nodal is not None:
        mpts, mw = conical_rule(2 * k)
        mphi, _ = shape_functions(k, mpts)
        Me = np.einsum("c,q,qa,qb->cab", adet, mw, mphi, mphi)
        M = sp.coo_matrix((Me.ravel(), (np.repeat(vd, nl, axis=1).ravel(), np.tile(vd, (1, nl)).ravel())),
                          shape=(V.ndofs, V.ndofs)).tocsr()
        Mf = M[free]
        Z = sp.csr_matrix((Q.ndofs, V.ndofs))
        G = sp.bmat([[Mf, None, None], [None, Mf, None], [None, None, Mf], [Z, Z, Z]], format="csr")
        G.sum_duplicates()
        G.sort_indices()
    if sensitivities:
        lev.visc_sens = _viscosity_sensitivity(lev, mesh, Lt)
        lev.forcing_map = Csr.from_scipy(G)
    if forcing_nodal is not None:
        lev.b = np.stack([G @ f.ravel() for f in forcing_nodal])
    return lev


def _viscosity_sensitivity(lev: LevelData, mesh, Lt) -> Csr:
    if Lt is None:
        raise ValueError("the viscosity sensitivity needs a log-viscosity field")
    nv = mesh.verts.shape[0]
    K = lev.K
    n, nfu = K.nrows, lev.nfu
    keys = np.repeat(np.arange(n, dtype=np.int64), np.diff(K.rowptr)) * n + K.col
    pos = -np.ones(lev.V.ndofs, dtype=np.int64)
    pos[lev.free_u] = np.arange(nfu)
    fi = pos[lev.V.cell_dofs]
    ev = np.exp(lev.log_visc[mesh.cells])
    nl = fi.shape[1]
    I = np.repeat(fi[:, :, None], nl, axis=2)
    Jc = np.repeat(fi[:, None, :], nl, axis=1)
    ok = (I >= 0) & (Jc >= 0)
    rows, cols, vals = [], [], []
    for t in range(4):
        val = (ev[:, t, None, None] * Lt[:, t])[ok]
        vtx = np.broadcast_to(mesh.cells[:, t, None, None], I.shape)[ok]
        for comp in range(3):
            key = (I[ok] + comp * nfu) * n + (Jc[ok] + comp * nfu)
            e = np.searchsorted(keys, key)
            assert np.array_equal(keys[e], key)
            rows.append(vtx)
            cols.append(e)
            vals.append(val)
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nv, K.nnz)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return Csr.from_scipy(S)


def vanka_patches(lev: LevelData):
    """(ptr, dofs, weights): velocity DoFs of every node of the cells around vertex v, then
    the pressure DoF of v; W_i = I (weights of the partition of unity are also returned)."""
    mesh = lev.mesh
    nv = mesh.verts.shape[0]
    cells, cd = mesh.cells, lev.V.cell_dofs
    nl = cd.shape[1]
    node = np.repeat(cd[:, None, :], 4, axis=1).ravel()             # (cell, vertex t, node)
    vtx = np.repeat(cells[:, :, None], nl, axis=2).ravel()
    pairs = np.unique(np.stack([vtx, node], axis=1), axis=0)
    upos = -np.ones(lev.V.ndofs, dtype=np.int64)
    upos[lev.free_u] = np.arange(lev.nfu)
    fu = upos[pairs[:, 1]]
    keep = fu >= 0
    pv, pu = pairs[keep, 0], fu[keep]
    nfu = lev.nfu
    rows, dofs = [], []
    for comp in range(3):
        rows.append(pv)
        dofs.append(pu + comp * nfu)
    rows.append(np.arange(nv))
    dofs.append(3 * nfu + np.arange(nv))
    r = np.concatenate(rows)
    d = np.concatenate(dofs)
    order = np.lexsort((d, r))
    r, d = r[order], d[order]
    counts = np.bincount(r, minlength=nv)
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    mult = np.bincount(d, minlength=lev.n).astype(np.float64)
    return ptr, d.astype(np.int32), 1.0 / mult[d]


def prolongation(fine: LevelData, coarse: LevelData, parent) -> Csr:
    """P = diag(P_u, P_u, P_u, P_p): coarse shape functions at the fine nodes (via the parent cell)."""
    fm, cm = fine.mesh, coarse.mesh
    x0, J, _, Jinv = _geometry(cm)

    def scalar(fs: Space3, cs: Space3, k: int):
        fc_nodes = fs.cell_dofs                                       # nc_f x nl_f
        first = np.full(fs.ndofs, -1, dtype=np.int64)
        flat = fc_nodes.ravel()
        cell_of = np.repeat(np.arange(fc_nodes.shape[0]), fc_nodes.shape[1])
        order = np.argsort(flat, kind="stable")
        uniq, idx = np.unique(flat[order], return_index=True)
        first[uniq] = cell_of[order][idx]
        pc = parent[first]                                            # coarse cell per fine node
        ref = np.einsum("nij,nj->ni", Jinv[pc], fs.coords - x0[pc])
        vals, _ = shape_functions(k, ref)
        rows = np.repeat(np.arange(fs.ndofs), vals.shape[1])
        cols = cs.cell_dofs[pc].ravel()
        v = vals.ravel()
        keep = np.abs(v) >= ZERO_TOL
        M = sp.coo_matrix((v[keep], (rows[keep], cols[keep])), shape=(fs.ndofs, cs.ndofs)).tocsr()
        M.sum_duplicates()
        return M

    Pu = scalar(fine.V, coarse.V, 2)[fine.free_u][:, coarse.free_u]
    Pp = scalar(fine.Q, coarse.Q, 1)
    P = sp.block_diag([Pu, Pu, Pu, Pp], format="csr")
    P.sort_indices()
    return Csr.from_scipy(P)


def build_hierarchy(name: str, meshes: List, forcing: Optional[str], nrhs: int, log_visc, sensitivities: bool):
    """Levels on the nested cube meshes (finest first), hMG with Chebyshev-accelerated Vanka
    relaxation (W_i = I) and a dense coarse solve; bumps forcing with homogeneous Dirichlet data."""
    from .frontend import SEEDS
    nlev = len(meshes)
    opts = dict(nu_p=2, nu_h=2, n_v=1, n_plevels=0, omega=0.5, smoother="chebyshev", cheb_lo=0.1, cheb_hi=1.1,
                eig_iters=20)
    fn = None
    if forcing == "bumps":
        seed = SEEDS.get(name.split("_")[0], 5)
        C, W, D = synth.gaussian_bump_params3d(nrhs, seed)
        X = Space3(meshes[0], 2).coords
        fn = np.stack([np.stack(synth.gaussian_bump_forcing3d(X[:, 0], X[:, 1], X[:, 2], C[i], W[i], D[i]))
                       for i in range(nrhs)])
    elif forcing not in (None, "none"):
        raise KeyError(f"3D workloads take forcing='bumps' or None (got {forcing!r})")
    levels: List[LevelData] = []
    for li in range(nlev):
        lv = None
        if log_visc is not None:
            nv = meshes[li].verts.shape[0]
            assert np.array_equal(meshes[li].verts, meshes[0].verts[:nv])
            lv = np.asarray(log_visc, dtype=np.float64)[:nv]
        lev = assemble_level(meshes[li], li, log_visc=lv, sensitivities=sensitivities and li == 0,
                             forcing_nodal=fn if li == 0 else None)
        if li < nlev - 1:
            lev.patch_ptr, lev.patch_dofs, lev.patch_weight = vanka_patches(lev)
        if li > 0:
            lev.P = prolongation(levels[li - 1], lev, meshes[li - 1].parent)
        levels.append(lev)
    return Hierarchy(name, levels, opts, False)
