"""Full-block-factorisation preconditioner for Scott-Vogelius (oracle).

Section 3.3, eq. "eq:fbf":
    P^{-1} = [I  -A~^{-1} B^T; 0  I] [A~^{-1}  0; 0  S~^{-1}] [I  0; -B A~^{-1}  I],
with A~^{-1} one phMG V-cycle on the velocity block A and S~^{-1} the inverse
of the block-diagonal pressure mass matrix (spectrally equivalent to the
inverse Schur complement).  Section 3.4: the FBF relaxation uses vertex-star
velocity patches only (ASMStarPC), not the closure.

Readings (the paper is silent):
  * Applied to r = [r_u; r_p]: y_u = A~^{-1} r_u, z_p = S~^{-1}(r_p - B y_u),
    z_u = y_u - A~^{-1} B^T z_p (the three factors right to left).
  * S~^{-1} = -M_p^{-1}: the Schur complement of K = [A B^T; B 0] is
    -B A^{-1} B^T, negative semi-definite, so its mass-matrix surrogate
    carries the minus sign (viscosity 1).
  * The velocity hierarchy has the levels of the monolithic one (SV P_k on the
    Alfeld mesh -> TH P2 velocity -> coarser P2), its matrices the velocity
    blocks A_l, its transfers the velocity blocks of the monolithic ones, the
    same smoother and cycle parameters, and a plain (non-bordered) coarse LU.

Pins: tests/test_oracle_fbf.py -- closed-form star patch sizes; the block
inverse of the pressure mass matrix reproduces polynomials; with the exact
A^{-1} and the exact Schur complement the factorisation is a generalised
inverse of K (K P K = K).
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.sparse as sp

from . import element
from .discretization import Stokes, cell_geometry
from .multigrid import Level, vcycle


def star_patches(disc: Stokes) -> List[np.ndarray]:
    """Free velocity DoFs (both components) of the entities of star(v): v, its edges, its cells."""
    V = disc.V
    cells = disc.mesh.cells
    nv = disc.mesh.verts.shape[0]
    k = V.k
    ne = len(V.edges)
    nint = (k - 1) * (k - 2) // 2
    around = [[] for _ in range(nv)]
    for c in range(cells.shape[0]):
        for v in cells[c]:
            around[int(v)].append(c)
    out = []
    for v in range(nv):
        nodes = set()
        for c in around[v]:
            for gid in V.cell_dofs[c]:
                gid = int(gid)
                if gid < nv:
                    ok = gid == v
                elif gid < nv + ne * (k - 1):
                    ok = v in V.edges[(gid - nv) // (k - 1)]
                else:
                    ok = v in [int(t) for t in cells[(gid - nv - ne * (k - 1)) // nint]]
                if ok:
                    nodes.add(gid)
        nodes = np.array(sorted(nodes), dtype=np.int64)
        ix = disc.u_index(0, nodes)
        ix = ix[ix >= 0]
        if ix.size:
            out.append(np.sort(np.concatenate([ix, ix + disc.nfu])))
    return out


def pressure_mass_inverse(disc: Stokes) -> sp.csr_matrix:
    """-M_p^{-1} for the discontinuous pressure space, cell block by cell block."""
    assert disc.kind == "SV"
    kq = disc.k - 1
    qpts, qw = element.quadrature(2 * kq)
    psi, _ = element.eval_basis(kq, qpts)
    rows, cols, vals = [], [], []
    for c in range(disc.mesh.cells.shape[0]):
        _, _, adet, _ = cell_geometry(disc.mesh.verts, disc.mesh.cells[c])
        Mc = np.einsum("q,qa,qb->ab", qw * adet, psi, psi)
        Mi = -np.linalg.inv(Mc)
        qd = disc.Q.cell_dofs[c]
        rows.append(np.repeat(qd, len(qd)))
        cols.append(np.tile(qd, len(qd)))
        vals.append(Mi.ravel())
    S = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(disc.nq, disc.nq))
    S.sort_indices()
    return S


def velocity_levels(levels: List[Level], discs: List[Stokes]) -> List[Level]:
    """The hierarchy on the velocity blocks: A_l, star patches, velocity transfer blocks."""
    out = []
    for li, (L, d) in enumerate(zip(levels, discs)):
        nu = 2 * d.nfu
        A = L.K[:nu, :nu].tocsr()
        VL = Level(K=A)
        if li < len(levels) - 1:
            VL.patches = star_patches(d)
        if li > 0:
            nuf = 2 * discs[li - 1].nfu
            VL.P = L.P[:nuf, :nu].tocsr()
        out.append(VL)
    return out


def fbf_apply(vlevels: List[Level], vopts, B: sp.csr_matrix, Sinv, r: np.ndarray,
              A_inv=None) -> np.ndarray:
    """z = P^{-1} r.  A_inv(v) replaces the velocity V-cycle when given (exact-inverse pin)."""
    nu = B.shape[1]
    cyc = A_inv if A_inv is not None else (lambda v: vcycle(vlevels, vopts, v))
    yu = cyc(r[:nu])
    zp = Sinv @ (r[nu:] - B @ yu)
    zu = yu - cyc(B.T @ zp)
    return np.concatenate([zu, zp])
