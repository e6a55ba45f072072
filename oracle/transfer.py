"""Grid-transfer operators (oracle).

Section 3.1: P is finite-element interpolation, R = P^T; for nested spaces
this is the L2 projection of the coarse function into the fine space and needs
no solve.  Section 3.2: the p-transfer between P_k/P_{k-1} and P_2/P_1 on the
same mesh is built the same way.  Entry P[i, j] is the j-th coarse basis
function evaluated at the i-th fine node; fine and coarse Dirichlet DoFs are
dropped (corrections vanish there).  Entries with |P_ij| < 1e-10 are exact
zeros of a basis function at a lattice node computed with rounding error
(every genuine entry is a basis value at a lattice point, |P_ij| >= 1/32) and
are dropped.
A Scott-Vogelius fine pressure node takes the value of the continuous coarse
pressure of the cell it belongs to.

Pins: tests/test_oracle_transfer.py -- P reproduces interpolants of P_2
velocities and P_1 pressures exactly, P 1 = 1 on pressure, and the Galerkin
product R K_f P equals the rediscretised K_c.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import element
from .discretization import cell_geometry

DROP_TOL = 1e-10


def _scalar_interp(f_space, c_space, fverts, fcells, cverts, ccells, parent):
    vals = {}
    for cf in range(fcells.shape[0]):
        cc = cf if parent is None else int(parent[cf])
        x0, J, _, _ = cell_geometry(cverts, ccells[cc])
        Jinv = np.linalg.inv(J)
        fd = f_space.cell_dofs[cf]
        pts = f_space.coords[fd]
        ref = (pts - x0) @ Jinv.T
        if c_space.k >= 1:
            phi, _ = element.eval_basis(c_space.k, ref)
        else:
            phi = np.ones((len(fd), 1))
        cd = c_space.cell_dofs[cc]
        for a, i in enumerate(fd):
            row = vals.setdefault(int(i), {})
            for b_, j in enumerate(cd):
                row[int(j)] = phi[a, b_]
    return vals


def prolongation(fine, coarse, parent=None) -> sp.csr_matrix:
    """P: coarse free DoFs -> fine free DoFs, block diagonal (u_x, u_y, p)."""
    fm, cm = fine.mesh, coarse.mesh
    Pu = _scalar_interp(fine.V, coarse.V, fm.verts, fm.cells, cm.verts, cm.cells, parent)
    Pp = _scalar_interp(fine.Q, coarse.Q, fm.verts, fm.cells, cm.verts, cm.cells, parent)
    fpos = np.full(fine.V.ndofs, -1)
    fpos[fine.free_u] = np.arange(fine.nfu)
    cpos = np.full(coarse.V.ndofs, -1)
    cpos[coarse.free_u] = np.arange(coarse.nfu)
    rows, cols, vals = [], [], []
    for i, row in Pu.items():
        if fpos[i] < 0:
            continue
        for j, v in row.items():
            if cpos[j] < 0 or abs(v) < DROP_TOL:
                continue
            for comp in range(2):
                rows.append(fpos[i] + comp * fine.nfu)
                cols.append(cpos[j] + comp * coarse.nfu)
                vals.append(v)
    for i, row in Pp.items():
        for j, v in row.items():
            if abs(v) < DROP_TOL:
                continue
            rows.append(2 * fine.nfu + i)
            cols.append(2 * coarse.nfu + j)
            vals.append(v)
    P = sp.csr_matrix((vals, (rows, cols)), shape=(fine.n, coarse.n))
    P.sum_duplicates()
    P.sort_indices()
    return P
