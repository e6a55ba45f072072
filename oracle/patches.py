"""Vanka-star patches (oracle).

Section 3.4 and figure "fig:patches": one patch per mesh vertex v.  The
pressure DoFs of the patch are those on the topological star of v (v itself,
the edges containing v, the cells containing v); the velocity DoFs are those
on the closure of the star, i.e. every velocity DoF of every cell containing
v.  For Scott-Vogelius the discontinuous pressure DoFs of the cells around v
all belong to the star (they are attached to the cells).

Readings where the paper is silent: boundary vertices get patches too;
eliminated (Dirichlet) velocity DoFs are not in any patch; empty patches are
dropped; the DoF list of a patch is ascending in the canonical numbering
(velocity first, then pressure, because of the block order).

The partition-of-unity operator W_i of eq. "eq:ASM" is not defined by the
paper.  Two readings are provided: W_i = I, and W_i = diag(1/c_j) with c_j
the number of patches that contain DoF j (an exact partition of unity).

Pins: tests/test_oracle_patches.py -- closed-form interior patch sizes,
sum_i R_i^T W_i R_i = I for the multiplicity weights, every free DoF covered.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from . import element


def vanka_star_patches(disc) -> List[np.ndarray]:
    V, Q = disc.V, disc.Q
    cells = disc.mesh.cells
    nv = disc.mesh.verts.shape[0]
    vert_cells = [[] for _ in range(nv)]
    for c in range(cells.shape[0]):
        for t in range(3):
            vert_cells[int(cells[c, t])].append(c)

    # entity of every local pressure node of a continuous pressure space:
    # the set of local vertices with nonzero barycentric index
    qmi = element.multi_indices(Q.k)
    q_support = [tuple(t for t in range(3) if a[t] > 0) for a in qmi]

    patches = []
    for v in range(nv):
        star = vert_cells[v]
        if not star:
            continue
        vel = set()
        prs = set()
        for c in star:
            vel.update(int(s) for s in V.cell_dofs[c])
            if Q.continuous:
                cv = cells[c]
                for n, supp in enumerate(q_support):
                    # the node lies on the entity spanned by these local vertices;
                    # it is in star(v) iff that entity contains v
                    if any(int(cv[t]) == v for t in supp):
                        prs.add(int(Q.cell_dofs[c, n]))
            else:
                prs.update(int(s) for s in Q.cell_dofs[c])
        vel = np.array(sorted(vel), dtype=np.int64)
        ux = disc.u_index(0, vel)
        uy = disc.u_index(1, vel)
        dofs = np.concatenate([ux[ux >= 0], uy[uy >= 0], disc.p_index(np.array(sorted(prs), dtype=np.int64))])
        if dofs.size == 0:
            continue
        patches.append(np.sort(dofs))
    return patches


def multiplicity_weights(patches: List[np.ndarray], n: int) -> List[np.ndarray]:
    """W_i = diag(1/c_j), c_j = number of patches containing DoF j."""
    count = np.zeros(n)
    for S in patches:
        count[S] += 1.0
    return [1.0 / count[S] for S in patches]


def patch_csr(patches: List[np.ndarray], weights: Optional[List[np.ndarray]] = None):
    """Flatten to (ptr, dofs[, weights]) arrays."""
    ptr = np.zeros(len(patches) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(S) for S in patches])
    dofs = np.concatenate(patches).astype(np.int32) if patches else np.zeros(0, np.int32)
    w = None if weights is None else np.concatenate(weights)
    return ptr, dofs, w
