"""Seeded triangle meshes and nested refinements.

The paper builds its hierarchies by quadrisection refinement R_u of a base
mesh, and for Scott-Vogelius one barycentric (Alfeld) refinement R_b of the
finest mesh only (Section 2.1, figure "fig:meshes"; Section 3.3).  These
functions produce exactly such nested meshes from a seeded base mesh.  Every
mesh is a vertex array ``verts`` (nv x 2, float64) and a cell array ``cells``
(nc x 3, int64, counter-clockwise).  A refined mesh carries ``parent``: for
each of its cells the index of the coarse cell that contains it.

Nothing here is finite-element or solver arithmetic: only geometry and
connectivity, shared as an input fixture by the oracle and the GPU path.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Mesh:
    verts: np.ndarray
    cells: np.ndarray
    parent: Optional[np.ndarray] = None   # cell -> containing cell of the next coarser mesh
    kind: str = "base"                    # "base" | "uniform" | "alfeld"
    meta: dict = field(default_factory=dict)

    @property
    def nv(self) -> int:
        return int(self.verts.shape[0])

    @property
    def nc(self) -> int:
        return int(self.cells.shape[0])


def _orient_ccw(verts: np.ndarray, cells: np.ndarray) -> np.ndarray:
    cells = np.array(cells, dtype=np.int64, copy=True)
    p0, p1, p2 = verts[cells[:, 0]], verts[cells[:, 1]], verts[cells[:, 2]]
    area2 = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0])
    flip = area2 < 0
    cells[flip, 1], cells[flip, 2] = cells[flip, 2].copy(), cells[flip, 1].copy()
    return cells


def structured_square(n: int) -> Mesh:
    """Unit square, n x n squares, each split by the diagonal (i,j)->(i+1,j+1).

    Vertex (i, j) sits at (i/n, j/n) and has id j*(n+1)+i.
    """
    xs = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    cells = []
    for j in range(n):
        for i in range(n):
            v00 = j * (n + 1) + i
            v10 = v00 + 1
            v01 = v00 + (n + 1)
            v11 = v01 + 1
            cells.append((v00, v10, v11))
            cells.append((v00, v11, v01))
    return Mesh(verts, np.asarray(cells, dtype=np.int64), kind="base", meta={"n": n})


def delaunay_square(npts: int, seed: int) -> Mesh:
    """Delaunay triangulation of ``npts`` seeded U[0,1]^2 points plus the 4 corners."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(npts, 2))
    corners = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    verts = np.concatenate([corners, pts], axis=0)
    tri = Delaunay(verts)
    cells = _orient_ccw(verts, tri.simplices.astype(np.int64))
    # stable cell order: sort by the sorted vertex triple
    key = np.sort(cells, axis=1)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    return Mesh(verts, cells[order], kind="base", meta={"npts": npts, "seed": seed})


def _boundary_vertex_mask(verts: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    x, y = verts[:, 0], verts[:, 1]
    return (np.abs(x) < tol) | (np.abs(x - 1) < tol) | (np.abs(y) < tol) | (np.abs(y - 1) < tol)


def jitter_interior(mesh: Mesh, amount: float, seed: int) -> Mesh:
    """Move every interior vertex by U[-amount, amount]^2 (seeded)."""
    rng = np.random.default_rng(seed)
    verts = mesh.verts.copy()
    d = rng.uniform(-amount, amount, size=verts.shape)
    interior = ~_boundary_vertex_mask(verts)
    verts[interior] += d[interior]
    return Mesh(verts, mesh.cells.copy(), mesh.parent, mesh.kind, dict(mesh.meta, jitter=amount))


def _edge_table(cells: np.ndarray):
    """Unique sorted vertex pairs and, per cell, the index of its 3 edges.

    Local edge e of a cell joins local vertices (e, (e+1)%3).
    """
    pairs = np.stack([cells[:, [0, 1]], cells[:, [1, 2]], cells[:, [2, 0]]], axis=1)  # nc x 3 x 2
    pairs = np.sort(pairs, axis=2).reshape(-1, 2)
    uniq, inv = np.unique(pairs, axis=0, return_inverse=True)
    return uniq, inv.reshape(-1, 3)


def refine_uniform(mesh: Mesh) -> Mesh:
    """Quadrisection: every triangle splits into 4 through its edge midpoints.

    New vertex ids: the coarse vertices keep theirs, edge midpoints follow in
    the order of the sorted unique edge list.
    """
    edges, cell_edges = _edge_table(mesh.cells)
    nv = mesh.nv
    mid = 0.5 * (mesh.verts[edges[:, 0]] + mesh.verts[edges[:, 1]])
    verts = np.concatenate([mesh.verts, mid], axis=0)
    a, b, c = mesh.cells[:, 0], mesh.cells[:, 1], mesh.cells[:, 2]
    mab = nv + cell_edges[:, 0]
    mbc = nv + cell_edges[:, 1]
    mca = nv + cell_edges[:, 2]
    children = np.stack([
        np.stack([a, mab, mca], axis=1),
        np.stack([mab, b, mbc], axis=1),
        np.stack([mca, mbc, c], axis=1),
        np.stack([mab, mbc, mca], axis=1),
    ], axis=1)  # nc x 4 x 3
    cells = children.reshape(-1, 3)
    parent = np.repeat(np.arange(mesh.nc, dtype=np.int64), 4)
    return Mesh(verts, cells, parent, "uniform", dict(mesh.meta))


def alfeld_split(mesh: Mesh) -> Mesh:
    """Barycentric (Alfeld) refinement: every triangle splits into 3 at its barycentre."""
    nv = mesh.nv
    g = mesh.verts[mesh.cells].mean(axis=1)
    verts = np.concatenate([mesh.verts, g], axis=0)
    a, b, c = mesh.cells[:, 0], mesh.cells[:, 1], mesh.cells[:, 2]
    gi = nv + np.arange(mesh.nc, dtype=np.int64)
    children = np.stack([
        np.stack([a, b, gi], axis=1),
        np.stack([b, c, gi], axis=1),
        np.stack([c, a, gi], axis=1),
    ], axis=1)
    cells = children.reshape(-1, 3)
    parent = np.repeat(np.arange(mesh.nc, dtype=np.int64), 3)
    return Mesh(verts, cells, parent, "alfeld", dict(mesh.meta))


def hierarchy(base: Mesh, nref: int, alfeld: bool = False) -> List[Mesh]:
    """Nested meshes, coarsest first: base, R_u(base), ..., and optionally R_b(finest)."""
    meshes = [base]
    for _ in range(nref):
        meshes.append(refine_uniform(meshes[-1]))
    if alfeld:
        meshes.append(alfeld_split(meshes[-1]))
    return meshes


# ---------------------------------------------------------------------------
# 3D: unit cube, n^3 cubes each split into 6 Kuhn tetrahedra
# ---------------------------------------------------------------------------

_KUHN = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def _kuhn_cells(n: int, vid: np.ndarray) -> np.ndarray:
    """Cells of the Kuhn split: cube (i,j,k) -> 6 tets c, c+e_s0, c+e_s0+e_s1, c+(1,1,1)
    for the permutations s in _KUHN order; vid maps lattice (i,j,k) to a vertex id."""
    cells = []
    idx = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), axis=-1).reshape(-1, 3)
    # cube order: i fastest, then j, then k
    idx = idx[np.lexsort((idx[:, 0], idx[:, 1], idx[:, 2]))]
    eye = np.eye(3, dtype=np.int64)
    for c in idx:
        for s in _KUHN:
            p0 = c
            p1 = p0 + eye[s[0]]
            p2 = p1 + eye[s[1]]
            p3 = p2 + eye[s[2]]
            cells.append([vid[tuple(p)] for p in (p0, p1, p2, p3)])
    return np.array(cells, dtype=np.int64)


def structured_cube(n: int, coarse: Optional[Mesh] = None) -> Mesh:
    """The unit cube with n^3 cubes, 6 Kuhn tetrahedra each (6 n^3 cells).

    Without ``coarse`` the vertex ids are lexicographic (i fastest).  With the
    mesh of n/2 cubes as ``coarse``, the vertices it shares keep their ids and
    come first (the remaining lattice points follow lexicographically), and
    ``parent`` maps every cell to the coarse tetrahedron that contains it: the
    Kuhn split of the halved lattice refines the coarse one (both are the
    cells of the hyperplanes x_i = const and x_i - x_j = const).
    """
    m = n + 1
    lat = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), axis=-1).reshape(-1, 3)
    lat = lat[np.lexsort((lat[:, 0], lat[:, 1], lat[:, 2]))]          # i fastest
    vid = np.zeros((m, m, m), dtype=np.int64)
    if coarse is None:
        vid[lat[:, 0], lat[:, 1], lat[:, 2]] = np.arange(lat.shape[0])
    else:
        nc_ = coarse.meta["n"]
        assert 2 * nc_ == n
        cpts = np.rint(coarse.verts * nc_).astype(np.int64) * 2     # coarse ids in fine lattice units
        taken = np.zeros((m, m, m), dtype=bool)
        vid[cpts[:, 0], cpts[:, 1], cpts[:, 2]] = np.arange(cpts.shape[0])
        taken[cpts[:, 0], cpts[:, 1], cpts[:, 2]] = True
        rest = lat[~taken[lat[:, 0], lat[:, 1], lat[:, 2]]]
        vid[rest[:, 0], rest[:, 1], rest[:, 2]] = cpts.shape[0] + np.arange(rest.shape[0])
    verts = np.zeros((m ** 3, 3))
    verts[vid[lat[:, 0], lat[:, 1], lat[:, 2]]] = lat / n
    cells = _kuhn_cells(n, vid)
    parent = None
    if coarse is not None:
        cen = verts[cells].mean(axis=1) * (n // 2)
        cube = np.minimum(np.floor(cen).astype(np.int64), n // 2 - 1)
        t = cen - cube
        order = np.argsort(-t, axis=1)
        perm = {s: q for q, s in enumerate(_KUHN)}
        pidx = np.array([perm[tuple(o)] for o in order], dtype=np.int64)
        cube_id = cube[:, 0] + (n // 2) * cube[:, 1] + (n // 2) ** 2 * cube[:, 2]
        parent = cube_id * 6 + pidx
    return Mesh(verts, cells, parent, "base" if coarse is None else "uniform", {"n": n, "dim": 3})


def cube_hierarchy(n0: int, nref: int) -> List[Mesh]:
    """Nested Kuhn cube meshes n0^3, (2 n0)^3, ..., coarsest first."""
    meshes = [structured_cube(n0)]
    for _ in range(nref):
        meshes.append(structured_cube(2 * meshes[-1].meta["n"], coarse=meshes[-1]))
    return meshes


def config_mesh_hierarchy(name: str) -> List[Mesh]:
    """Mesh hierarchies of the benchmark workloads (coarsest first).

    * ``cfg1``: structured 4x4 refined once -> 8x8 (Taylor-Hood P2/P1, 2 h-levels).
    * ``cfg2``: Delaunay of 64 seeded points + corners, 3 quadrisections.
    * ``cfg3``: structured 8x8, 4 quadrisections -> 128x128 (``cfg3_r1``,
      ``cfg3_r2``: 1 and 2 quadrisections, the same recipe at 16x16 and 32x32).
    * ``cfg4``: 16x16 structured with interior jitter 0.2h, 2 quadrisections, Alfeld split.
    * ``cfg5``: unit cube 4^3 -> 8^3 -> 16^3, 6 Kuhn tetrahedra per cube (``cfg5_r1``:
      4^3 -> 8^3; ``cube_tiny``: 1^3 -> 2^3).
    * ``tiny2``/``tiny4``: 1x1 -> 2x2 and 2x2 -> 4x4 structured (dense-operator pins).
    """
    if name == "cfg1":
        return hierarchy(structured_square(4), 1)
    if name == "cfg2":
        return hierarchy(delaunay_square(64, seed=2), 3)
    if name == "cfg2_r2":
        return hierarchy(delaunay_square(64, seed=2), 2)
    if name == "cfg2_r1":
        return hierarchy(delaunay_square(64, seed=2), 1)
    if name == "cfg3":
        return hierarchy(structured_square(8), 4)
    if name == "cfg3_r0":
        return hierarchy(structured_square(8), 0)
    if name == "cfg3_r2":
        return hierarchy(structured_square(8), 2)
    if name == "cfg3_r1":
        return hierarchy(structured_square(8), 1)
    if name == "cfg4":
        base = jitter_interior(structured_square(16), 0.2 / 16, seed=4)
        return hierarchy(base, 2, alfeld=True)
    if name == "cfg4_r0":
        base = jitter_interior(structured_square(16), 0.2 / 16, seed=4)
        return hierarchy(base, 0, alfeld=True)
    if name == "sv_small":
        base = jitter_interior(structured_square(4), 0.2 / 4, seed=4)
        return hierarchy(base, 1, alfeld=True)
    if name == "cfg5":
        return cube_hierarchy(4, 2)
    if name == "cfg5_r1":
        return cube_hierarchy(4, 1)
    if name == "cube_tiny":
        return cube_hierarchy(1, 1)
    if name == "tiny2":
        return hierarchy(structured_square(1), 1)
    if name == "tiny4":
        return hierarchy(structured_square(2), 1)
    raise KeyError(name)
