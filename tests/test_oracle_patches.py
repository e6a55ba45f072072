"""Pins of the oracle's Vanka-star patches (Section 3.4, figure "fig:patches")."""
import numpy as np
import pytest

import synth
from oracle.discretization import assemble_stokes
from oracle.patches import multiplicity_weights, vanka_star_patches


def _closed_form(kind, k, n):
    """DoFs of an interior vertex patch with n surrounding cells (2D).

    velocity on the closure of the star: 1 + n vertices, 2n edges with k-1
    nodes each, n cells with (k-1)(k-2)/2 interior nodes, two components;
    pressure on the star: TH P_{k-1}: the vertex, n edges with k-2 nodes, n
    cells with (k-2)(k-3)/2 nodes; SV: n cells with k(k+1)/2 nodes each.
    """
    vel = 1 + n + 2 * n * (k - 1) + n * (k - 1) * (k - 2) // 2
    prs = (1 + n * (k - 2) + n * (k - 2) * (k - 3) // 2) if kind == "TH" else n * k * (k + 1) // 2
    return 2 * vel + prs


def test_closed_form_values_quoted_in_the_design():
    assert _closed_form("TH", 2, 6) == 39
    assert _closed_form("TH", 3, 6) == 81
    assert _closed_form("TH", 4, 6) == 141
    assert _closed_form("SV", 4, 12) == 362
    assert _closed_form("SV", 4, 3) == 92


@pytest.mark.parametrize("kind,k,mesh", [
    ("TH", 2, synth.structured_square(6)),
    ("TH", 3, synth.structured_square(5)),
    ("TH", 4, synth.refine_uniform(synth.delaunay_square(12, seed=9))),
    ("SV", 4, synth.alfeld_split(synth.structured_square(4))),
    ("SV", 3, synth.alfeld_split(synth.refine_uniform(synth.delaunay_square(8, seed=4)))),
])
def test_interior_patch_sizes_match_closed_form(kind, k, mesh):
    d = assemble_stokes(mesh, k, kind)
    patches = vanka_star_patches(d)
    cells = mesh.cells
    nv = mesh.nv
    vc = [[] for _ in range(nv)]
    for c in range(cells.shape[0]):
        for v in cells[c]:
            vc[int(v)].append(c)
    # patches are emitted for every vertex with a non-empty star, in vertex order
    assert len(patches) == sum(1 for v in range(nv) if vc[v])
    bnd_vert = d.V.boundary[:nv]
    checked = 0
    for v in range(nv):
        closure_verts = set(int(w) for c in vc[v] for w in cells[c])
        if any(bnd_vert[w] for w in closure_verts):
            continue
        assert len(patches[v]) == _closed_form(kind, k, len(vc[v])), v
        checked += 1
    assert checked > 0


def test_partition_of_unity_and_coverage():
    d = assemble_stokes(synth.refine_uniform(synth.delaunay_square(10, seed=2)), 3, "TH")
    patches = vanka_star_patches(d)
    W = multiplicity_weights(patches, d.n)
    S = np.zeros((d.n, d.n))
    for P, w in zip(patches, W):
        S[P, P] += w
    assert np.allclose(S, np.eye(d.n), atol=1e-15)
    for P in patches:
        assert np.all(np.diff(P) > 0)


def test_patch_contains_velocity_and_pressure_blocks_in_order():
    d = assemble_stokes(synth.structured_square(4), 2, "TH")
    for P in vanka_star_patches(d):
        isp = P >= 2 * d.nfu
        # velocity first, pressure after (ascending canonical order)
        assert np.all(np.diff(isp.astype(int)) >= 0)
