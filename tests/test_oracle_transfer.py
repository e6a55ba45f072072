"""Pins of the oracle's transfer operators (Sections 3.1, 3.2)."""
import numpy as np
import pytest

import synth
from oracle import transfer
from oracle.discretization import assemble_stokes


def _poly(deg, coeffs):
    def f(x, y):
        out = np.zeros_like(x)
        t = 0
        for i in range(deg + 1):
            for j in range(deg + 1 - i):
                out += coeffs[t] * x ** i * y ** j
                t += 1
        return out
    return f


PAIRS = [
    # (fine mesh, coarse mesh, parent, fine (k, kind), coarse (k, kind))
    ("h", 2, "TH", 2, "TH"),
    ("p", 4, "TH", 2, "TH"),
    ("p", 3, "TH", 2, "TH"),
    ("palf", 4, "SV", 2, "TH"),
    ("half", 2, "TH", 2, "TH"),
]


def _meshes(kind):
    base = synth.delaunay_square(9, seed=6)
    if kind == "h":
        fine = synth.refine_uniform(base)
        return fine, base, fine.parent
    if kind == "p":
        fine = synth.refine_uniform(base)
        return fine, fine, None
    if kind == "palf":
        fine = synth.alfeld_split(base)
        return fine, fine, None
    if kind == "half":
        fine = synth.alfeld_split(base)
        return fine, base, fine.parent
    raise KeyError(kind)


@pytest.mark.parametrize("rel,kf,kindf,kc,kindc", PAIRS)
def test_interpolation_reproduces_coarse_polynomials(rel, kf, kindf, kc, kindc):
    fm, cm, parent = _meshes(rel)
    fd = assemble_stokes(fm, kf, kindf)
    cd = assemble_stokes(cm, kc, kindc)
    rng = np.random.default_rng(2)
    for space_f, space_c, deg in ((fd.V, cd.V, kc), (fd.Q, cd.Q, kc - 1)):
        rows = transfer._scalar_interp(space_f, space_c, fm.verts, fm.cells, cm.verts, cm.cells, parent)
        q = _poly(deg, rng.standard_normal(40))
        qc = q(space_c.coords[:, 0], space_c.coords[:, 1])
        qf = q(space_f.coords[:, 0], space_f.coords[:, 1])
        got = np.array([sum(v * qc[j] for j, v in rows[i].items()) for i in range(space_f.ndofs)])
        assert np.abs(got - qf).max() < 1e-12 * max(1.0, np.abs(qf).max())


@pytest.mark.parametrize("rel,kf,kindf,kc,kindc", PAIRS)
def test_galerkin_equals_rediscretisation_and_constant_pressure(rel, kf, kindf, kc, kindc):
    fm, cm, parent = _meshes(rel)
    fd = assemble_stokes(fm, kf, kindf)
    cd = assemble_stokes(cm, kc, kindc)
    P = transfer.prolongation(fd, cd, parent)
    G = (P.T @ fd.K @ P).toarray()
    Kc = cd.K.toarray()
    assert np.abs(G - Kc).max() <= 1e-12 * np.abs(Kc).max()
    ones = np.zeros(cd.n)
    ones[2 * cd.nfu:] = 1.0
    assert np.allclose((P @ ones)[2 * fd.nfu:], 1.0, atol=1e-14)
    assert np.abs((P @ ones)[: 2 * fd.nfu]).max() == 0.0
