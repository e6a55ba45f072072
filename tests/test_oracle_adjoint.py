"""Pins of the oracle's variable-viscosity assembly and adjoint gradients (not gpu).

The gradients are checked against central finite differences of the objective
computed with a sparse direct solve of the bordered system, so neither the
multigrid cycle nor FGMRES enters the reference.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import adjoint
from oracle import multigrid as omg
from oracle import problems as oproblems
from oracle.discretization import assemble_stokes


def _direct(K, z, b):
    Kb = sp.bmat([[K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]], format="csc")
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:-1]


def _bump_nodal(disc, nrhs, seed):
    C, W, D = synth.gaussian_bump_params(nrhs, seed)
    out = np.zeros((nrhs, 2, disc.V.ndofs))
    for b in range(nrhs):
        fx, fy = synth.gaussian_bump_forcing(disc.V.coords[:, 0], disc.V.coords[:, 1], C[b], W[b], D[b])
        out[b, 0], out[b, 1] = fx, fy
    return out


def _J(name, lv, fn, T):
    levels, discs, opts, _ = oproblems.build(name, with_rhs=False, log_visc=lv)
    d = discs[0]
    B = adjoint.forcing_rhs(d, fn)
    X = np.stack([_direct(d.K, d.null_vector(), b) for b in B])
    return adjoint.objective(X, T, d.nfu), X, levels, discs, opts


def test_zero_and_constant_log_viscosity():
    mesh = synth.delaunay_square(10, seed=3)
    d1 = assemble_stokes(mesh, 3, "TH")
    d0 = assemble_stokes(mesh, 3, "TH", log_visc=np.zeros(mesh.nv))
    assert abs(d0.K - d1.K).max() <= 1e-14 * abs(d1.K).max()
    c = 0.37
    dc = assemble_stokes(mesh, 3, "TH", log_visc=np.full(mesh.nv, c))
    n2 = 2 * d1.nfu
    vel = (dc.K[:n2, :n2] - np.exp(c) * d1.K[:n2, :n2])
    assert abs(vel).max() <= 1e-13 * abs(d1.K).max()
    assert abs(dc.K[n2:, :] - d1.K[n2:, :]).max() == 0.0


def test_linear_log_viscosity_integrates_exactly():
    """With l = log(1 + x) at the vertices the interpolant nu_h is 1 + x exactly, and for
    u = (psi, 0), psi = x(1-x)y(1-y) (exact in P4), u^T K u = int (1 + x) |grad psi|^2,
    a polynomial integral evaluated here by a tensor Gauss rule."""
    from oracle.discretization import interpolate
    mesh = synth.structured_square(3)
    lv = np.log(1.0 + mesh.verts[:, 0])
    d = assemble_stokes(mesh, 4, "TH", log_visc=lv)
    psi = lambda x, y: x * (1 - x) * y * (1 - y)
    v = interpolate(d, lambda x, y: (psi(x, y), np.zeros_like(x)))
    # int (1+x)(psi_x^2 + psi_y^2) over the unit square
    gx = lambda x, y: (1 - 2 * x) * y * (1 - y)
    from numpy.polynomial.legendre import leggauss
    g, w = leggauss(12)
    g, w = 0.5 * (g + 1), 0.5 * w
    X, Y = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w)
    ref = np.sum(W * (1 + X) * (gx(X, Y) ** 2 + gx(Y, X) ** 2))
    assert abs(v @ (d.K @ v) - ref) <= 1e-14


@pytest.mark.parametrize("name", ["tiny4", "cfg1"])
def test_viscosity_gradient_matches_finite_differences(name):
    mesh0 = synth.config_mesh_hierarchy(name)[-1]
    lv = synth.log_viscosity(mesh0.verts, seed=5)
    levels, discs, opts, _ = oproblems.build(name, with_rhs=False, log_visc=lv)
    d = discs[0]
    nrhs = 2
    fn = _bump_nodal(d, nrhs, seed=6)
    rng = np.random.default_rng(7)
    T = rng.standard_normal((nrhs, d.n)) * 0.01
    J0, X, levels, discs, opts = _J(name, lv, fn, T)
    omg.setup(levels, opts)
    J, gl, gf, Lam = adjoint.gradients(levels, opts, discs[0], X, T, rtol=1e-13)
    assert abs(J - J0) <= 1e-14 * abs(J0)
    h = 1e-5
    for trial in range(3):
        dl = rng.standard_normal(mesh0.nv)
        Jp = _J(name, lv + h * dl, fn, T)[0]
        Jm = _J(name, lv - h * dl, fn, T)[0]
        fd = (Jp - Jm) / (2 * h)
        an = gl @ dl
        print(f"{name} viscosity direction {trial}: adjoint {an:.12e} fd {fd:.12e}")
        assert abs(an - fd) <= 1e-7 * abs(fd)


@pytest.mark.parametrize("name", ["tiny4", "cfg1"])
def test_forcing_gradient_matches_finite_differences(name):
    mesh0 = synth.config_mesh_hierarchy(name)[-1]
    lv = synth.log_viscosity(mesh0.verts, seed=5)
    levels, discs, opts, _ = oproblems.build(name, with_rhs=False, log_visc=lv)
    d = discs[0]
    nrhs = 2
    fn = _bump_nodal(d, nrhs, seed=8)
    rng = np.random.default_rng(9)
    T = rng.standard_normal((nrhs, d.n)) * 0.01
    J0, X, levels, discs, opts = _J(name, lv, fn, T)
    omg.setup(levels, opts)
    _, gl, gf, _ = adjoint.gradients(levels, opts, discs[0], X, T, rtol=1e-13)
    h = 1e-3                     # J is quadratic in f: the central difference is exact
    for trial in range(2):
        df = rng.standard_normal(fn.shape)
        fd = (_J(name, lv, fn + h * df, T)[0] - _J(name, lv, fn - h * df, T)[0]) / (2 * h)
        an = float(np.sum(gf * df))
        print(f"{name} forcing direction {trial}: adjoint {an:.12e} fd {fd:.12e}")
        assert abs(an - fd) <= 1e-9 * abs(fd)
