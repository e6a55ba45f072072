"""Pins of the oracle's 3D Taylor-Hood P2/P1 discretisation on Kuhn cube meshes (not gpu).

Closed forms and invariants: a polynomial Stokes solution in the discrete
space is reproduced exactly, B annihilates interpolated curls, the interior
Vanka-star patch has 196 DoFs, the transfers reproduce P2 / P1 fields, the
Galerkin product equals the rediscretised coarse operator, and the adjoint
gradients equal central differences of direct solves.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import adjoint
from oracle import problems as oproblems
from oracle import stokes3d as s3


def _direct(K, z, b):
    Kb = sp.bmat([[K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]], format="csc")
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:-1]


# psi = x^2 y + y^2 z + x y z;  u = (d psi/dy, -d psi/dx, 0) is divergence free and quadratic
def _u(x, y, z):
    return (x * x + 2 * y * z + x * z, -(2 * x * y + y * z), np.zeros_like(x))


def _p(x, y, z):
    return x + 2 * y - 3 * z


def _f(x, y, z):
    # -lap u + grad p = (-2, 0, 0) + (1, 2, -3)
    return (np.full_like(x, -1.0), np.full_like(x, 2.0), np.full_like(x, -3.0))


def test_symmetry_spd_and_pressure_kernel():
    mesh = synth.structured_cube(2)
    d = s3.assemble(mesh, 2)
    assert abs(d.K - d.K.T).max() <= 1e-14 * abs(d.K).max()
    A = d.K[: 3 * d.nfu, : 3 * d.nfu].toarray()
    assert np.linalg.eigvalsh(A).min() > 0
    assert np.abs(d.K @ d.null_vector()).max() <= 1e-14 * abs(d.K).max()
    # DoF counts: (2n-1)^3 free velocity nodes per component, (n+1)^3 pressure nodes
    assert d.nfu == 3 ** 3 and d.nq == 27 and d.n == 3 * 27 + 27


def test_divergence_of_interpolated_curl_is_zero():
    mesh = synth.structured_cube(3)
    d = s3.assemble(mesh, 2)
    X = d.V.coords
    u = _u(X[:, 0], X[:, 1], X[:, 2])
    div = sum(d.B_full[c] @ u[c] for c in range(3))
    assert np.abs(div).max() <= 1e-13


def test_polynomial_solution_is_reproduced():
    mesh = synth.structured_cube(2)
    d = s3.assemble(mesh, 2, forcing=_f, dirichlet=_u)
    x = _direct(d.K, d.null_vector(), d.b)
    ref = s3.interpolate(d, _u, _p)
    x[3 * d.nfu:] -= x[3 * d.nfu:].mean()
    ref[3 * d.nfu:] -= ref[3 * d.nfu:].mean()
    assert np.abs(x - ref).max() <= 1e-11


def test_interior_vanka_patch_size():
    levels, discs, opts, _ = oproblems.build("cfg5_r1", with_rhs=False)
    d = discs[1]                                   # the 4^3 mesh
    patches = s3.vanka_star_patches(d)
    mesh = d.mesh
    v = int(np.flatnonzero(np.all(np.isclose(mesh.verts, 0.5), axis=1))[0])
    assert len(patches[v]) == 196                  # 3 x (15 vertices + 50 edges) + 1 pressure
    assert max(len(S) for S in patches) == 196


def test_transfers_reproduce_polynomials_and_galerkin():
    levels, discs, opts, _ = oproblems.build("cfg5_r1", with_rhs=False)
    fine, coarse = discs
    parent = synth.config_mesh_hierarchy("cfg5_r1")[-1].parent
    Pu = s3._scalar_interp(fine.V, coarse.V, fine.mesh, coarse.mesh, parent)
    Pp = s3._scalar_interp(fine.Q, coarse.Q, fine.mesh, coarse.mesh, parent)
    q2 = lambda X: X[:, 0] ** 2 + X[:, 1] * X[:, 2] - X[:, 2] + 0.5
    q1 = lambda X: 2 * X[:, 0] - X[:, 1] + 3 * X[:, 2] + 1
    assert np.abs(Pu @ q2(coarse.V.coords) - q2(fine.V.coords)).max() <= 1e-13
    assert np.abs(Pp @ q1(coarse.Q.coords) - q1(fine.Q.coords)).max() <= 1e-13
    assert np.abs(Pu @ np.ones(coarse.V.ndofs) - 1).max() <= 1e-13
    P = levels[1].P
    G = (P.T @ fine.K @ P - coarse.K)
    assert abs(G).max() <= 1e-12 * abs(coarse.K).max()


def test_adjoint_gradients_match_finite_differences_3d():
    name = "cube_tiny"
    mesh0 = synth.config_mesh_hierarchy(name)[-1]
    lv = synth.log_viscosity(mesh0.verts, seed=5)
    nrhs = 2

    def J_of(l, fn, T):
        levels, discs, opts, _ = oproblems.build(name, with_rhs=False, log_visc=l)
        d = discs[0]
        B = adjoint.forcing_rhs(d, fn)
        X = np.stack([_direct(d.K, d.null_vector(), b) for b in B])
        return adjoint.objective(X, T, d.nfu, 3), X, levels, discs, opts

    _, discs, _, _ = oproblems.build(name, with_rhs=False, log_visc=lv)
    d = discs[0]
    rng = np.random.default_rng(4)
    C, W, D = synth.gaussian_bump_params3d(nrhs, 6)
    X0 = d.V.coords
    fn = np.stack([np.stack(synth.gaussian_bump_forcing3d(X0[:, 0], X0[:, 1], X0[:, 2], C[i], W[i], D[i]))
                   for i in range(nrhs)])
    T = rng.standard_normal((nrhs, d.n)) * 0.01
    J0, X, levels, discs, opts = J_of(lv, fn, T)
    # adjoint states from direct solves (the multigrid adjoint is pinned in 2D and densely)
    G = adjoint.objective_gradient(X, T, d.nfu, 3)
    KT = discs[0].K.T.tocsr()
    Lam = np.stack([_direct(KT, d.null_vector(), g) for g in G])
    gl = adjoint.viscosity_gradient(discs[0], X, Lam)
    gf = adjoint.forcing_gradient(discs[0], Lam)
    h = 1e-5
    dl = rng.standard_normal(lv.shape)
    fd = (J_of(lv + h * dl, fn, T)[0] - J_of(lv - h * dl, fn, T)[0]) / (2 * h)
    assert abs(gl @ dl - fd) <= 1e-7 * abs(fd)
    df = rng.standard_normal(fn.shape)
    fdf = (J_of(lv, fn + 1e-3 * df, T)[0] - J_of(lv, fn - 1e-3 * df, T)[0]) / 2e-3
    assert abs(np.sum(gf * df) - fdf) <= 1e-9 * abs(fdf)
