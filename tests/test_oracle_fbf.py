"""Pins of the oracle's full-block-factorisation preconditioner (not gpu)."""
import numpy as np
import pytest

import synth
from oracle import element, fbf
from oracle import problems as oproblems
from oracle.discretization import assemble_stokes, cell_geometry


@pytest.mark.parametrize("k,expected", [(2, 14), (3, 38), (4, 74)])
def test_star_patch_size_closed_form(k, expected):
    """Interior vertex with n = 6 cells: 2 [1 + n(k-1) + n(k-1)(k-2)/2] velocity DoFs."""
    d = assemble_stokes(synth.structured_square(4), k, "TH")
    patches = fbf.star_patches(d)
    v = int(np.flatnonzero(np.all(np.isclose(d.mesh.verts, 0.5), axis=1))[0])
    # patches are listed per vertex that has free DoFs; every vertex has its own (v is interior)
    sizes = [len(S) for S in patches]
    n = 6
    assert 2 * (1 + n * (k - 1) + n * (k - 1) * (k - 2) // 2) == expected
    assert max(sizes) == expected
    # the patch of v contains v's own velocity DoFs
    own = d.u_index(0, np.array([v]))[0]
    assert any(own in S and len(S) == expected for S in patches)


def test_pressure_mass_inverse_reproduces_polynomials():
    """-S_inv applied to the moments b_i = int q psi_i gives the coefficients of q for q in P_{k-1}."""
    mesh = synth.alfeld_split(synth.jitter_interior(synth.structured_square(2), 0.05, seed=1))
    d = assemble_stokes(mesh, 3, "SV")
    Sinv = fbf.pressure_mass_inverse(d)
    kq = d.k - 1
    qpts, qw = element.quadrature(2 * kq + 2)
    psi, _ = element.eval_basis(kq, qpts)
    for q in (lambda x, y: np.ones_like(x), lambda x, y: x * y - 2 * y * y + x):
        b = np.zeros(d.nq)
        for c in range(mesh.cells.shape[0]):
            x0, J, adet, _ = cell_geometry(mesh.verts, mesh.cells[c])
            X = x0 + qpts @ J.T
            b[d.Q.cell_dofs[c]] += (qw * adet * q(X[:, 0], X[:, 1])) @ psi
        coef = -(Sinv @ b)
        assert np.abs(coef - q(d.Q.coords[:, 0], d.Q.coords[:, 1])).max() <= 1e-12


def test_exact_block_factorisation_is_a_generalised_inverse():
    """With A~^{-1} = A^{-1} and S~ the exact Schur complement -B A^{-1} B^T (pseudo-inverse
    for the constant-pressure kernel), the factorisation satisfies K P K = K."""
    mesh = synth.alfeld_split(synth.jitter_interior(synth.structured_square(2), 0.05, seed=1))
    d = assemble_stokes(mesh, 3, "SV")
    K = d.K.toarray()
    nu = 2 * d.nfu
    A, B = K[:nu, :nu], K[nu:, :nu]
    Ainv = np.linalg.inv(A)
    S = -B @ Ainv @ B.T
    Sp = np.linalg.pinv(S, rcond=1e-10)
    P = np.stack([fbf.fbf_apply(None, None, B, Sp, e, A_inv=lambda v: Ainv @ v) for e in np.eye(d.n)], axis=1)
    assert np.abs(K @ P @ K - K).max() <= 1e-9 * np.abs(K).max()


def test_velocity_levels_of_sv_hierarchy():
    levels, discs, opts, _ = oproblems.build("sv_small")
    vl = fbf.velocity_levels(levels, discs)
    assert [L.n for L in vl] == [2 * d.nfu for d in discs]
    for li in range(1, len(vl)):
        assert vl[li].P.shape == (vl[li - 1].n, vl[li].n)
    # A_l is the vector Laplacian: symmetric positive definite
    A = vl[-1].K.toarray()
    assert np.linalg.eigvalsh(A).min() > 0
