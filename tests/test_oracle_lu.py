"""Pins of the oracle's dense LU (Section 3.4: patch systems solved by LU)."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import lu
from oracle.discretization import assemble_stokes
from oracle.patches import vanka_star_patches


def _patch_mats():
    d = assemble_stokes(synth.refine_uniform(synth.delaunay_square(8, seed=1)), 3, "TH")
    K = d.K
    out = [K[S][:, S].toarray() for S in vanka_star_patches(d)[:25]]
    dsv = assemble_stokes(synth.alfeld_split(synth.structured_square(2)), 4, "SV")
    out += [dsv.K[S][:, S].toarray() for S in vanka_star_patches(dsv)[:8]]
    return out


@pytest.mark.parametrize("seed", range(4))
def test_lu_matches_lapack_getrf_random(seed):
    A = np.random.default_rng(seed).standard_normal((37, 37))
    LU, piv = lu.lu_factor(A)
    LU2, piv2 = scipy.linalg.lu_factor(A)
    assert np.array_equal(piv, piv2)
    assert np.abs(LU - LU2).max() < 1e-12 * np.abs(LU2).max()


def test_lu_reconstructs_patch_matrices_and_matches_lapack():
    eps = np.finfo(float).eps
    for A in _patch_mats():
        m = A.shape[0]
        LU, piv = lu.lu_factor(A)
        L = np.tril(LU, -1) + np.eye(m)
        U = np.triu(LU)
        PA = A.copy()
        for k in range(m):
            PA[[k, piv[k]]] = PA[[piv[k], k]]
        assert np.abs(PA - L @ U).max() <= 10 * m * eps * np.abs(A).max()
        _, piv2 = scipy.linalg.lu_factor(A)
        assert np.array_equal(piv, piv2)


def test_solves_match_numpy():
    for A in _patch_mats()[:10]:
        b = np.random.default_rng(3).standard_normal(A.shape[0])
        LU, piv = lu.lu_factor(A)
        cond = np.linalg.cond(A)
        x = lu.lu_solve(LU, piv, b)
        xt = lu.lu_solve_transposed(LU, piv, b)
        ref = np.linalg.solve(A, b)
        reft = np.linalg.solve(A.T, b)
        assert np.linalg.norm(x - ref) <= 1e-13 * cond * np.linalg.norm(ref)
        assert np.linalg.norm(xt - reft) <= 1e-13 * cond * np.linalg.norm(reft)


def test_singular_patch_is_reported():
    A = np.random.default_rng(0).standard_normal((6, 6))
    A[:, 2] = 0.0
    with pytest.raises(lu.SingularPatch):
        lu.lu_factor(A)
