"""End-to-end pins of the oracle solver: FGMRES + phMG / hMG V-cycles."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fgmres, multigrid, problems
from oracle.discretization import divergence_at_quadrature


def _direct(K, z, b):
    Kb = sp.bmat([[K, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]], format="csc")
    return spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:-1]


def _normalise(x, nfu):
    y = x.copy()
    y[2 * nfu:] -= y[2 * nfu:].mean()
    return y


def test_cfg1_fgmres_hmg_converges_to_direct_solution():
    levels, discs, opts, b = problems.build("cfg1")
    multigrid.setup(levels, opts)
    K = levels[0].K
    res = fgmres.fgmres(lambda v: K @ v, lambda v: multigrid.vcycle(levels, opts, v), b, rtol=1e-8)
    assert res.converged and res.iters < 30
    assert np.linalg.norm(b - K @ res.x) <= 1e-8 * np.linalg.norm(b) * 1.0001
    ref = _direct(K, discs[0].null_vector(), b)
    d = discs[0]
    err = np.linalg.norm(_normalise(res.x, d.nfu) - _normalise(ref, d.nfu)) / np.linalg.norm(ref)
    assert err < 1e-6


def test_scott_vogelius_phmg_solve_is_divergence_free():
    """Section 2.1: with SV, div u_h = 0 pointwise once the discrete system is solved."""
    levels, discs, opts, b = problems.build("sv_small")
    multigrid.setup(levels, opts)
    K = levels[0].K
    res = fgmres.fgmres(lambda v: K @ v, lambda v: multigrid.vcycle(levels, opts, v), b, rtol=1e-12)
    assert res.converged
    div = divergence_at_quadrature(discs[0], res.x)
    assert np.abs(div).max() < 1e-10
