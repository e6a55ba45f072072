"""Pins of the oracle's additive Schwarz sweep against the dense eq. "eq:ASM"."""
import numpy as np
import pytest

import synth
from oracle import relax
from oracle.discretization import assemble_stokes
from oracle.patches import multiplicity_weights, vanka_star_patches


def _dense_Minv(K, patches, weights):
    n = K.shape[0]
    M = np.zeros((n, n))
    for i, S in enumerate(patches):
        inv = np.linalg.inv(K[np.ix_(S, S)])
        if weights is not None:
            inv = weights[i][:, None] * inv
        M[np.ix_(S, S)] += inv
    return M


CASES = [("TH", 2, synth.structured_square(2)), ("TH", 3, synth.structured_square(4)),
         ("SV", 2, synth.alfeld_split(synth.structured_square(1))),
         ("SV", 4, synth.alfeld_split(synth.structured_square(2)))]


@pytest.mark.parametrize("kind,k,mesh", CASES, ids=[f"{c[0]}{c[1]}" for c in CASES])
@pytest.mark.parametrize("weighted", [False, True])
def test_sweep_equals_dense_operator(kind, k, mesh, weighted):
    d = assemble_stokes(mesh, k, kind)
    patches = vanka_star_patches(d)
    W = multiplicity_weights(patches, d.n) if weighted else None
    factors = relax.setup_patches(d.K, patches)
    K = d.K.toarray()
    Minv = _dense_Minv(K, patches, W)
    rng = np.random.default_rng(11)
    b, x = rng.standard_normal(d.n), rng.standard_normal(d.n)
    w = 0.37
    x1 = relax.asm_sweeps(d.K, patches, factors, W, w, b, x, 1)
    ref = x + w * Minv @ (b - K @ x)
    assert np.abs(x1 - ref).max() <= 1e-12 * np.abs(ref).max()
    S = np.eye(d.n) - w * Minv @ K
    x3 = relax.asm_sweeps(d.K, patches, factors, W, w, b, x, 3)
    ref3 = x.copy()
    for _ in range(3):
        ref3 = S @ ref3 + w * Minv @ b
    assert np.abs(x3 - ref3).max() <= 1e-11 * np.abs(ref3).max()
    xt = relax.asm_sweeps(d.K, patches, factors, W, w, b, x, 1, transpose=True)
    reft = x + w * Minv.T @ (b - K.T @ x)
    assert np.abs(xt - reft).max() <= 1e-12 * np.abs(reft).max()


def _cheb_T(Y, nu):
    """T_nu(Y) by the three-term recurrence (matrix or scalar)."""
    I = np.eye(Y.shape[0]) if np.ndim(Y) == 2 else 1.0
    Tm, T = I, Y
    if nu == 0:
        return I
    for _ in range(nu - 1):
        Tm, T = T, 2 * (Y @ T if np.ndim(Y) == 2 else Y * T) - Tm
    return T


@pytest.mark.parametrize("kind,k,mesh", CASES[:3], ids=[f"{c[0]}{c[1]}" for c in CASES[:3]])
@pytest.mark.parametrize("nu", [1, 2, 4])
def test_chebyshev_error_propagator_closed_form(kind, k, mesh, nu):
    """x_nu - x* = T_nu((theta - M^{-1}K)/delta) / T_nu(theta/delta) (x_0 - x*) for b = K x*."""
    d = assemble_stokes(mesh, k, kind)
    patches = vanka_star_patches(d)
    factors = relax.setup_patches(d.K, patches)
    K = d.K.toarray()
    Minv = _dense_Minv(K, patches, None)
    emin, emax = 0.7, 9.3
    theta, delta = 0.5 * (emax + emin), 0.5 * (emax - emin)
    E = _cheb_T((theta * np.eye(d.n) - Minv @ K) / delta, nu) / _cheb_T(theta / delta, nu)
    rng = np.random.default_rng(21)
    xs, x0 = rng.standard_normal(d.n), rng.standard_normal(d.n)
    b = K @ xs
    got = relax.chebyshev_sweeps(d.K, patches, factors, None, emin, emax, b, x0, nu)
    ref = xs + E @ (x0 - xs)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_arnoldi_estimates_largest_eigenvalue():
    d = assemble_stokes(synth.refine_uniform(synth.delaunay_square(8, seed=3)), 2, "TH")
    patches = vanka_star_patches(d)
    factors = relax.setup_patches(d.K, patches)
    K = d.K.toarray()
    ev = np.linalg.eigvals(_dense_Minv(K, patches, None) @ K)
    lam = relax.estimate_lambda_max(d.K, patches, factors, None, 20)
    assert 0.995 * ev.real.max() <= lam <= 1.0001 * ev.real.max()


def _arnoldi_case():
    d = assemble_stokes(synth.refine_uniform(synth.delaunay_square(8, seed=3)), 2, "TH")
    patches = vanka_star_patches(d)
    factors = relax.setup_patches(d.K, patches)
    A = _dense_Minv(d.K.toarray(), patches, None) @ d.K.toarray()
    return d, patches, factors, A


def test_arnoldi_basis_is_orthonormal_and_satisfies_the_arnoldi_relation():
    """Classical Gram-Schmidt applied twice keeps the basis orthonormal to rounding over 60 steps,
    where a single pass loses orthogonality to ~1e-6 on this operator (shown below with the same
    start vector); M^{-1} K V_k = V_{k+1} H with H upper Hessenberg (a transposed or shifted index
    in H fails it)."""
    d, patches, factors, A = _arnoldi_case()
    V, H, k = relax.arnoldi(d.K, patches, factors, None, 60)
    assert k == 60
    G = V.T @ V
    assert np.abs(G - np.eye(k + 1)).max() <= 1e-13
    assert np.abs(A @ V[:, :k] - V @ H).max() <= 1e-12 * np.abs(A).max()
    assert np.allclose(np.tril(H, -2), 0.0)
    # single-pass classical Gram-Schmidt on the same operator: orthogonality is lost
    n = A.shape[0]
    W = np.zeros((n, k + 1))
    v = relax.power_start(n)
    W[:, 0] = v / np.linalg.norm(v)
    for j in range(k):
        w = A @ W[:, j]
        w = w - W[:, : j + 1] @ (W[:, : j + 1].T @ w)
        W[:, j + 1] = w / np.linalg.norm(w)
    assert np.abs(W.T @ W - np.eye(k + 1)).max() > 1e-8


@pytest.mark.parametrize("k", [3, 6])
def test_ritz_values_equal_brute_force_rayleigh_ritz(k):
    """The Ritz values of k Arnoldi steps are the eigenvalues of Q^T A Q for an orthonormal basis Q of
    the Krylov space span{v, A v, ..., A^{k-1} v}, built here explicitly and orthonormalised by
    numpy's QR."""
    d, patches, factors, A = _arnoldi_case()
    V, H, kk = relax.arnoldi(d.K, patches, factors, None, k)
    v = relax.power_start(A.shape[0])
    Kr = np.empty((A.shape[0], k))
    Kr[:, 0] = v / np.linalg.norm(v)
    for j in range(1, k):
        Kr[:, j] = A @ Kr[:, j - 1]
        Kr[:, j] /= np.linalg.norm(Kr[:, j])
    Q, _ = np.linalg.qr(Kr)
    want = np.sort_complex(np.linalg.eigvals(Q.T @ A @ Q))
    got = np.sort_complex(np.linalg.eigvals(H[:kk, :kk]))
    assert np.abs(got - want).max() <= 1e-8 * np.abs(want).max()
    assert relax.estimate_lambda_max(d.K, patches, factors, None, k) == pytest.approx(want.real.max(), rel=1e-8)
