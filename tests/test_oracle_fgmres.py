"""Pins of the oracle's restarted FGMRES (Section 4: FGMRES(30))."""
import numpy as np
import pytest

from oracle.fgmres import fgmres


def _krylov_min_residual(A, b, x0, basis_cols):
    """min_y ||b - A(x0 + Q y)|| over the span of the given columns (brute force)."""
    Q, _ = np.linalg.qr(basis_cols)
    r0 = b - A @ x0
    y = np.linalg.lstsq(A @ Q, r0, rcond=None)[0]
    return np.linalg.norm(r0 - A @ Q @ y)


def _problem(n=40, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    return A, b


def test_identity_preconditioned_history_is_minimal_residual():
    A, b = _problem()
    x0 = np.random.default_rng(9).standard_normal(b.shape)
    res = fgmres(lambda v: A @ v, lambda v: v.copy(), b, x0=x0, rtol=1e-10, restart=30)
    r0 = np.linalg.norm(b - A @ x0)
    # orthonormal basis of K_j(A, r0) by repeated multiplication + two rounds of
    # modified Gram-Schmidt (a route independent of the CGS2/Givens code under test)
    kry = [(b - A @ x0) / r0]
    for j in range(1, len(res.history) + 1):
        ref = _krylov_min_residual(A, b, x0, np.stack(kry, axis=1)) / r0
        assert abs(res.history[j - 1] - ref) <= 1e-9 * ref + 1e-13, j
        w = A @ kry[-1]
        for _ in range(2):
            for q in kry:
                w = w - (q @ w) * q
        kry.append(w / np.linalg.norm(w))
    assert res.converged
    assert np.linalg.norm(res.x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.cond(A) * np.linalg.norm(b)


def test_flexible_preconditioner_minimises_over_z_span():
    A, b = _problem(30, 1)
    rng = np.random.default_rng(4)
    scales = [np.exp(rng.uniform(-0.5, 0.5, size=b.shape)) for _ in range(40)]
    calls = []

    def prec(v):
        z = scales[len(calls)] * v
        calls.append(z)
        return z

    res = fgmres(lambda v: A @ v, prec, b, rtol=1e-12, restart=30)
    for j in range(1, min(len(res.history), 30) + 1):
        ref = _krylov_min_residual(A, b, np.zeros_like(b), np.stack(calls[:j], axis=1)) / np.linalg.norm(b)
        assert abs(res.history[j - 1] - ref) <= 1e-9 * ref + 1e-12, j


def test_restart_and_maxit():
    A, b = _problem(60, 2)
    res = fgmres(lambda v: A @ v, lambda v: v.copy(), b, rtol=1e-10, restart=5, maxit=1000)
    assert res.converged and res.iters > 5
    assert np.linalg.norm(b - A @ res.x) <= 1.01e-10 * np.linalg.norm(b) * 10
    res2 = fgmres(lambda v: A @ v, lambda v: v.copy(), b, rtol=1e-14, restart=5, maxit=7)
    assert not res2.converged and res2.iters == 7


def test_exact_solution_in_first_step():
    A = np.diag(np.arange(1.0, 6.0))
    b = np.zeros(5)
    b[2] = 3.0
    res = fgmres(lambda v: A @ v, lambda v: v.copy(), b, rtol=1e-12)
    assert res.iters == 1 and res.converged
    assert np.allclose(res.x, [0, 0, 1, 0, 0])
