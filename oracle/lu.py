"""Dense LU with partial pivoting and triangular solves (oracle).

Section 3.4: each patch system K^(i) = I^(i) K I^(i)^T is solved exactly by
LU factorisation.  The paper does not state the pivoting policy; the reading
here is textbook right-looking Gaussian elimination with partial pivoting
(largest |entry| of the current column on or below the diagonal, ties to the
lowest row index), for every patch alike.

A pivot with |u_kk| <= 1e-14 * ||K^(i)||_inf is reported as singular.

Pins: tests/test_oracle_lu.py -- P K = L U to 10 m eps, pivots and factors
equal to LAPACK getrf through scipy.linalg.lu_factor, solve against
numpy.linalg.solve.
"""
from __future__ import annotations

import numpy as np

SINGULAR_RTOL = 1e-14


class SingularPatch(ArithmeticError):
    pass


def lu_factor(A: np.ndarray):
    """Return (LU, piv): unit-lower L below the diagonal, U on and above; piv[k] = row swapped with k."""
    LU = np.array(A, dtype=np.float64, copy=True)
    m = LU.shape[0]
    piv = np.arange(m)
    scale = np.abs(LU).sum(axis=1).max() if m else 0.0
    for k in range(m):
        p = k + int(np.argmax(np.abs(LU[k:, k])))
        if abs(LU[p, k]) <= SINGULAR_RTOL * scale:
            raise SingularPatch(f"zero pivot at column {k}")
        piv[k] = p
        if p != k:
            LU[[k, p], :] = LU[[p, k], :]
        LU[k + 1:, k] /= LU[k, k]
        LU[k + 1:, k + 1:] -= np.outer(LU[k + 1:, k], LU[k, k + 1:])
    return LU, piv


def lu_solve(LU: np.ndarray, piv: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve A x = b from the factors of lu_factor (forward then backward substitution)."""
    x = np.array(b, dtype=np.float64, copy=True)
    m = LU.shape[0]
    for k in range(m):
        p = piv[k]
        if p != k:
            x[k], x[p] = x[p], x[k]
    for i in range(m):
        x[i] -= LU[i, :i] @ x[:i]
    for i in range(m - 1, -1, -1):
        x[i] = (x[i] - LU[i, i + 1:] @ x[i + 1:]) / LU[i, i]
    return x


def lu_solve_transposed(LU: np.ndarray, piv: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve A^T x = b from the same factors: U^T w = b, L^T v = w, x = P^T v."""
    x = np.array(b, dtype=np.float64, copy=True)
    m = LU.shape[0]
    for i in range(m):
        x[i] = (x[i] - LU[:i, i] @ x[:i]) / LU[i, i]
    for i in range(m - 1, -1, -1):
        x[i] -= LU[i + 1:, i] @ x[i + 1:]
    for k in range(m - 1, -1, -1):
        p = piv[k]
        if p != k:
            x[k], x[p] = x[p], x[k]
    return x
