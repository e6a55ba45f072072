"""Additive Schwarz (Vanka) relaxation (oracle).

Section 3.4, eq. "eq:ASM": M^{-1} = sum_i I^(i)^T W_i (K^(i))^{-1} I^(i) with
K^(i) = I^(i) K I^(i)^T, and one relaxation sweep is x <- x + omega M^{-1}
(b - K x).  All patches use the same residual (additive / block Jacobi).

Reading where the paper is silent: the contributions of the patches to one
DoF are summed in ascending patch order, then scaled by omega and added to x.

Section 4 (solver set-up paragraph): in the experiments the damping is set
through Chebyshev iteration using an estimate of the largest eigenvalue of
M^{-1} K; each Chebyshev iteration applies the additive Schwarz
preconditioner once.  Reading where the paper is silent: the Chebyshev
semi-iteration of Saad (Iterative Methods, Alg. "Chebyshev acceleration")
on the interval [lo * lam, hi * lam] with lam the estimate; lam is the
largest real part of the Ritz values of a fixed number of Arnoldi steps on
M^{-1} K from the deterministic start vector v_j = 1 + sin(j)/2 (the same
kind of Krylov estimate PETSc's Chebyshev smoother uses).

Pins: tests/test_oracle_relax.py -- one sweep equals x + omega M^{-1}(b-Kx)
with M^{-1} formed densely from numpy.linalg.inv of every patch matrix; nu
sweeps equal the nu-th power of the dense propagator; the transposed sweep
equals the dense transpose; nu Chebyshev steps equal the closed form of the
Chebyshev error propagator T_nu((theta - M^{-1}K)/delta) / T_nu(theta/delta);
the Arnoldi basis is orthonormal to rounding and satisfies M^{-1} K V_k =
V_{k+1} H; its Ritz values equal a brute-force Rayleigh-Ritz projection onto an
explicitly built Krylov basis; the estimate is within 0.5% of the largest real
part of the dense eigenvalues of M^{-1}K.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from .lu import lu_factor, lu_solve, lu_solve_transposed


def extract_patch(K, S: np.ndarray) -> np.ndarray:
    """K^(i) = I^(i) K I^(i)^T as a dense matrix."""
    return K[S][:, S].toarray()


def setup_patches(K, patches: List[np.ndarray]):
    return [lu_factor(extract_patch(K, S)) for S in patches]


def asm_correction(patches, factors, weights: Optional[list], r: np.ndarray, transpose: bool = False) -> np.ndarray:
    """sum_i I^(i)^T W_i (K^(i))^{-1} I^(i) r, patches visited in ascending order.

    With transpose=True the adjoint operator sum_i I^(i)^T (K^(i))^{-T} W_i I^(i) r.
    """
    dx = np.zeros_like(r)
    for i, S in enumerate(patches):
        LU, piv = factors[i]
        if not transpose:
            y = lu_solve(LU, piv, r[S])
            if weights is not None:
                y = weights[i] * y
        else:
            rr = r[S] if weights is None else weights[i] * r[S]
            y = lu_solve_transposed(LU, piv, rr)
        dx[S] += y
    return dx


def asm_sweeps(K, patches, factors, weights, omega: float, b: np.ndarray, x: np.ndarray, nu: int,
               transpose: bool = False) -> np.ndarray:
    """nu sweeps of x <- x + omega M^{-1} (b - K x) (or with M^{-T}, K^T when transpose)."""
    x = np.array(x, dtype=np.float64, copy=True)
    KK = K.T.tocsr() if transpose else K
    for _ in range(nu):
        r = b - KK @ x
        x = x + omega * asm_correction(patches, factors, weights, r, transpose)
    return x


def power_start(n: int) -> np.ndarray:
    return 1.0 + 0.5 * np.sin(np.arange(n, dtype=np.float64))


def arnoldi(K, patches, factors, weights, iters: int, transpose: bool = False):
    """`iters` Arnoldi steps on M^{-1} K from v_0 = power_start / ||.||, classical Gram-Schmidt
    applied twice.  Returns (V, H, k): the orthonormal basis V (n x (k+1)), the upper Hessenberg
    H ((k+1) x k) with M^{-1} K V[:, :k] = V H, and the number of steps k taken (fewer on an
    exact breakdown)."""
    KK = K.T.tocsr() if transpose else K
    n = K.shape[0]
    k = min(iters, n)
    V = np.zeros((n, k + 1))
    H = np.zeros((k + 1, k))
    v = power_start(n)
    V[:, 0] = v / np.linalg.norm(v)
    for j in range(k):
        w = asm_correction(patches, factors, weights, KK @ V[:, j], transpose)
        h = V[:, : j + 1].T @ w
        w = w - V[:, : j + 1] @ h
        h2 = V[:, : j + 1].T @ w
        w = w - V[:, : j + 1] @ h2
        H[: j + 1, j] = h + h2
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            k = j + 1
            break
        V[:, j + 1] = w / H[j + 1, j]
    return V, H, k


def estimate_lambda_max(K, patches, factors, weights, iters: int, transpose: bool = False) -> float:
    """Largest real part of the Ritz values of `iters` Arnoldi steps on M^{-1} K: the
    eigenvalues of the leading k x k block of the Hessenberg matrix (numpy.linalg.eigvals as a
    library step)."""
    V, H, k = arnoldi(K, patches, factors, weights, iters, transpose)
    return float(np.linalg.eigvals(H[:k, :k]).real.max())


def chebyshev_sweeps(K, patches, factors, weights, emin: float, emax: float, b: np.ndarray, x: np.ndarray, nu: int,
                     transpose: bool = False) -> np.ndarray:
    """nu steps of Chebyshev acceleration of x <- x + M^{-1}(b - K x) for eigenvalues in [emin, emax]."""
    x = np.array(x, dtype=np.float64, copy=True)
    KK = K.T.tocsr() if transpose else K
    theta = 0.5 * (emax + emin)
    delta = 0.5 * (emax - emin)
    sigma = theta / delta
    rho_prev = 1.0 / sigma
    d = None
    for it in range(nu):
        z = asm_correction(patches, factors, weights, b - KK @ x, transpose)
        if it == 0:
            d = z / theta
        else:
            rho = 1.0 / (2.0 * sigma - rho_prev)
            d = (rho * rho_prev) * d + (2.0 * rho / delta) * z
            rho_prev = rho
        x = x + d
    return x
