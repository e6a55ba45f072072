"""Restarted flexible GMRES, right preconditioned (oracle).

Section 4 (solver paragraph): FGMRES with a Krylov subspace of at most 30
vectors, converged when the l2 norm of the residual has dropped by the
requested factor.  Flexible GMRES (Saad) stores the preconditioned vectors
z_j = B v_j and updates x with them.

Readings where the paper is silent:
  * Orthogonalisation is classical Gram-Schmidt applied twice (CGS2): h =
    V^T w, w -= V h, h2 = V^T w, w -= V h2, h += h2.
  * Givens rotations: rho = hypot(a, b), c = a/rho, s = b/rho.
  * A cycle ends when the Givens residual estimate |g_{j+1}| <= rtol * ||r_0||,
    on an exact breakdown (||w|| == 0), after `restart` iterations, or at maxit
    inner iterations in total.  x is then updated with Z y and the true
    residual b - K x formed; the solve has converged when the true residual
    satisfies ||b - K x|| <= rtol ||r_0|| (the paper's criterion is the
    residual itself), otherwise it restarts unless maxit is reached.
  * x_0 is the initial guess given (zero in every benchmark); r_0 = b - K x_0.

Pins: tests/test_oracle_fgmres.py -- with the identity preconditioner the
residual history equals brute-force minimal-residual solutions over the
explicit Krylov basis (numpy.linalg.lstsq); the solution of a nonsingular
system equals numpy.linalg.solve within rtol * cond.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np


@dataclass
class FgmresResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: float
    history: List[float] = field(default_factory=list)   # |g_{j+1}| / ||r_0|| per inner iteration


def fgmres(matvec: Callable, precond: Callable, b: np.ndarray, x0: np.ndarray = None,
           rtol: float = 1e-8, restart: int = 30, maxit: int = 1000) -> FgmresResult:
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    r0 = beta
    target = rtol * r0
    history: List[float] = []
    iters = 0
    if beta <= target or r0 == 0.0:
        return FgmresResult(x, 0, True, 0.0 if r0 == 0 else beta / r0, history)
    converged = False
    while True:
        V = np.zeros((n, restart + 1))
        Z = np.zeros((n, restart))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[:, 0] = r / beta
        ncols = 0
        for j in range(restart):
            Z[:, j] = precond(V[:, j])
            w = matvec(Z[:, j])
            h = V[:, : j + 1].T @ w
            w = w - V[:, : j + 1] @ h
            h2 = V[:, : j + 1].T @ w
            w = w - V[:, : j + 1] @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            a, c = H[j, j], H[j + 1, j]
            rho = np.hypot(a, c)
            cs[j], sn[j] = a / rho, c / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            ncols = j + 1
            history.append(abs(g[j + 1]) / r0)
            if abs(g[j + 1]) <= target or hn == 0.0 or iters >= maxit:
                break
            V[:, j + 1] = w / hn
        y = np.zeros(ncols)
        for i in range(ncols - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1: ncols] @ y[i + 1:]) / H[i, i]
        x = x + Z[:, :ncols] @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= target:
            converged = True
            break
        if iters >= maxit:
            break
        # restart: the cycle is exhausted, or the Givens estimate was below the
        # target while the true residual is not (rounding), or an exact breakdown
    return FgmresResult(x, iters, converged, beta / r0, history)
