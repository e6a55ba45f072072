"""hMG / phMG V-cycles and the coarse direct solve (oracle).

Section 3.1, eq. "eq:TG-operator": one h-level of the cycle is nu pre-sweeps
of relaxation, the coarse correction x += P_l K_{l+1}^{-1} R_l (b - K_l x),
then nu post-sweeps; applied recursively down to an exact coarse solve.
Section 3.2, eq. "eq:DC-TG-operator": on the p-levels (the high-order level 0
and, for gradual coarsening, intermediate orders) the same shape with nu_p
sweeps, where the correction on K_1 is (I - G_1) K_1^{-1}, G_1 being the
error propagator of n_V successive hMG cycles.  The paper's solver section
uses an exact direct solve on the coarsest grid.

Readings where the paper is silent:
  * nu_1 = nu_2 (= nu_p on p-levels, nu_h on h-levels); the same omega on
    every level; every cycle starts from x = 0.
  * (I - G_1) K_1^{-1} applied to b_1 is n_V stationary hMG iterations from
    e = 0, each a V-cycle started from the current e.
  * The smoother is damped Richardson (omega) or, as in the paper's
    experiments, Chebyshev acceleration over [cheb_lo, cheb_hi] * lambda_max.
  * With all of the boundary Dirichlet the coarsest matrix is singular with
    kernel z (constant pressure); the coarse solve is the bordered system
    [K_c z; z^T 0][x; lam] = [b; 0], factored once by the oracle's LU.

Pins: tests/test_oracle_multigrid.py -- the coarse solve equals
numpy.linalg.lstsq; a two-level cycle equals the dense propagator
(I - w M^{-1} K)^nu (I - P K_c^+ R K)(I - w M^{-1} K)^nu applied to unit
vectors; phMG with n_V cycles equals the dense defect-correction form.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .lu import lu_factor, lu_solve, lu_solve_transposed
from .relax import asm_sweeps, chebyshev_sweeps, estimate_lambda_max, setup_patches


@dataclass
class Level:
    K: sp.csr_matrix
    patches: Optional[list] = None       # list of index arrays (None on the coarsest level)
    weights: Optional[list] = None       # W_i diagonals, or None for W_i = I
    P: Optional[sp.csr_matrix] = None    # prolongation from the next coarser level
    factors: Optional[list] = None
    coarse: Optional[tuple] = None       # (LU, piv, bordered?) on the coarsest level
    null: Optional[np.ndarray] = None    # kernel vector on the coarsest level
    lmax: Optional[float] = None         # estimate of the largest eigenvalue of M^{-1} K (Chebyshev)

    @property
    def n(self) -> int:
        return self.K.shape[0]


@dataclass
class CycleOpts:
    nu_p: int = 2
    nu_h: int = 2
    n_v: int = 1
    n_plevels: int = 1       # number of levels relaxed with nu_p (0 = pure hMG)
    omega: float = 0.5       # Richardson damping
    smoother: str = "richardson"   # or "chebyshev"
    cheb_lo: float = 0.1     # Chebyshev interval [cheb_lo, cheb_hi] * lambda_max estimate
    cheb_hi: float = 1.1
    eig_iters: int = 20      # Arnoldi steps of the lambda_max estimate


def setup(levels: List[Level], opts: Optional[CycleOpts] = None) -> None:
    """Patch LU on every non-coarsest level (and the lambda_max estimate for
    Chebyshev smoothing); bordered dense LU on the coarsest."""
    for L in levels[:-1]:
        L.factors = setup_patches(L.K, L.patches)
        if opts is not None and opts.smoother == "chebyshev":
            L.lmax = estimate_lambda_max(L.K, L.patches, L.factors, L.weights, opts.eig_iters)
    C = levels[-1]
    Kc = C.K.toarray()
    if C.null is not None:
        z = C.null
        n = Kc.shape[0]
        Kb = np.zeros((n + 1, n + 1))
        Kb[:n, :n] = Kc
        Kb[:n, n] = z
        Kb[n, :n] = z
        LU, piv = lu_factor(Kb)
        C.coarse = (LU, piv, True)
    else:
        LU, piv = lu_factor(Kc)
        C.coarse = (LU, piv, False)


def coarse_solve(C: Level, b: np.ndarray, transpose: bool = False) -> np.ndarray:
    LU, piv, bordered = C.coarse
    rhs = np.concatenate([b, [0.0]]) if bordered else b
    x = lu_solve_transposed(LU, piv, rhs) if transpose else lu_solve(LU, piv, rhs)
    return x[:-1] if bordered else x


def _relax(L: Level, opts: CycleOpts, b, x, nu, transpose):
    if opts.smoother == "chebyshev":
        # the transposed cycle keeps the forward interval, so it is the exact adjoint
        lam = L.lmax
        return chebyshev_sweeps(L.K, L.patches, L.factors, L.weights, opts.cheb_lo * lam, opts.cheb_hi * lam,
                                b, x, nu, transpose)
    return asm_sweeps(L.K, L.patches, L.factors, L.weights, opts.omega, b, x, nu, transpose)


def cycle(levels: List[Level], opts: CycleOpts, l: int, b: np.ndarray, x: np.ndarray,
          transpose: bool = False) -> np.ndarray:
    """One cycle on level l with initial guess x; returns the new x."""
    if l == len(levels) - 1:
        return coarse_solve(levels[l], b, transpose)
    L = levels[l]
    K = L.K.T.tocsr() if transpose else L.K
    nu = opts.nu_p if l < opts.n_plevels else opts.nu_h
    x = _relax(L, opts, b, x, nu, transpose)
    r = b - K @ x
    P = levels[l + 1].P
    bc = P.T @ r
    e = np.zeros(levels[l + 1].n)
    if l + 1 < opts.n_plevels or l + 1 == len(levels) - 1 or l >= opts.n_plevels:
        # next level is a p-level, the coarsest level, or we are inside hMG: one cycle
        e = cycle(levels, opts, l + 1, bc, e, transpose)
    else:
        # last p-level: G_1 = n_V successive hMG cycles on K_{l+1}
        for _ in range(opts.n_v):
            e = cycle(levels, opts, l + 1, bc, e, transpose)
    x = x + P @ e
    x = _relax(L, opts, b, x, nu, transpose)
    return x


def vcycle(levels: List[Level], opts: CycleOpts, b: np.ndarray, transpose: bool = False) -> np.ndarray:
    """Preconditioner application z = B b (x starts at 0)."""
    x = np.zeros(levels[0].n)
    if opts.n_plevels == 0:
        for _ in range(opts.n_v):
            x = cycle(levels, opts, 0, b, x, transpose)
        return x
    return cycle(levels, opts, 0, b, x, transpose)
