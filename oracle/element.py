"""Reference triangle: Lagrange nodes, nodal basis, quadrature (oracle).

Section 2.1 uses continuous P_k velocities with P_{k-1} continuous (Taylor-Hood)
or discontinuous (Scott-Vogelius) pressures.  The paper does not fix the node
placement; this oracle reads it as equispaced Lagrange nodes.

Route chosen here (deliberately different from the GPU path's front-end):
  * basis: the monomials x^i y^j (i+j <= k) with a Vandermonde matrix inverted
    at the nodes, so phi_n = sum_m C[m, n] x^i_m y^j_m;
  * quadrature: collapsed (Duffy) tensor Gauss-Legendre on [0,1]^2 with the
    Jacobian (1 - t) written out explicitly.

Pins: tests/test_oracle_element.py (nodal property, partition of unity,
exact monomial integrals), plus the MMS convergence rates of the whole
discretisation.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def multi_indices(k: int):
    """All barycentric multi-indices (a0, a1, a2), a0+a1+a2 = k, ascending lexicographic."""
    out = []
    for a0 in range(k + 1):
        for a1 in range(k + 1 - a0):
            out.append((a0, a1, k - a0 - a1))
    return tuple(out)


def node_points(k: int) -> np.ndarray:
    """Reference coordinates (xi, eta) = (a1/k, a2/k) of each multi-index (k >= 1)."""
    mi = multi_indices(k)
    if k == 0:
        return np.array([[1.0 / 3.0, 1.0 / 3.0]])
    return np.array([[a1 / k, a2 / k] for (_, a1, a2) in mi], dtype=np.float64)


def _monomial_exponents(k: int):
    return [(i, j) for d in range(k + 1) for i in range(d, -1, -1) for j in [d - i]]


@lru_cache(maxsize=None)
def basis_coefficients(k: int) -> np.ndarray:
    """C with V C = I, V[n, m] = x_n^i_m y_n^j_m (Vandermonde at the nodes)."""
    pts = node_points(k)
    exps = _monomial_exponents(k)
    V = np.array([[x ** i * y ** j for (i, j) in exps] for (x, y) in pts])
    return np.linalg.inv(V)


def eval_basis(k: int, pts: np.ndarray):
    """Values and reference gradients of all nodal basis functions at pts.

    Returns (phi, dphi) with phi[q, n] and dphi[q, n, 0:2].
    """
    C = basis_coefficients(k)
    exps = _monomial_exponents(k)
    x, y = pts[:, 0], pts[:, 1]
    M = np.stack([x ** i * y ** j for (i, j) in exps], axis=1)
    Mx = np.stack([(i * x ** (i - 1) * y ** j if i > 0 else np.zeros_like(x)) for (i, j) in exps], axis=1)
    My = np.stack([(j * x ** i * y ** (j - 1) if j > 0 else np.zeros_like(x)) for (i, j) in exps], axis=1)
    phi = M @ C
    dphi = np.stack([Mx @ C, My @ C], axis=2)
    return phi, dphi


@lru_cache(maxsize=None)
def quadrature(degree: int):
    """Points and weights on the reference triangle exact for total degree <= degree.

    Collapsed map xi = s (1 - t), eta = t on [0,1]^2; the integrand picks up
    the Jacobian (1 - t), so n = degree // 2 + 2 Gauss-Legendre points per
    direction are enough.
    """
    n = degree // 2 + 2
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    for a in range(n):
        for b in range(n):
            s, t = g[a], g[b]
            pts.append((s * (1.0 - t), t))
            wts.append(w[a] * w[b] * (1.0 - t))
    return np.array(pts), np.array(wts)
