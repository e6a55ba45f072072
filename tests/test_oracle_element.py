"""Pins of the oracle's reference element and quadrature (not gpu)."""
from math import factorial

import numpy as np
import pytest

from oracle import element


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_nodal_basis_is_kronecker_at_nodes(k):
    phi, _ = element.eval_basis(k, element.node_points(k))
    assert np.allclose(phi, np.eye(phi.shape[0]), atol=1e-11)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_basis_partition_of_unity_and_gradient_sum(k):
    pts = np.random.default_rng(0).uniform(0, 0.5, size=(7, 2))
    phi, dphi = element.eval_basis(k, pts)
    assert np.allclose(phi.sum(axis=1), 1.0, atol=1e-12)
    assert np.allclose(dphi.sum(axis=1), 0.0, atol=1e-10)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_basis_reproduces_linear_function(k):
    # sum_n x_n phi_n(x) = x for any Lagrange basis of degree >= 1
    nodes = element.node_points(k)
    pts = np.random.default_rng(1).uniform(0, 0.5, size=(5, 2))
    phi, dphi = element.eval_basis(k, pts)
    assert np.allclose(phi @ nodes, pts, atol=1e-12)
    assert np.allclose(np.einsum("qnj,ni->qij", dphi, nodes), np.eye(2)[None], atol=1e-10)


@pytest.mark.parametrize("deg", [0, 2, 5, 8, 12])
def test_quadrature_exact_for_monomials(deg):
    # int over the reference triangle of x^a y^b = a! b! / (a + b + 2)!
    pts, w = element.quadrature(deg)
    for a in range(deg + 1):
        b = deg - a
        exact = factorial(a) * factorial(b) / factorial(a + b + 2)
        assert abs(np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b) - exact) < 1e-14


def test_multi_index_order():
    assert element.multi_indices(2) == ((0, 0, 2), (0, 1, 1), (0, 2, 0), (1, 0, 1), (1, 1, 0), (2, 0, 0))
