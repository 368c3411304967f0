"""Pins of the reference-element data (closed forms and exactness)."""
import numpy as np
import pytest

from oracle import nodes


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_gll_quadrature_exact_to_degree_2p_minus_1(p):
    xi, w, _ = nodes.gll(p)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13
    # degree 2p is not integrated exactly (the rule has 2p-1 exactness only)
    assert abs(np.dot(w, xi ** (2 * p)) - 2.0 / (2 * p + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_gll_known_nodes_and_symmetry(p):
    xi, w, D = nodes.gll(p)
    assert np.allclose(xi, -xi[::-1], atol=1e-15)
    assert np.allclose(w, w[::-1], atol=1e-15)
    # D maps symmetric nodes antisymmetrically: D[i,j] = -D[p-i, p-j]
    assert np.allclose(D, -D[::-1, ::-1], atol=1e-13)
    if p == 2:
        assert np.allclose(xi, [-1, 0, 1]) and np.allclose(w, [1 / 3, 4 / 3, 1 / 3])
    if p == 4:
        assert np.allclose(xi, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1])
        assert np.allclose(w, [0.1, 49 / 90, 32 / 45, 49 / 90, 0.1])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_derivative_matrix_exact_on_polynomials(p):
    xi, _, D = nodes.gll(p)
    for k in range(p + 1):
        assert np.allclose(D @ xi ** k, k * xi ** max(k - 1, 0) if k else 0.0, atol=1e-12)
    # closed-form corner entries
    assert abs(D[0, 0] + p * (p + 1) / 4) < 1e-14 and abs(D[p, p] - p * (p + 1) / 4) < 1e-14
    # generic Lagrange derivative agrees with the GLL closed form
    assert np.allclose(nodes.lagrange_derivative(xi), D, atol=1e-12)


def test_gauss_legendre_and_interpolation():
    xi, w, D = nodes.gl(4)
    for k in range(10):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13
    xc, _, _ = nodes.gll(2)
    xf = np.linspace(-1, 1, 7)
    L = nodes.lagrange_eval(xc, xf)
    # interpolation reproduces quadratics exactly, and the rows sum to one
    assert np.allclose(L @ (xc ** 2 - 0.3 * xc), xf ** 2 - 0.3 * xf)
    assert np.allclose(L.sum(1), 1.0)
