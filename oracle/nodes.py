"""Reference-element data: nodes, weights, derivative and interpolation matrices.

The auxiliary grid carries degree-q tensor-product nodal polynomials whose
nodes also define the quadrature rule (Sec. 6.1 and Sec. 6.2 of the paper).
The library uses Gauss-Lobatto-Legendre (GLL) nodes, so that nodal face values
exist; Gauss-Legendre (GL) nodes, the family the paper names, are provided for
completeness.

Test infrastructure only; see the package docstring.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def legendre_value(p, x):
    """P_p(x) by the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    x = np.asarray(x, dtype=np.float64)
    if p == 0:
        return np.ones_like(x)
    pm, pc = np.ones_like(x), x.copy()
    for k in range(1, p):
        pm, pc = pc, ((2 * k + 1) * x * pc - k * pm) / (k + 1)
    return pc


def gll(p):
    """GLL nodes xi_0=-1 < ... < xi_p=1, weights and derivative matrix for degree p.

    Nodes: the end points and the roots of P_p'.  Weights: 2/(p(p+1) P_p(xi_i)^2).
    Derivative matrix Dhat[i, j] = l_j'(xi_i) for the Lagrange basis l_j on the
    nodes: P_p(xi_i) / (P_p(xi_j) (xi_i - xi_j)) off the diagonal,
    -p(p+1)/4 at (0, 0), +p(p+1)/4 at (p, p), 0 elsewhere on the diagonal.
    """
    if p < 1:
        raise ValueError("GLL needs degree >= 1")
    coeffs = np.zeros(p + 1)
    coeffs[p] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(coeffs)))) if p > 1 else np.array([])
    xi = np.concatenate([[-1.0], inner, [1.0]])
    lp = legendre_value(p, xi)
    w = 2.0 / (p * (p + 1) * lp ** 2)
    n = p + 1
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = lp[i] / (lp[j] * (xi[i] - xi[j]))
    D[0, 0] = -p * (p + 1) / 4.0
    D[p, p] = p * (p + 1) / 4.0
    return xi, w, D


def gl(p):
    """Gauss-Legendre nodes and weights (p+1 points) and their derivative matrix."""
    xi, w = npleg.leggauss(p + 1)
    return xi, w, lagrange_derivative(xi)


def lagrange_eval(nodes, x):
    """Matrix L[a, j] = l_j(x_a) of the Lagrange basis on ``nodes`` at points ``x``.

    Written as the plain product formula l_j(x) = prod_{m != j} (x - x_m)/(x_j - x_m).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return L


def lagrange_derivative(nodes, x=None):
    """Matrix G[a, j] = l_j'(x_a) (product rule on the product formula)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    if x is None:
        x = nodes
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    G = np.zeros((len(x), n))
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.ones(len(x)) / (nodes[j] - nodes[k])
            for m in range(n):
                if m != j and m != k:
                    term *= (x - nodes[m]) / (nodes[j] - nodes[m])
            G[:, j] += term
    return G
