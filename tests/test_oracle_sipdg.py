"""Pins of the SIPDG operator and right-hand side.

* Two independent constructions agree: the Kronecker sum of 1D matrices and
  the element-by-element assembly of the 3D bilinear form (eq. sip_bilinear).
* The matrix is symmetric positive definite (dense eigensolver).
* Patch test: for a global polynomial u of degree <= p in each variable,
  rho = -Lap u / (4 pi) and g = u, the discrete solution is u at the nodes,
  because GLL quadrature is exact for every integral that appears.
* Planted mistakes in the oracle (wrong lift sign, dropped consistency term,
  transposed 1D block) are caught by these pins.
"""
import numpy as np
import pytest

from oracle import assemble, fdm, layout, sipdg

MESHES = [((2, 2, 2), 2, (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)),
          ((3, 2, 2), 1, (-1.0, -2.0, -1.5), (1.0, 1.0, 2.0)),
          ((2, 3, 2), 3, (-1.0, -2.0, -1.5), (1.0, 1.0, 2.0)),
          ((1, 2, 2), 4, (0.0, 0.0, 0.0), (1.0, 2.0, 2.0))]


def _f(x, y, z):
    return np.exp(-x * x - 0.5 * y * y) * np.cos(z)


def _g(x, y, z):
    return x * x + y - z * y + 0.3


@pytest.mark.parametrize("E,p,lo,hi", MESHES)
def test_kronecker_sum_equals_elementwise_assembly(E, p, lo, hi):
    axes = sipdg.make_axes(E, p, lo, hi)
    A1 = sipdg.dense_matrix(axes)
    A2, b2 = assemble.assemble(E, p, lo, hi, _f, _g)
    assert np.abs(A1 - A2).max() <= 1e-13 * np.abs(A1).max()
    X, Y, Z = sipdg.node_grid(axes)
    full = np.ones((axes[2].N, axes[1].N, axes[0].N))
    b1 = sipdg.rhs(axes, _f(X, Y, Z) * full, layout.boundary_faces_of(_g(X, Y, Z) * full))
    assert np.abs(b1.reshape(-1) - b2).max() <= 1e-13 * np.abs(b2).max()
    # matrix-free apply equals the dense matrix
    u = np.random.default_rng(0).standard_normal(full.shape)
    assert np.allclose(sipdg.apply(axes, u).reshape(-1), A1 @ u.reshape(-1), rtol=0, atol=1e-12 * np.abs(A1).max())


@pytest.mark.parametrize("E,p,lo,hi", MESHES)
def test_symmetric_positive_definite(E, p, lo, hi):
    A = sipdg.dense_matrix(sipdg.make_axes(E, p, lo, hi))
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


def _poly_case(p):
    """u = product of degree-p polynomials, and -Lap u."""
    cx = np.array([0.3, -1.0, 0.5, 0.25, -0.1, 0.05, 0.02][:p + 1])
    cy = np.array([1.0, 0.2, -0.7, 0.1, 0.3, -0.02, 0.01][:p + 1])
    cz = np.array([-0.5, 0.4, 0.3, -0.2, 0.1, 0.04, -0.03][:p + 1])
    P = np.polynomial.polynomial
    px, py, pz = (P.Polynomial(c) for c in (cx, cy, cz))

    def u(x, y, z):
        return px(x) * py(y) * pz(z)

    def lap(x, y, z):
        return (px.deriv(2)(x) * py(y) * pz(z) + px(x) * py.deriv(2)(y) * pz(z)
                + px(x) * py(y) * pz.deriv(2)(z))
    return u, lap


def _patch_error(axes, p):
    u, lap = _poly_case(p)
    X, Y, Z = sipdg.node_grid(axes)
    full = np.ones((axes[2].N, axes[1].N, axes[0].N))
    uex = u(X, Y, Z) * full
    b = sipdg.rhs(axes, -lap(X, Y, Z) * full / (4 * np.pi), layout.boundary_faces_of(uex))
    v = np.linalg.solve(sipdg.dense_matrix(axes), b.reshape(-1)).reshape(full.shape)
    return np.abs(v - uex).max() / np.abs(uex).max()


@pytest.mark.parametrize("E,p,lo,hi", MESHES)
def test_patch_test_recovers_polynomials(E, p, lo, hi):
    axes = sipdg.make_axes(E, p, lo, hi)
    assert _patch_error(axes, p) < 1e-11


def test_patch_test_fails_beyond_degree_p():
    # degree p+1 is not reproduced: the test has teeth
    E, p, lo, hi = MESHES[0]
    axes = sipdg.make_axes(E, p, lo, hi)
    assert _patch_error(axes, p + 1) > 1e-6


def test_axis_permutation_equivariance():
    axes = sipdg.make_axes((3, 3, 3), 2, (-1.0,) * 3, (2.0,) * 3)
    u = np.random.default_rng(1).standard_normal((9, 9, 9))
    y = sipdg.apply(axes, u)
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1)]:
        assert np.allclose(sipdg.apply(axes, u.transpose(perm)), y.transpose(perm), atol=1e-12)


def test_penalty_value_and_coercivity_margin():
    # sigma = (p+1)^2/(eps h) with eps = 1/8
    assert sipdg.penalty(4, 1.0) == 200.0
    assert abs(sipdg.penalty(3, 2.5) - 51.2) < 1e-12
    # with a penalty far below the coercivity threshold the matrix is indefinite
    axes = sipdg.make_axes((3, 1, 1), 4, (0, 0, 0), (3, 1, 1), eps=40.0)
    assert np.linalg.eigvalsh(axes[0].A).min() < 0


# ---- planted mistakes: each must break one of the pins above ---------------

def _mutated_axis(kind, E=3, p=3, a=-1.0, b=2.0):
    ax = sipdg.Axis1D(E, p, a, b)
    n = p + 1
    if kind == "lift_sign":
        ax.liftL = ax.sigma * np.eye(E * n)[0] - ax.dL[0] * 0 - np.pad(ax.dL, (0, (E - 1) * n))
    elif kind == "drop_consistency":
        # remove the -{u'}[[v]] - [[u]]{v'} terms at the first interior face
        jmp = np.zeros(E * n); jmp[n - 1] = 1; jmp[n] = -1
        avg = np.zeros(E * n); avg[:n] = 0.5 * ax.dR; avg[n:2 * n] = 0.5 * ax.dL
        ax.A = ax.A + np.outer(jmp, avg) + np.outer(avg, jmp)
    elif kind == "transpose_block":
        blk = ax.A[0:n, n:2 * n].copy()
        ax.A[0:n, n:2 * n] = blk.T
    return ax


@pytest.mark.parametrize("kind", ["lift_sign", "drop_consistency", "transpose_block"])
def test_planted_mistakes_are_caught(kind):
    p = 3
    good = sipdg.make_axes((3, 2, 2), p, (-1.0, -1.0, -1.0), (2.0, 1.0, 1.0))
    bad = [_mutated_axis(kind, 3, p, -1.0, 2.0), good[1], good[2]]
    caught = _patch_error(bad, p) > 1e-8
    A_bad = sipdg.dense_matrix(bad)
    A_ref, _ = assemble.assemble((3, 2, 2), p, (-1.0, -1.0, -1.0), (2.0, 1.0, 1.0))
    caught = caught or np.abs(A_bad - A_ref).max() > 1e-10
    assert caught
