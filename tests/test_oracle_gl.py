"""Pins of the oracle's Gauss-Legendre node family (the nodes Sec. 6.2 names).

* The GL rule integrates polynomials of degree 2p + 1 exactly, so the diagonal GL mass is the
  exact Gram matrix of the Lagrange basis (checked against a rule of much higher order).
* The face traces eL, eR and derivatives dL, dR reproduce polynomials of degree <= p at the
  element ends.
* The Kronecker-sum matrix equals the element-by-element assembly of the bilinear form with GL
  quadrature on elements and faces; it is symmetric positive definite.
* Patch test: a global polynomial of degree <= p per variable is reproduced at the nodes (every
  integral is exact), degree p + 1 is not.
* Closed form: the potential of a Gaussian density converges to erf(sqrt(a) r)/r, and with GL
  nodes (exact quadrature) at least as closely as with GLL collocation.
* The V-cycle-preconditioned CG on the GL hierarchy converges to the exact discrete solution
  (point-Jacobi smoothing sees less of the GL operator than of the GLL one, so it needs more
  iterations).
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import assemble, fdm, mg, nodes, pcg, sipdg
from workloads import configs

MESHES = [((2, 2, 2), 2, (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)),
          ((3, 2, 2), 1, (-1.0, -2.0, -1.5), (1.0, 1.0, 2.0)),
          ((2, 3, 2), 3, (-1.0, -2.0, -1.5), (1.0, 1.0, 2.0)),
          ((1, 2, 2), 4, (0.0, 0.0, 0.0), (1.0, 2.0, 2.0))]


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_gl_rule_exact_to_degree_2p_plus_1_and_mass_is_the_gram_matrix(p):
    xi, w, _ = nodes.gl(p)
    for k in range(2 * p + 2):
        assert abs(np.sum(w * xi ** k) - (1 - (-1) ** (k + 1)) / (k + 1)) < 1e-13
    # degree 2p + 2 is not integrated exactly (the rule has teeth)
    k = 2 * p + 2
    assert abs(np.sum(w * xi ** k) - 2.0 / (k + 1)) > 1e-6
    xq, wq = npleg.leggauss(3 * p + 5)
    L = nodes.lagrange_eval(xi, xq)
    G = L.T @ (wq[:, None] * L)
    assert np.abs(G - np.diag(w)).max() < 1e-13


@pytest.mark.parametrize("p", [1, 2, 4, 5])
def test_traces_reproduce_polynomials_at_the_element_ends(p):
    ax = sipdg.Axis1D(3, p, -1.5, 3.0, family="gl")
    J = ax.h / 2.0
    c = np.random.default_rng(p).standard_normal(p + 1)
    P = np.polynomial.polynomial.Polynomial(c)
    for e in range(ax.E):
        x0, x1 = ax.a + e * ax.h, ax.a + (e + 1) * ax.h
        u = P(ax.x[e * ax.n:(e + 1) * ax.n])
        assert abs(ax.eL @ u - P(x0)) < 1e-12 * (1 + abs(P(x0)))
        assert abs(ax.eR @ u - P(x1)) < 1e-12 * (1 + abs(P(x1)))
        assert abs(ax.dL @ u - P.deriv()(x0)) < 1e-10 * (1 + abs(P.deriv()(x0)))
        assert abs(ax.dR @ u - P.deriv()(x1)) < 1e-10 * (1 + abs(P.deriv()(x1)))
    assert J > 0 and np.all(np.abs(ax.xi) < 1.0)     # no GL node on a face


def _f(x, y, z):
    return np.exp(-x * x - 0.5 * y * y) * np.cos(z)


def _g(x, y, z):
    return x * x + y - z * y + 0.3


@pytest.mark.parametrize("E,p,lo,hi", MESHES)
def test_kronecker_sum_equals_elementwise_assembly_gl(E, p, lo, hi):
    axes = sipdg.make_axes(E, p, lo, hi, family="gl")
    A1 = sipdg.dense_matrix(axes)
    A2, b2 = assemble.assemble(E, p, lo, hi, _f, _g, family="gl")
    assert np.abs(A1 - A2).max() <= 1e-12 * np.abs(A1).max()
    assert np.abs(A1 - A1.T).max() <= 1e-13 * np.abs(A1).max()
    assert np.linalg.eigvalsh(A1).min() > 0
    X, Y, Z = sipdg.node_grid(axes)
    full = np.ones((axes[2].N, axes[1].N, axes[0].N))
    faces = [_g(*fp) for fp in sipdg.face_points(axes)]
    b1 = sipdg.rhs(axes, _f(X, Y, Z) * full, faces)
    assert np.abs(b1.reshape(-1) - b2).max() <= 1e-12 * np.abs(b2).max()
    u = np.random.default_rng(0).standard_normal(full.shape)
    assert np.allclose(sipdg.apply(axes, u).reshape(-1), A1 @ u.reshape(-1), rtol=0, atol=1e-12 * np.abs(A1).max())


def test_gl_and_gll_differ():
    """The two families give different matrices (the family switch is not a no-op)."""
    E, p, lo, hi = MESHES[0]
    A_gl = sipdg.dense_matrix(sipdg.make_axes(E, p, lo, hi, family="gl"))
    A_gll = sipdg.dense_matrix(sipdg.make_axes(E, p, lo, hi))
    assert np.abs(A_gl - A_gll).max() > 1e-3 * np.abs(A_gll).max()


def test_face_points_of_gll_are_the_boundary_nodes():
    from oracle import layout
    axes = sipdg.make_axes((2, 3, 2), 3, (-1.0, -2.0, -1.5), (1.0, 1.0, 2.0))
    X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
    fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
    for f, fp in enumerate(sipdg.face_points(axes)):
        assert np.array_equal(fp[0], fx[f]) and np.array_equal(fp[1], fy[f]) and np.array_equal(fp[2], fz[f])


def _poly_case(p):
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


def _patch_error_gl(E, p, lo, hi, q):
    axes = sipdg.make_axes(E, p, lo, hi, family="gl")
    u, lap = _poly_case(q)
    X, Y, Z = sipdg.node_grid(axes)
    full = np.ones((axes[2].N, axes[1].N, axes[0].N))
    uex = u(X, Y, Z) * full
    faces = [u(*fp) for fp in sipdg.face_points(axes)]
    b = sipdg.rhs(axes, -lap(X, Y, Z) * full / (4 * np.pi), faces)
    v = np.linalg.solve(sipdg.dense_matrix(axes), b.reshape(-1)).reshape(full.shape)
    return np.abs(v - uex).max() / np.abs(uex).max()


@pytest.mark.parametrize("E,p,lo,hi", MESHES)
def test_patch_test_gl(E, p, lo, hi):
    assert _patch_error_gl(E, p, lo, hi, p) < 1e-11


def test_patch_test_gl_fails_beyond_degree_p():
    E, p, lo, hi = MESHES[0]
    assert _patch_error_gl(E, p, lo, hi, p + 1) > 1e-6


def _gaussian_error(mesh, dens, family):
    axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi, family=family)
    X, Y, Z = sipdg.node_grid(axes)
    full = np.ones((axes[2].N, axes[1].N, axes[0].N))
    vex = dens.potential(X, Y, Z) * full
    faces = [dens.potential(*fp) for fp in sipdg.face_points(axes)]
    b = sipdg.rhs(axes, dens.density(X, Y, Z) * full, faces)
    v = fdm.FDM(axes).solve(b)
    M = sipdg.mass(axes)
    return np.sqrt(np.sum(M * (v - vex) ** 2) / np.sum(M * vex ** 2))


def test_gaussian_potential_converges_with_gl_nodes():
    wl = configs.single()
    dens = wl.batch.densities[0]
    e4 = _gaussian_error(wl.meshes[0], dens, "gl")
    e8 = _gaussian_error(configs.Mesh((8, 8, 8), 3, (-5,) * 3, (5,) * 3), dens, "gl")
    g4 = _gaussian_error(wl.meshes[0], dens, "gll")
    assert e4 < 5e-2
    assert e8 < e4 / 8                    # about h^(p+1)
    assert e4 <= g4                       # the exact GL rule is at least as accurate as GLL collocation


def test_vcycle_pcg_on_the_gl_hierarchy_reaches_the_exact_solution():
    E, p, lo, hi = (4, 4, 4), 4, (-3.0,) * 3, (3.0,) * 3
    H = mg.Hierarchy(E, p, lo, hi, family="gl")
    assert [L.p for L in H.levels][:3] == [4, 2, 1]
    axes = H.levels[0].axes
    X, Y, Z = sipdg.node_grid(axes)
    full = np.ones((axes[2].N, axes[1].N, axes[0].N))
    f = np.exp(-(X ** 2 + 0.5 * Y ** 2 + (Z - 0.3) ** 2)) * full
    faces = [0.1 / np.sqrt(fp[0] ** 2 + fp[1] ** 2 + fp[2] ** 2) for fp in sipdg.face_points(axes)]
    b = sipdg.rhs(axes, f, faces)
    ex = fdm.FDM(axes).solve(b)
    x, its = pcg.pcg(H.levels[0].A, b, H.vcycle, rtol=1e-11)[:2]
    # point Jacobi sees less of the GL operator (the face couplings are spread over every node
    # of a line: lambda_max(D^-1 A) 6.8 against 2.3 for GLL), so the same smoother needs more
    # iterations (34 against 13 for GLL on this problem)
    assert its <= 40
    assert np.abs(x - ex).max() <= 1e-9 * np.abs(ex).max()
    Hg = mg.Hierarchy(E, p, lo, hi)
    assert H.lam[0][1] > 2.0 * Hg.lam[0][1]
