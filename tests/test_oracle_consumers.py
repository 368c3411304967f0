"""Pins of the oracle's consumers of the grid potentials (Hartree and exchange actions projected
on a basis, adaptively compressed exchange) against closed forms and exact identities.

* The quadrature is exact on products of low degree: the projected Hartree action with
  polynomial factors equals the analytic box integral (pins the weights and the index order).
* The projected Hartree action of primitive Gaussians converges to the continuum Coulomb
  integral (ij|cd) (Boys F0), at about h^(p+1).
* The projected exchange action on the occupied orbitals converges to sum_s (is|as), and with
  homogeneous Dirichlet data it is symmetric (reciprocity of the discrete solve).
* The compressed exchange reproduces the exchange action on the occupied span exactly and
  annihilates what is orthogonal to its vectors (rank N_occ).
"""
import numpy as np

from oracle import consumers, exchange, fdm, layout, sipdg
from workloads import gaussians


def _box_axes(E, p, lo, hi):
    return sipdg.make_axes(E, p, lo, hi)


def _grid(axes):
    return np.broadcast_arrays(*sipdg.node_grid(axes))


def test_hartree_action_quadrature_exact_on_low_degree_products():
    lo, hi = (-1.0, 0.5, -2.0), (1.5, 2.0, 1.0)
    axes = _box_axes((2, 3, 2), 3, lo, hi)   # GLL p = 3: exact to degree 5 per variable
    X, Y, Z = _grid(axes)
    # monomials x^a y^b z^c as exponent triples: basis (3), vectors (2), potential (1)
    basis = [(0, 0, 0), (1, 0, 0), (0, 2, 1)]
    vecs = [(0, 1, 0), (2, 0, 1)]
    pot = (1, 0, 1)

    def mono(e):
        return X ** e[0] * Y ** e[1] * Z ** e[2]

    def box_int(e):
        return np.prod([(hi[d] ** (e[d] + 1) - lo[d] ** (e[d] + 1)) / (e[d] + 1) for d in range(3)])

    w = consumers.weights(axes)
    got = consumers.hartree_action(w, [mono(e) for e in basis], [mono(e) for e in vecs], mono(pot))
    assert got.shape == (3, 2)
    for i, eb in enumerate(basis):
        for a, ev in enumerate(vecs):
            tot = tuple(eb[d] + ev[d] + pot[d] for d in range(3))
            assert max(tot) <= 5
            assert abs(got[i, a] - box_int(tot)) <= 1e-12 * max(1.0, abs(box_int(tot))), (i, a)


def _prims():
    return gaussians.Primitives([0.7, 1.3, 0.5], [[0.3, -0.2, 0.1], [-0.4, 0.3, 0.0], [0.1, 0.2, -0.3]])


def test_hartree_action_converges_to_coulomb_integral():
    pr = _prims()
    ia, ib, _, _, _ = pr.product_terms()
    G = pr.coulomb_pair_matrix()
    c, d = 0, 2                      # source density chi_0 chi_2
    src = int(np.nonzero((ia == c) & (ib == d))[0][0])
    errs = []
    for E in (6, 12):
        axes = _box_axes((E,) * 3, 4, (-6.0,) * 3, (6.0,) * 3)
        X, Y, Z = _grid(axes)
        chi = pr.values(X, Y, Z)
        fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
        faces = [pr.pair_potentials(fx[f], fy[f], fz[f])[src].reshape(fx[f].shape) for f in range(6)]
        vH = fdm.FDM(axes).solve(sipdg.rhs(axes, chi[c] * chi[d], faces))
        J = consumers.hartree_action(consumers.weights(axes), chi, chi, vH)
        ref = np.empty((len(pr), len(pr)))
        for t in range(len(ia)):
            ref[ia[t], ib[t]] = ref[ib[t], ia[t]] = G[t, src]
        errs.append(np.abs(J - ref).max() / np.abs(ref).max())
    assert errs[0] < 3e-2
    assert errs[1] < errs[0] / 20


def _orbitals():
    prims = gaussians.Primitives([0.6, 1.4, 0.9, 0.45], [[0.4, 0, 0], [0.4, 0, 0], [-0.5, 0.2, 0.1],
                                                          [-0.5, 0.2, 0.1]])
    C = gaussians.lowdin(np.array([[1.0, 0.2, -0.3], [0.4, -1.0, 0.2], [0.3, 0.5, 1.0], [-0.2, 0.1, 0.6]]),
                         prims.overlap())
    return gaussians.Orbitals(prims, C)


def _pair_faces(axes, orb, homogeneous=False):
    """faces[a][s] for the pair densities psi_a psi_s of the orbital set (closed form or zero)."""
    X, Y, Z = _grid(axes)
    fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
    n = orb.norb
    vals = [orb.pair_potentials(fx[f].reshape(-1), fy[f].reshape(-1), fz[f].reshape(-1)) for f in range(6)]
    out = []
    for a in range(n):
        row = []
        for s in range(n):
            q = exchange.pair_index(a, s, n)
            row.append([np.zeros(fx[f].shape) if homogeneous else vals[f][q].reshape(fx[f].shape)
                        for f in range(6)])
        out.append(row)
    return out


def test_exchange_action_converges_to_two_electron_integrals():
    orb = _orbitals()
    n = orb.norb
    Cp = orb._pair_coeffs()
    G = orb.prims.coulomb_pair_matrix()
    ref = np.array([[sum(Cp[exchange.pair_index(i, s, n)] @ G @ Cp[exchange.pair_index(a, s, n)]
                         for s in range(n)) for a in range(n)] for i in range(n)])
    errs = []
    for E in (6, 12):
        axes = _box_axes((E,) * 3, 4, (-6.0,) * 3, (6.0,) * 3)
        psi = list(orb.values(*_grid(axes)))
        out, _ = consumers.exchange_action(axes, psi, psi, psi, _pair_faces(axes, orb), fdm.FDM(axes).solve)
        errs.append(np.abs(out - ref).max() / np.abs(ref).max())
    assert errs[0] < 5e-2
    assert errs[1] < errs[0] / 20


def test_exchange_action_symmetric_and_energy_with_homogeneous_data():
    orb = _orbitals()
    axes = _box_axes((4, 4, 4), 3, (-6.0,) * 3, (6.0,) * 3)
    psi = list(orb.values(*_grid(axes)))
    F = fdm.FDM(axes)
    faces = _pair_faces(axes, orb, homogeneous=True)
    out, W = consumers.exchange_action(axes, psi, psi, psi, faces, F.solve)
    assert np.abs(out - out.T).max() <= 1e-12 * np.abs(out).max()
    # the trace is the exchange energy over ordered pairs, from the pair-energy oracle
    fp = [faces[i][j] for i, j in exchange.pairs(orb.norb)]
    _, Wx, _, EX = exchange.exchange(axes, psi, fp, F.solve)
    assert abs(np.trace(out) - EX) <= 1e-12 * abs(EX)
    for k in range(orb.norb):
        assert np.allclose(W[k], Wx[k], atol=1e-14 * np.abs(Wx[k]).max())


def test_compressed_exchange_matches_exchange_on_the_occupied_span():
    orb = _orbitals()
    axes = _box_axes((4, 4, 4), 3, (-6.0,) * 3, (6.0,) * 3)
    X, Y, Z = _grid(axes)
    psi = list(orb.values(X, Y, Z))
    w = consumers.weights(axes)
    F = fdm.FDM(axes)
    faces = _pair_faces(axes, orb, homogeneous=True)
    _, W = consumers.exchange_action(axes, psi, psi, psi, faces, F.solve)
    xi, M, L = consumers.ace(w, psi, W)
    assert np.allclose(np.triu(L, 1), 0.0) and np.allclose(L @ L.T, M, rtol=0, atol=1e-13 * np.abs(M).max())
    # arbitrary basis: the primitives and two polynomials
    phi = list(orb.prims.values(X, Y, Z)) + [X * Y, 1.0 + 0.0 * Z]
    exact = consumers.inner(w, phi, W)                 # (phi_i, K psi_a)
    got = consumers.ace_action(w, phi, psi, xi)
    assert np.abs(got - exact).max() <= 1e-11 * np.abs(exact).max()
    # a vector orthogonal to every xi_k is annihilated
    g = X * np.exp(-0.1 * (X ** 2 + Y ** 2 + Z ** 2))
    G = consumers.inner(w, xi, xi)
    c = np.linalg.solve(G, consumers.inner(w, xi, [g])[:, 0])
    g_perp = g - np.tensordot(c, xi, axes=1)
    assert np.abs(consumers.ace_action(w, phi, [g_perp], xi)).max() <= 1e-11 * np.abs(exact).max()
