"""Pins of the closed-form input generators (independent of the method)."""
import numpy as np

from workloads import configs, gaussians


def _grid(half, n):
    x = np.linspace(-half, half, n)
    w = np.full(n, x[1] - x[0]); w[0] = w[-1] = 0.5 * w[0]
    return x, w


def test_overlap_matches_quadrature_and_lowdin_orthonormal():
    wl = configs.exchange8()
    prims = wl.orbitals.prims
    S = prims.overlap()
    assert np.allclose(np.diag(S), 1.0)
    C = wl.orbitals.C
    assert np.allclose(C.T @ S @ C, np.eye(C.shape[1]), atol=1e-10)
    # analytic overlap of two primitives against a trapezoid rule
    p2 = gaussians.Primitives([0.7, 1.3], [[0.2, -0.1, 0.0], [-0.4, 0.3, 0.5]])
    x, w = _grid(7.0, 141)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    chi = p2.values(X, Y, Z)
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    assert abs(np.sum(W * chi[0] * chi[1]) - p2.overlap()[0, 1]) < 1e-8


def test_potential_solves_poisson_pointwise():
    # -Lap v = 4 pi rho at a few points, by central differences of the erf form
    dens = gaussians.GaussianDensity([1.0, 0.5], [1.2, 0.4], [[0.1, 0.0, 0.2], [-0.5, 0.3, 0.0]])
    h = 1e-3
    for pt in [(0.3, 0.2, -0.1), (1.5, -0.7, 0.9), (-2.0, 0.5, 0.4)]:
        x, y, z = pt
        lap = 0.0
        for d in range(3):
            e = np.zeros(3); e[d] = h
            lap += (dens.potential(x + e[0], y + e[1], z + e[2]) - 2 * dens.potential(x, y, z)
                    + dens.potential(x - e[0], y - e[1], z - e[2])) / h ** 2
        assert abs(-lap - 4 * np.pi * dens.density(x, y, z)) < 1e-4 * max(1.0, 4 * np.pi * dens.density(x, y, z))
    # value at a centre: 2 sqrt(a/pi) for a unit Gaussian
    g1 = gaussians.GaussianDensity([1.0], [2.0], [[0.0, 0.0, 0.0]])
    assert abs(g1.potential(0.0, 0.0, 0.0) - 2 * np.sqrt(2 / np.pi)) < 1e-12


def test_pair_potential_and_boys_energy_agree():
    # (ij|ij) from the Boys formula equals int rho_ij v_ij with the erf potential
    prims = gaussians.Primitives([0.8, 1.5, 0.5], [[0.3, 0, 0], [-0.4, 0.2, 0.1], [0.0, -0.3, 0.2]])
    C = gaussians.lowdin(np.array([[1.0, 0.3], [0.2, -1.0], [0.5, 0.4]]), prims.overlap())
    orb = gaussians.Orbitals(prims, C)
    x, w = _grid(8.0, 97)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
    phi = orb.values(X, Y, Z).reshape(2, -1)
    V = orb.pair_potentials(X.reshape(-1), Y.reshape(-1), Z.reshape(-1))
    ref = orb.pair_coulomb()
    for k, (i, j) in enumerate(orb.pairs()):
        quad = np.sum(W * phi[i] * phi[j] * V[k])
        assert abs(quad - ref[k]) < 2e-4 * abs(ref[0])
    # density normalisation: the pair density of an orbital with itself has unit charge
    assert abs(np.sum(W * phi[0] ** 2) - 1.0) < 1e-6
    assert abs(np.sum(W * phi[0] * phi[1])) < 1e-6


def test_uneven_split_and_seeding():
    wl = configs.uneven()
    counts = np.bincount(wl.batch.mesh_ids, minlength=3)
    assert list(counts) == [86, 85, 85]
    wl2 = configs.uneven()
    assert np.allclose(wl.batch.densities[17].alpha, wl2.batch.densities[17].alpha)
