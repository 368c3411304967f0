"""Pins of the oracle against closed forms and exact identities.

* The discrete potential of a Gaussian density converges to erf(sqrt(a) r)/r
  at roughly the rate h^(p+1) (a mistake in 4 pi, the mass or the lift would
  stall the convergence at O(1)).
* Discrete pair energies K_ij converge to the continuum (ij|ij) (Boys F0).
* Exchange identities: reciprocity <rho_a, v_b>_M = <rho_b, v_a>_M for
  homogeneous boundary data, linearity and scaling of the solve, the
  ordered-pair sum for E_X, and W_k against a brute-force double loop.
"""
import numpy as np
import pytest

from oracle import exchange, fdm, layout, sipdg
from workloads import configs, gaussians


def _discrete_potential(mesh, dens):
    axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
    X, Y, Z = sipdg.node_grid(axes)
    full = np.ones((axes[2].N, axes[1].N, axes[0].N))
    vex = dens.potential(X, Y, Z) * full
    b = sipdg.rhs(axes, dens.density(X, Y, Z) * full, layout.boundary_faces_of(vex))
    v = fdm.FDM(axes).solve(b)
    M = sipdg.mass(axes)
    return np.sqrt(np.sum(M * (v - vex) ** 2) / np.sum(M * vex ** 2))


def test_single_gaussian_pair_converges_to_erf_potential():
    wl = configs.single()
    dens = wl.batch.densities[0]
    e_4p3 = _discrete_potential(wl.meshes[0], dens)
    e_8p3 = _discrete_potential(configs.Mesh((8, 8, 8), 3, (-5,) * 3, (5,) * 3), dens)
    e_4p5 = _discrete_potential(configs.Mesh((4, 4, 4), 5, (-5,) * 3, (5,) * 3), dens)
    assert 1e-2 < e_4p3 < 4e-2
    assert e_8p3 < e_4p3 / 8          # about h^(p+1)
    assert e_4p5 < e_4p3 / 8          # p-refinement


def _small_orbitals():
    prims = gaussians.Primitives([0.6, 1.4, 0.9, 0.45], [[0.4, 0, 0], [0.4, 0, 0], [-0.5, 0.2, 0.1], [-0.5, 0.2, 0.1]])
    C = gaussians.lowdin(np.array([[1.0, 0.2, -0.3], [0.4, -1.0, 0.2], [0.3, 0.5, 1.0], [-0.2, 0.1, 0.6]]),
                         prims.overlap())
    return gaussians.Orbitals(prims, C)


def _exchange_case(E, p, half, orb):
    axes = sipdg.make_axes((E,) * 3, p, (-half,) * 3, (half,) * 3)
    X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
    phi = list(orb.values(X, Y, Z))
    fx = layout.boundary_faces_of(X); fy = layout.boundary_faces_of(Y); fz = layout.boundary_faces_of(Z)
    faces_pairs = []
    for q in range(len(orb.pairs())):
        faces_pairs.append([None] * 6)
    for f in range(6):
        vals = orb.pair_potentials(fx[f].reshape(-1), fy[f].reshape(-1), fz[f].reshape(-1))
        for q in range(len(vals)):
            faces_pairs[q][f] = vals[q].reshape(fx[f].shape)
    return axes, phi, faces_pairs


def test_pair_energies_converge_to_continuum():
    orb = _small_orbitals()
    ref = orb.pair_coulomb()
    errs = []
    for E in (6, 12):
        axes, phi, fp = _exchange_case(E, 4, 6.0, orb)
        F = fdm.FDM(axes)
        _, _, K, _ = exchange.exchange(axes, phi, fp, F.solve)
        errs.append(np.abs(K - ref).max() / np.abs(ref).max())
    assert errs[0] < 3e-2
    assert errs[1] < errs[0] / 20     # about h^(p+1) with p = 4


def test_exchange_identities():
    orb = _small_orbitals()
    axes, phi, fp = _exchange_case(4, 3, 6.0, orb)
    F = fdm.FDM(axes)
    v, W, K, EX = exchange.exchange(axes, phi, fp, F.solve)
    norb = len(phi)
    # E_X is the sum over ordered pairs
    tot = sum(K[exchange.pair_index(i, j, norb)] for i in range(norb) for j in range(norb))
    assert abs(EX - tot) < 1e-13 * abs(EX)
    # W_k by a brute-force double loop over s
    for k in range(norb):
        Wk = sum(phi[s] * v[exchange.pair_index(s, k, norb)] for s in range(norb))
        assert np.allclose(W[k], Wk, atol=1e-14)
    # reciprocity and linearity with homogeneous Dirichlet data
    M = sipdg.mass(axes)
    zero = [np.zeros_like(f) for f in fp[0]]
    ra, rb = phi[0] * phi[1], phi[2] ** 2
    va = F.solve(sipdg.rhs(axes, ra, zero))
    vb = F.solve(sipdg.rhs(axes, rb, zero))
    assert abs(np.sum(M * ra * vb) - np.sum(M * rb * va)) < 1e-12 * abs(np.sum(M * rb * va))
    vab = F.solve(sipdg.rhs(axes, 2.0 * ra - 0.5 * rb, zero))
    assert np.allclose(vab, 2.0 * va - 0.5 * vb, atol=1e-12 * np.abs(vab).max())
