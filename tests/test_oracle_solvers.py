"""Pins of the exact solve, the multigrid V-cycle and PCG.

* FDM equals a dense LU solve (textbook routine) on small meshes.
* Prolongation reproduces coarse polynomials exactly.
* The V-cycle, formed as an explicit matrix B on a tiny mesh, is symmetric
  positive definite and I - BA is a contraction (eigenvalues of BA in (0, 2)).
* The Lanczos estimate brackets the true largest eigenvalue of D^-1 A.
* PCG converges to the FDM solution.
"""
import numpy as np
import pytest

from oracle import fdm, layout, mg, pcg, sipdg


@pytest.mark.parametrize("E,p", [((3, 2, 4), 2), ((4, 4, 4), 3), ((2, 2, 3), 4)])
def test_fdm_equals_dense_solve(E, p):
    axes = sipdg.make_axes(E, p, (-1.0, -2.0, 0.0), (2.0, 1.0, 3.0))
    b = np.random.default_rng(3).standard_normal((axes[2].N, axes[1].N, axes[0].N))
    x_dense = np.linalg.solve(sipdg.dense_matrix(axes), b.reshape(-1))
    x = fdm.FDM(axes).solve(b).reshape(-1)
    assert np.abs(x - x_dense).max() <= 1e-12 * np.abs(x_dense).max()


def test_hierarchy_specs():
    assert mg.hierarchy((4, 4, 4), 3) == [((4, 4, 4), 3), ((4, 4, 4), 1)]
    assert mg.hierarchy((16,) * 3, 4) == [((16,) * 3, 4), ((16,) * 3, 2), ((16,) * 3, 1), ((8,) * 3, 1)]
    assert len(mg.hierarchy((32,) * 3, 4)) == 5
    assert mg.hierarchy((12,) * 3, 4)[-1] == ((6,) * 3, 1)


@pytest.mark.parametrize("Ef,pf,Ec,pc", [(4, 4, 4, 2), (4, 2, 4, 1), (4, 3, 4, 1), (4, 1, 2, 1), (4, 2, 2, 2)])
def test_prolongation_reproduces_coarse_polynomials(Ef, pf, Ec, pc):
    fine = sipdg.Axis1D(Ef, pf, -1.0, 3.0)
    coarse = sipdg.Axis1D(Ec, pc, -1.0, 3.0)
    P = mg.prolongation_1d(fine, coarse)
    for k in range(pc + 1):
        assert np.allclose(P @ coarse.x ** k, fine.x ** k, atol=1e-12)
    assert np.allclose(P.sum(1), 1.0)


def _explicit(op, n):
    cols = [op(np.eye(n)[:, c]) for c in range(n)]
    return np.array(cols).T


@pytest.mark.parametrize("E,p,nl", [((4, 4, 2), 2, 3), ((4, 2, 2), 3, 2)])
def test_vcycle_is_symmetric_positive_definite_contraction(E, p, nl):
    H = mg.Hierarchy(E, p, (0.0,) * 3, tuple(float(e) for e in E), n_levels=nl)
    L = H.levels[0]
    shape = L.shape
    n = int(np.prod(shape))
    B = _explicit(lambda v: H.vcycle(v.reshape(shape)).reshape(-1), n)
    A = sipdg.dense_matrix(L.axes)
    assert np.abs(B - B.T).max() <= 1e-11 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    ev = np.linalg.eigvals(B @ A).real
    assert ev.min() > 0 and ev.max() < 2.0
    # the cycle is a real contraction, not just SPD
    assert np.abs(1.0 - ev).max() < 0.8


def test_lanczos_brackets_largest_eigenvalue():
    H = mg.Hierarchy((4, 4, 4), 2, (0.0,) * 3, (4.0,) * 3, n_levels=2)
    L = H.levels[0]
    A = sipdg.dense_matrix(L.axes)
    d = L.D.reshape(-1)
    lmax = np.linalg.eigvalsh(A / np.sqrt(d)[:, None] / np.sqrt(d)[None, :]).max()
    lo, hi = H.lam[0]
    ritz = hi / 1.1
    assert ritz <= lmax * (1 + 1e-12) and ritz >= 0.97 * lmax
    assert abs(hi / lo - 60.0) < 1e-12


def test_chebyshev_smoother_is_symmetric():
    H = mg.Hierarchy((4, 2, 2), 2, (0.0,) * 3, (4.0, 2.0, 2.0), n_levels=2)
    shape = H.levels[0].shape
    n = int(np.prod(shape))
    S = _explicit(lambda v: H.chebyshev(0, v.reshape(shape), np.zeros(shape)).reshape(-1), n)
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()


def test_pcg_converges_to_exact_solution():
    E, p = (8, 8, 8), 2
    H = mg.Hierarchy(E, p, (-4.0,) * 3, (4.0,) * 3)
    axes = H.levels[0].axes
    b = np.random.default_rng(5).standard_normal(H.levels[0].shape)
    x_ex = fdm.FDM(axes).solve(b)
    x, it, true_rel, hist = pcg.solve(H, b, rtol=1e-12)
    assert true_rel < 2e-12
    assert np.abs(x - x_ex).max() / np.abs(x_ex).max() < 1e-9
    assert it < 40
    # residual history decreases geometrically on average
    assert hist[-1] < hist[0] * 1e-12
