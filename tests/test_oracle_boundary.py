"""Pins of the oracle's quadrature Dirichlet data (Sec. 6.3) to what fixes it independently.

* Closed form: for a sum of normalised Gaussians well inside the box, the quadrature
  of int rho(r')/|r - r'| converges spectrally to the full-space potential
  sum_c w_c erf(sqrt(a_c) d)/d.  A wrong weight, a dropped term, a swapped axis or a
  wrong sign in the distance fails this by orders of magnitude.
* Brute force: explicit loops over every boundary node and every grid node, with the
  nodes and weights built here from the GLL rule, on a tiny anisotropic mesh.
* Symmetry: a source even in x gives equal data on the faces x- and x+ and data on the
  y and z faces that is even in X.
"""
import numpy as np

from oracle import boundary, nodes, sipdg
from workloads.gaussians import GaussianDensity

DENS = GaussianDensity([1.0, -0.5], [0.45, 0.6], [[0.7, -0.4, 0.3], [-0.9, 0.5, -0.2]])


def _axes(E, p, lo, hi):
    return sipdg.make_axes(E, p, lo, hi)


def _grid(axes):
    return np.broadcast_arrays(*sipdg.node_grid(axes))


def test_converges_to_the_closed_form_potential():
    axes = _axes((4, 5, 6), 10, [-9.0] * 3, [9.0] * 3)
    X, Y, Z = _grid(axes)
    f = DENS.density(X, Y, Z)
    assert np.abs(f[0]).max() < 1e-15          # the source vanishes on the boundary
    pts = boundary.boundary_points(axes)
    sel = np.concatenate([pts[::41], pts[:1], pts[-1:]])     # includes two corners
    g = boundary.potential_at(axes, f, sel)
    ex = DENS.potential(sel[:, 0], sel[:, 1], sel[:, 2])
    err10 = np.max(np.abs(g - ex)) / np.max(np.abs(ex))
    assert err10 < 2e-8, err10
    axes8 = _axes((4, 5, 6), 8, [-9.0] * 3, [9.0] * 3)
    X8, Y8, Z8 = _grid(axes8)
    g8 = boundary.potential_at(axes8, DENS.density(X8, Y8, Z8), sel)
    err8 = np.max(np.abs(g8 - ex)) / np.max(np.abs(ex))
    assert err8 > 20 * err10                   # spectral: two degrees gain more than an order


def test_matches_brute_force_loops_on_a_tiny_mesh():
    E, p = (2, 1, 3), 2
    lo, hi = [-1.0, 0.0, -2.0], [2.0, 1.5, 1.0]
    axes = _axes(E, p, lo, hi)
    xi, w = nodes.gll(p)[:2]
    coords, wts = [], []
    for d in range(3):
        h = (hi[d] - lo[d]) / E[d]
        coords.append([lo[d] + e * h + 0.5 * h * (xi[i] + 1.0) for e in range(E[d]) for i in range(p + 1)])
        wts.append([0.5 * h * w[i] for e in range(E[d]) for i in range(p + 1)])
    NX, NY, NZ = (len(c) for c in coords)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((NZ, NY, NX))
    hmin = min((hi[d] - lo[d]) / E[d] for d in range(3))

    def g_at(r):
        s = 0.0
        for k in range(NZ):
            for j in range(NY):
                for i in range(NX):
                    dist = np.sqrt((r[0] - coords[0][i]) ** 2 + (r[1] - coords[1][j]) ** 2 + (r[2] - coords[2][k]) ** 2)
                    if dist > 1e-6 * hmin:
                        s += wts[0][i] * wts[1][j] * wts[2][k] * f[k, j, i] / dist
        return s

    pts = []
    for side in (0, -1):                       # x faces [Z][Y]
        pts += [(coords[0][side], coords[1][j], coords[2][k]) for k in range(NZ) for j in range(NY)]
    for side in (0, -1):                       # y faces [Z][X]
        pts += [(coords[0][i], coords[1][side], coords[2][k]) for k in range(NZ) for i in range(NX)]
    for side in (0, -1):                       # z faces [Y][X]
        pts += [(coords[0][i], coords[1][j], coords[2][side]) for j in range(NY) for i in range(NX)]
    ref = np.array([g_at(r) for r in pts])
    got = np.concatenate([a.reshape(-1) for a in boundary.dirichlet_data(axes, f)])
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_even_source_gives_mirrored_faces():
    axes = _axes((3, 2, 2), 4, [-3.0, -2.0, -2.5], [3.0, 2.0, 1.5])
    X, Y, Z = _grid(axes)
    d = GaussianDensity([1.0, 1.0], [0.9, 0.9], [[0.8, 0.3, -0.4], [-0.8, 0.3, -0.4]])
    f = d.density(X, Y, Z)
    f = 0.5 * (f + f[:, :, ::-1])              # exactly even in X on the symmetric GLL grid
    gxm, gxp, gym, gyp, gzm, gzp = boundary.dirichlet_data(axes, f)
    scale = max(np.abs(a).max() for a in (gxm, gym, gzm))
    assert np.max(np.abs(gxm - gxp)) <= 1e-13 * scale
    for a in (gym, gyp, gzm, gzp):
        assert np.max(np.abs(a - a[:, ::-1])) <= 1e-13 * scale
    assert np.max(np.abs(gym - gyp)) > 1e-3 * scale      # y is not a symmetry of the source
