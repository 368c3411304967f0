"""GPU parity of the consumers of the potentials (Hartree and exchange actions projected on a basis,
adaptively compressed exchange) against the oracle, through the C ABI.

Bars: the quadrature projections to FP64 rounding (1e-12 of the largest entry); the exchange
action, whose potentials come from solves stopped at the parity residual 1e-11, to 1e-8 of the
largest entry (the potential bar); the compressed-exchange vectors, from the same W, to 1e-10;
the compressed operator reproducing the exchange action on the occupied orbitals to 1e-9 (the
solves' residual leaves M = (psi_k, W_l) symmetric only to about that level).
"""
import numpy as np
import pytest

from oracle import boundary, consumers, exchange, fdm, layout, sipdg
from workloads import gaussians

from _cases import PARITY_RTOL, oracle_axes, oracle_grid, to_em

pytestmark = pytest.mark.gpu
DG_ERR_ARG = -1


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


class _Mesh:
    def __init__(self, E, p, lo, hi):
        self.E, self.p, self.lo, self.hi = tuple(E), p, tuple(lo), tuple(hi)


def _em(mesh, arrs):
    """Oracle-order arrays [k][Z, Y, X] -> one element-major stack."""
    return np.concatenate([to_em(np.asarray(a), mesh) for a in arrs])


@pytest.mark.parametrize("E,p,nb,nu", [((4, 6, 3), 4, 11, 5), ((16, 16, 16), 4, 20, 17), ((5, 3, 7), 3, 3, 1)])
def test_hartree_action_matches_oracle(gpu_lib, E, p, nb, nu):
    mesh = _Mesh(E, p, (-2.0, -3.0, -1.5), (2.0, 3.0, 1.5))
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=0)
    axes = oracle_axes(mesh)
    shape = (axes[2].N, axes[1].N, axes[0].N)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((nb,) + shape)
    u = rng.standard_normal((nu,) + shape)
    vH = rng.standard_normal(shape)
    got = ctx.hartree_action(_t(_em(mesh, phi)), _t(_em(mesh, u)), _t(to_em(vH, mesh))).cpu().numpy()
    ref = consumers.hartree_action(consumers.weights(axes), phi, u, vH)
    assert got.shape == ref.shape == (nb, nu)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def _orbitals():
    prims = gaussians.Primitives([0.6, 1.4, 0.9, 0.45], [[0.4, 0, 0], [0.4, 0, 0], [-0.5, 0.2, 0.1],
                                                          [-0.5, 0.2, 0.1]])
    C = gaussians.lowdin(np.array([[1.0, 0.2, -0.3], [0.4, -1.0, 0.2], [0.3, 0.5, 1.0], [-0.2, 0.1, 0.6]]),
                         prims.overlap())
    return gaussians.Orbitals(prims, C)


MESH = _Mesh((6, 5, 4), 4, (-6.0, -5.0, -4.0), (6.0, 5.0, 4.0))
U_IDX = [0, 2]  # the vectors u_a: two of the orbitals (so u_a psi_s is an orbital pair density)


def _closed_form_faces_oracle(axes, orb, homogeneous):
    X, Y, Z = oracle_grid(axes)
    fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
    vals = [orb.pair_potentials(fx[f].reshape(-1), fy[f].reshape(-1), fz[f].reshape(-1)) for f in range(6)]
    n = orb.norb
    return [[[np.zeros(fx[f].shape) if homogeneous else vals[f][exchange.pair_index(a, s, n)].reshape(fx[f].shape)
              for f in range(6)] for s in range(n)] for a in U_IDX]


def _closed_form_faces_gpu(ctx, orb, homogeneous):
    _, fxyz = ctx.mesh_coords(0)
    nface = ctx.info[0]["n_face"]
    n = orb.norb
    if homogeneous:
        return np.zeros(len(U_IDX) * n * nface)
    vals = orb.pair_potentials(fxyz[0], fxyz[1], fxyz[2]).reshape(-1, nface)
    return np.concatenate([vals[exchange.pair_index(a, s, n)] for a in U_IDX for s in range(n)])


def _problem(gpu_lib, homogeneous):
    orb = _orbitals()
    ctx = gpu_lib.Context([(MESH.E, MESH.p, MESH.lo, MESH.hi)], n_levels=0, rtol=PARITY_RTOL, precision="fp64")
    xyz, _ = ctx.mesh_coords(0)
    psi_g = orb.values(xyz[0], xyz[1], xyz[2]).reshape(orb.norb, -1)
    phi_g = np.concatenate([orb.prims.values(xyz[0], xyz[1], xyz[2]).reshape(len(orb.prims), -1),
                            (xyz[0] * xyz[1]).reshape(1, -1)])
    axes = oracle_axes(MESH)
    X, Y, Z = oracle_grid(axes)
    psi_o = list(orb.values(X, Y, Z))
    phi_o = list(orb.prims.values(X, Y, Z)) + [X * Y]
    return orb, ctx, axes, psi_g, phi_g, psi_o, phi_o


@pytest.mark.parametrize("homogeneous", [False, True])
def test_exchange_action_matches_oracle(gpu_lib, homogeneous):
    orb, ctx, axes, psi_g, phi_g, psi_o, phi_o = _problem(gpu_lib, homogeneous)
    g = _closed_form_faces_gpu(ctx, orb, homogeneous)
    out, W, st = ctx.exchange_action(_t(phi_g.reshape(-1)), _t(psi_g[U_IDX].reshape(-1)), _t(psi_g.reshape(-1)),
                                     g_pairs=_t(g), keep_w=True)
    assert len(st) == len(U_IDX) * orb.norb and all(s["status"] == 0 for s in st)
    ref, Wref = consumers.exchange_action(axes, phi_o, [psi_o[a] for a in U_IDX], psi_o,
                                          _closed_form_faces_oracle(axes, orb, homogeneous), fdm.FDM(axes).solve)
    out = out.cpu().numpy()
    assert out.shape == ref.shape
    assert np.abs(out - ref).max() <= 1e-8 * np.abs(ref).max()
    W = W.cpu().numpy().reshape(len(U_IDX), -1)
    for a in range(len(U_IDX)):
        Wr = to_em(Wref[a], MESH)
        assert np.abs(W[a] - Wr).max() <= 1e-8 * np.abs(Wr).max(), a


def test_exchange_action_with_quadrature_data(gpu_lib):
    """No Dirichlet data given: the library computes them by quadrature of u_a psi_s; the oracle
    does the same with its own direct sum (on this 6 x 5 x 4 mesh)."""
    orb, ctx, axes, psi_g, phi_g, psi_o, phi_o = _problem(gpu_lib, False)
    out, _, st = ctx.exchange_action(_t(phi_g.reshape(-1)), _t(psi_g[U_IDX].reshape(-1)), _t(psi_g.reshape(-1)))
    assert all(s["status"] == 0 for s in st)
    faces = [[boundary.dirichlet_data(axes, psi_o[a] * psi_o[s]) for s in range(orb.norb)] for a in U_IDX]
    ref, _ = consumers.exchange_action(axes, phi_o, [psi_o[a] for a in U_IDX], psi_o, faces, fdm.FDM(axes).solve)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-8 * np.abs(ref).max()


def test_compressed_exchange_vectors_and_action(gpu_lib):
    orb, ctx, axes, psi_g, phi_g, psi_o, phi_o = _problem(gpu_lib, True)
    n = orb.norb
    g = np.zeros(n * n * ctx.info[0]["n_face"])
    tpsi = _t(psi_g.reshape(-1))
    tphi = _t(phi_g.reshape(-1))
    exact, W, _ = ctx.exchange_action(tphi, tpsi, tpsi, g_pairs=_t(g), keep_w=True)
    xi = ctx.ace_build(tpsi, W)
    # the vectors against the oracle's construction from the same W
    w = consumers.weights(axes)
    W_o = [layout.to_global(x, MESH.E, MESH.p + 1) for x in W.cpu().numpy().reshape(n, -1)]
    xi_o, _, _ = consumers.ace(w, psi_o, W_o)
    xi_g = xi.cpu().numpy().reshape(n, -1)
    for k in range(n):
        ref = to_em(xi_o[k], MESH)
        assert np.abs(xi_g[k] - ref).max() <= 1e-10 * np.abs(ref).max(), k
    # the compressed operator equals the exchange action on the occupied orbitals
    got = ctx.ace_action(tphi, tpsi, xi).cpu().numpy()
    ex = exact.cpu().numpy()
    assert np.abs(got - ex).max() <= 1e-9 * np.abs(ex).max()
    # and against the oracle's compressed action from its own vectors
    ref = consumers.ace_action(w, phi_o, psi_o, xi_o)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_compressed_exchange_rejects_an_indefinite_overlap(gpu_lib):
    orb, ctx, axes, psi_g, phi_g, psi_o, phi_o = _problem(gpu_lib, True)
    tpsi = _t(psi_g.reshape(-1))
    with pytest.raises(gpu_lib.DgError, match="breakdown"):
        ctx.ace_build(tpsi, _t(-psi_g.reshape(-1)))   # M = -(psi_k, psi_l): negative definite


def test_consumer_arguments_are_checked(gpu_lib):
    ctx = gpu_lib.Context([(MESH.E, MESH.p, MESH.lo, MESH.hi)], n_levels=0)
    nd = ctx.info[0]["n_dofs"]
    lib, h = gpu_lib.lib, ctx._h
    x = _t(np.ones(2 * nd))
    p = gpu_lib._ptr
    assert lib.dg_hartree_action(h, 0, 0, p(x), 1, p(x), p(x), p(x), None) == DG_ERR_ARG
    assert lib.dg_hartree_action(h, 1, 1, p(x), 1, p(x), p(x), p(x), None) == DG_ERR_ARG
    assert lib.dg_hartree_action(h, 0, 1, None, 1, p(x), p(x), p(x), None) == DG_ERR_ARG
    assert lib.dg_ace_build(h, 0, 65, p(x), p(x), p(x), None) == DG_ERR_ARG
    assert lib.dg_exchange_action(h, 0, 1, p(x), 1, p(x), 0, p(x), None, p(x), None, None, None) == \
        DG_ERR_ARG
    assert lib.dg_ace_action(h, 0, 1, p(x), 1, p(x), 0, p(x), p(x), None) == DG_ERR_ARG
