"""Parity of the quadrature Dirichlet data (Sec. 6.3) against the oracle.

The library computes g_s(r) = sum_q W_q f_s(x_q)/|r - x_q| at every boundary node in
FP64 (dg_boundary_data, and dg_exchange_apply with no Dirichlet data given); the oracle
sums the same terms directly in NumPy.  The two add the ~10^5-10^6 terms in different
orders, so they agree to rounding: 1e-12 of the largest value of each source.
"""
import numpy as np
import pytest

from oracle import boundary, fdm, layout, sipdg
from oracle import exchange as ox
from workloads import configs
from workloads.gaussians import GaussianDensity

from _cases import ENERGY_BAR, PARITY_RTOL, POT_BAR, oracle_axes, oracle_grid, rel_l2_M

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _sources(X, Y, Z, k):
    """Seeded smooth sources: Gaussian sums (positive) and signed products with a cosine."""
    rng = np.random.default_rng(100 + k)
    d = GaussianDensity(rng.uniform(0.5, 1.5, 3), rng.uniform(0.3, 2.0, 3), rng.uniform(-1.5, 1.5, (3, 3)))
    f = d.density(X, Y, Z)
    if k % 2:
        f = f * np.cos(0.7 * X + 0.2 * k) - 0.3 * f
    return f


def _mesh(E, p, lo, hi):
    return configs.Mesh(E, p, lo, hi)


@pytest.mark.parametrize("E,p,nsrc", [((3, 4, 5), 3, 1), ((3, 4, 5), 3, 7), ((2, 3, 2), 4, 52), ((2, 2, 1), 7, 3),
                                       ((8, 8, 8), 1, 5), ((3, 2, 2), 4, 36), ((2, 2, 3), 3, 96), ((2, 3, 2), 4, 2)])
def test_boundary_data_matches_oracle(gpu_lib, E, p, nsrc):
    """Ragged face counts (not a multiple of the 256-node block), one and several source
    tiles (1, 2 and 3 sources unpadded; 52: two tiles of 28; 96: two of the widest, 48), the 36-source tile
    of the exchange workload, a single element along z (every node of it on the z faces) and
    degree 1 (half the nodes of each row on an element face)."""
    lo, hi = [-3.0, -2.5, -4.0], [3.5, 2.0, 3.0]
    mesh = _mesh(E, p, lo, hi)
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=2 if p == 1 else 0)
    xyz, _ = ctx.mesh_coords(0)
    f = np.concatenate([_sources(xyz[0], xyz[1], xyz[2], k) for k in range(nsrc)])
    g = ctx.boundary_data(_t(f)).cpu().numpy().reshape(nsrc, -1)
    axes = oracle_axes(mesh)
    X, Y, Z = oracle_grid(axes)
    fo = np.stack([_sources(X, Y, Z, k) for k in range(nsrc)])
    go = boundary.potential_at(axes, fo, boundary.boundary_points(axes))
    assert g.shape == go.shape
    for k in range(nsrc):
        assert np.max(np.abs(g[k] - go[k])) <= RTOL * np.max(np.abs(go[k])), k


def test_boundary_data_zero_sources_and_errors(gpu_lib):
    import torch
    ctx = gpu_lib.Context([((2, 2, 2), 2, [-1.0] * 3, [1.0] * 3)])
    g = ctx.boundary_data(torch.empty(0, dtype=torch.float64, device="cuda"))
    assert g.numel() == 0
    with pytest.raises(ValueError):
        ctx.boundary_data(torch.zeros(5, dtype=torch.float64, device="cuda"))   # not whole fields


def test_boundary_data_exchange8_all_pairs_sampled(gpu_lib):
    """The 36 pair densities of the 8-orbital workload (16^3 elements, p = 4, 38,400 boundary
    nodes, 512,000 nodes): every pair at a sample of boundary nodes (all eight corners, points
    of every face) against the oracle's direct sum over all nodes."""
    wl = configs.exchange8()
    mesh, orb = wl.meshes[0], wl.orbitals
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels)
    n = orb.norb
    pairs = [(i, j) for i in range(n) for j in range(i, n)]
    xyz, _ = ctx.mesh_coords(0)
    phi = orb.values(xyz[0], xyz[1], xyz[2]).reshape(n, -1)
    rho = np.stack([phi[i] * phi[j] for i, j in pairs])
    g = ctx.boundary_data(_t(rho)).cpu().numpy().reshape(len(pairs), -1)
    axes = oracle_axes(mesh)
    X, Y, Z = oracle_grid(axes)
    po = orb.values(X, Y, Z)
    fo = np.stack([po[i] * po[j] for i, j in pairs])
    pts = boundary.boundary_points(axes)
    NX = axes[0].N
    corners = [0, NX - 1, NX * (NX - 1), NX * NX - 1]            # x- face [Z][Y] corners
    idx = np.unique(np.concatenate([np.arange(0, pts.shape[0], 613), corners, [pts.shape[0] - 1]]))
    go = boundary.potential_at(axes, fo, pts[idx])
    for q in range(len(pairs)):
        assert np.max(np.abs(g[q, idx] - go[q])) <= RTOL * np.max(np.abs(go[q])), pairs[q]


def test_exchange_with_quadrature_data(gpu_lib):
    """dg_exchange_apply with no Dirichlet data computes it by quadrature from the pair
    densities: the same data as dg_boundary_data gives, and at the parity tolerance the pair
    potentials and energies of a sampled pair meet the bars against the oracle's exact solve
    with the oracle's own quadrature data.  Three orbitals of the exchange workload on a
    coarser 6^3-element, p = 4 mesh of the box [-7.5, 7.5]^3 keep the oracle's direct sum
    over every boundary node short."""
    orb = configs.exchange8(norb=3).orbitals
    mesh = configs.cube(6, 4, 7.5)
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=3, rtol=PARITY_RTOL)
    n = orb.norb
    pairs = [(i, j) for i in range(n) for j in range(i, n)]
    xyz, _ = ctx.mesh_coords(0)
    phi = orb.values(xyz[0], xyz[1], xyz[2]).reshape(n, -1)
    phi_t = _t(phi.reshape(-1))
    W, K, EX, st, v = ctx.exchange(phi_t, None, keep_potentials=True)
    assert all(s["status"] == 0 and s["rel_residual"] <= PARITY_RTOL for s in st)
    g = ctx.boundary_data(_t(np.stack([phi[i] * phi[j] for i, j in pairs])))
    W2, K2, _, _, _ = ctx.exchange(phi_t, g)
    assert np.max(np.abs(K.cpu().numpy() - K2.cpu().numpy())) <= 1e-13 * np.max(np.abs(K2.cpu().numpy()))
    v = v.cpu().numpy().reshape(len(pairs), -1)
    K = K.cpu().numpy()
    axes = oracle_axes(mesh)
    X, Y, Z = oracle_grid(axes)
    po = orb.values(X, Y, Z)
    i, j = 0, 2
    fo = np.stack([po[i] * po[i], po[i] * po[j], po[j] * po[j]])
    faces = [layout.split_faces(gq, [a.E for a in axes], axes[0].n)
             for gq in boundary.potential_at(axes, fo, boundary.boundary_points(axes))]
    v_o, _, K_o, _ = ox.exchange(axes, [po[i], po[j]], faces, fdm.FDM(axes).solve)
    for q, vq, Kq in zip([ox.pair_index(a, b, n) for a, b in ((i, i), (i, j), (j, j))], v_o, K_o):
        assert rel_l2_M(axes, mesh, v[q], vq) <= POT_BAR, q
        assert abs(K[q] - Kq) <= ENERGY_BAR, q


def test_solve_batch_with_quadrature_data(gpu_lib):
    """dg_poisson_solve_batch with no Dirichlet data computes it by quadrature for every mesh of
    an interleaved two-mesh batch: the same potentials, bit for bit, as with the data computed
    first by dg_boundary_data, and a sampled potential against the oracle's exact solve with
    the oracle's own quadrature data at the parity tolerance."""
    m0 = configs.Mesh((4, 4, 4), 4, (-4.0,) * 3, (4.0,) * 3)
    m1 = configs.Mesh((3, 4, 5), 3, (-3.0, -3.5, -4.0), (3.0, 3.5, 4.5))
    ctx = gpu_lib.Context([(m.E, m.p, m.lo, m.hi) for m in (m0, m1)], rtol=PARITY_RTOL)
    ids = [0, 1, 1, 0, 1]
    rhos = []
    for k, mid in enumerate(ids):
        xyz, _ = ctx.mesh_coords(mid)
        rhos.append(_sources(xyz[0], xyz[1], xyz[2], k))
    rho = _t(np.concatenate(rhos))
    v, st = ctx.solve_batch(rho, None, mesh_ids=ids)
    assert all(s["status"] == 0 and s["rel_residual"] <= PARITY_RTOL for s in st)
    g = np.concatenate([ctx.boundary_data(_t(rhos[k]), mesh_id=mid).cpu().numpy() for k, mid in enumerate(ids)])
    v2, _ = ctx.solve_batch(rho, _t(g), mesh_ids=ids)
    v, v2 = v.cpu().numpy(), v2.cpu().numpy()
    assert np.array_equal(v, v2)
    axes = oracle_axes(m1)
    X, Y, Z = oracle_grid(axes)
    f = _sources(X, Y, Z, 2)
    faces = layout.split_faces(boundary.potential_at(axes, f, boundary.boundary_points(axes)),
                               [a.E for a in axes], axes[0].n)
    ref = fdm.FDM(axes).solve(sipdg.rhs(axes, f, faces))
    n0, n1 = ctx.info[0]["n_dofs"], ctx.info[1]["n_dofs"]
    off = n0 + n1                       # right-hand side 2: after one field of each mesh
    assert rel_l2_M(axes, m1, v[off:off + n1], ref) <= POT_BAR
