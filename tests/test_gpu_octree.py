"""GPU parity of the adaptive octree path (dg_octree_*) against the octree oracle, through the
C ABI: the refined mesh (element list, nodes, Dirichlet points) exactly; the operator on every
multigrid level, the right-hand side, the smoother bounds, one V-cycle and full MG-PCG solves
at FP64 rounding bars; the polynomial reproduction of the hanging-face discretisation at a size
the dense oracle cannot solve.

Bars: operator, right-hand side and transfers 1e-12 of the largest entry (FP64 rounding of a
few hundred terms); Lanczos bounds 1e-9 relative (30 Lanczos steps amplify rounding); one
V-cycle 1e-9 (smoothing polynomials of degree 6 and 10 in lam_hi); solves at rtol 1e-12 to
1e-9 of the largest entry and the oracle's iteration count within one.
"""
import numpy as np
import pytest

from oracle import octree, pcg

pytestmark = pytest.mark.gpu


def _gauss(a, c):
    return lambda x, y, z: np.exp(-a * ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2))


def _two_centres(x, y, z):
    return _gauss(12.0, (0.5, 0.2, -0.3))(x, y, z) + 0.5 * _gauss(30.0, (-0.6, -0.4, 0.5))(x, y, z)


_CENTRES = [(0.5, 0.2, -0.3, 12.0), (-0.6, -0.4, 0.5, 30.0), (1.1, -0.9, 0.4, 50.0), (-1.2, 1.0, -0.8, 20.0)]


def _molecule(x, y, z):
    """Four atom-like Gaussians of different widths (the kind of density Sec. 6.2 refines on)."""
    return sum(np.exp(-a * ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)) for cx, cy, cz, a in _CENTRES)


# 6^3 base cells on [-4, 4]^3, degree 4, delta_q 1e-10, three refinements: 1,630 elements, 203,750 nodes
LARGE = ((6, 6, 6), (-4.0, -4.0, -4.0), (4.0, 4.0, 4.0), 4, 1e-10, 3)


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


# (ne, lo, hi, q, delta_q, max_depth): isotropic and anisotropic (4:1:1-like) base cells
CASES = [
    ((2, 2, 2), (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0), 4, 1e-4, 2),
    ((3, 2, 1), (-2.0, -1.5, -0.8), (2.0, 1.5, 0.8), 2, 1e-5, 3),
    ((1, 2, 2), (-3.0, -1.5, -1.5), (3.0, 1.5, 1.5), 3, 1e-5, 3),
    ((2, 2, 2), (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0), 1, 1e-5, 3),
]


def _pair(gpu_lib, case, **opts):
    ne, lo, hi, q, dq, depth = case
    g = gpu_lib.Octree(ne, lo, hi, q=q, rho=_two_centres, delta_q=dq, max_depth=depth, **opts)
    t = octree.Octree(ne, lo, hi, q, rho=_two_centres, delta_q=dq, max_depth=depth)
    return g, t


@pytest.mark.parametrize("case", CASES)
def test_refined_mesh_matches_oracle(gpu_lib, case):
    g, t = _pair(gpu_lib, case)
    cells = t.cells()
    assert g.n_elements == len(cells) and g.max_generation == t.max_gen and t.max_gen >= 1
    lohi, gen = g.elements()
    ref = np.array([np.concatenate(t.bounds(c)) for c in cells])
    assert np.array_equal(gen, [c.gen for c in cells])
    assert np.abs(lohi - ref).max() <= 1e-14 * np.abs(ref).max()
    m = t.mesh()
    xyz = g.nodes()
    assert np.abs(xyz - np.array(m.nodes())).max() <= 1e-14 * 4
    bxyz = g.boundary_points()
    assert np.abs(bxyz - np.array(m.boundary_points())).max() <= 1e-14 * 4
    print(f"case {case}: {g.n_elements} elements, {g.n_dofs} nodes, generations {t.max_gen}, {g.n_levels} levels")


@pytest.mark.parametrize("case", CASES)
def test_operator_rhs_bounds_and_vcycle_match_oracle(gpu_lib, case):
    g, t = _pair(gpu_lib, case)
    H = octree.Hierarchy(t)
    assert g.n_levels == len(H.meshes)
    rng = np.random.default_rng(11)
    for l, m in enumerate(H.meshes):
        li = g.level_info(l)
        assert li["n_elements"] == len(m.cells) and li["q"] == m.q
        u = rng.standard_normal((2, m.ndof))
        got = g.apply(_t(u), level=l).cpu().numpy()
        ref = np.stack([m.apply(u[k]) for k in range(2)])
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), l
        if l + 1 < len(H.meshes):
            lo, hi = H.lam[l]
            assert abs(li["lam_hi"] - hi) <= 1e-9 * hi and abs(li["lam_lo"] - lo) <= 1e-9 * lo, l
    m = H.meshes[0]
    X, Y, Z = m.nodes()
    f = np.stack([_two_centres(X, Y, Z), np.cos(X) * Y])
    bx, by, bz = m.boundary_points()
    gb = np.stack([0.2 * np.sin(bx) + by * bz, np.zeros_like(bx)])
    b = g.rhs(_t(f), _t(gb)).cpu().numpy()
    bref = np.stack([m.rhs(f[k], gb[k]) for k in range(2)])
    assert np.abs(b - bref).max() <= 1e-12 * np.abs(bref).max()
    z = g.vcycle(_t(bref)).cpu().numpy()
    zref = np.stack([H.vcycle(bref[k]) for k in range(2)])
    assert np.abs(z - zref).max() <= 1e-9 * np.abs(zref).max()


@pytest.mark.parametrize("case,cheb", [(CASES[0], (6, 10)), (CASES[1], (6, 10)), (CASES[2], (6, 10)),
                                       (CASES[0], (8, 4)), (CASES[1], (8, 4))])
def test_solve_matches_oracle_pcg(gpu_lib, case, cheb):
    """Full solves; (8, 4) Chebyshev steps (degree >= 2 levels, degree-1 levels) is the octree
    benchmark's setting, (6, 10) the library default."""
    g, t = _pair(gpu_lib, case, rtol=1e-12, cheb_degree=cheb[0], cheb_degree_h=cheb[1])
    H = octree.Hierarchy(t, degree=cheb[0], degree_h=cheb[1])
    m = H.meshes[0]
    X, Y, Z = m.nodes()
    bx, by, bz = m.boundary_points()
    f = np.stack([_two_centres(X, Y, Z), _gauss(3.0, (0.1, 0.0, 0.2))(X, Y, Z)])
    gb = np.stack([np.zeros_like(bx), 0.05 * np.cos(bx + by)])
    b = np.stack([m.rhs(f[k], gb[k]) for k in range(2)])
    x, st = g.solve(_t(b))
    x = x.cpu().numpy()
    for k in range(2):
        xr, it, rel, _ = pcg.pcg(H.levels[0].A, b[k], H.vcycle, rtol=1e-12)
        assert st[k]["status"] == 0 and st[k]["rel_residual"] <= 2e-12
        assert abs(st[k]["iters"] - it) <= 1, (st[k]["iters"], it)
        assert np.abs(x[k] - xr).max() <= 1e-9 * np.abs(xr).max()


def _poly(x, y, z):
    u = 1.0 + x * x * y - 0.5 * z ** 3 + x * y * z + 0.3 * y ** 3 - x
    return u, -(2.0 * y - 3.0 * z + 1.8 * y) / (4.0 * np.pi)


def test_hanging_faces_reproduce_a_polynomial_at_size(gpu_lib):
    """Consistency of SIPDG on the hanging-face mesh, checked where no dense oracle reaches: a
    cubic that solves the PDE is the discrete solution (degree 4, several thousand elements)."""
    ne, lo, hi, q, dq, depth = LARGE
    g = gpu_lib.Octree(ne, lo, hi, q=q, rho=_molecule, delta_q=dq, max_depth=depth, rtol=1e-13, max_iter=400)
    assert g.max_generation == 3 and g.n_elements == 1630
    xyz = g.nodes()
    u, f = _poly(*xyz)
    gu, _ = _poly(*g.boundary_points())
    b = g.rhs(_t(f[None]), _t(gu[None]))
    x, st = g.solve(b)
    print(f"{g.n_elements} elements, {g.n_dofs} nodes: {st[0]['iters']} iterations")
    assert st[0]["status"] == 0
    assert np.abs(x.cpu().numpy()[0] - u).max() <= 1e-8 * np.abs(u).max()


def test_residual_of_a_large_solve_against_the_oracle_operator(gpu_lib):
    """Full size: the oracle's matrix-free operator recomputes b - A x of the GPU solution."""
    ne, lo, hi, q, dq, depth = LARGE
    g = gpu_lib.Octree(ne, lo, hi, q=q, rho=_molecule, delta_q=dq, max_depth=depth, rtol=1e-10)
    t = octree.Octree(ne, lo, hi, q, rho=_molecule, delta_q=dq, max_depth=depth)
    m = t.mesh()
    assert g.n_elements == len(m.cells)
    X, Y, Z = m.nodes()
    f = _molecule(X, Y, Z)
    bx, by, bz = m.boundary_points()
    b = m.rhs(f, np.zeros_like(bx))
    x, st = g.solve(_t(b[None]))
    x = x.cpu().numpy()[0]
    rel = np.linalg.norm(b - m.apply(x)) / np.linalg.norm(b)
    assert st[0]["status"] == 0 and rel <= 2e-10 and abs(rel - st[0]["rel_residual"]) <= 1e-12


@pytest.mark.parametrize("case", CASES[:3])
def test_boundary_data_by_quadrature_matches_oracle(gpu_lib, case):
    """Sec. 6.3's Dirichlet data on the octree grid, and the right-hand side built from them."""
    g, t = _pair(gpu_lib, case)
    m = t.mesh()
    X, Y, Z = m.nodes()
    f = np.stack([_two_centres(X, Y, Z), np.cos(X) * _gauss(2.0, (0.0, 0.1, 0.0))(X, Y, Z),
                  _gauss(6.0, (-0.3, 0.2, 0.1))(X, Y, Z)])
    got = g.boundary_data(_t(f)).cpu().numpy()
    ref = m.boundary_data(f)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    b = g.rhs(_t(f)).cpu().numpy()              # no data given: by quadrature
    bref = np.stack([m.rhs(f[k], ref[k]) for k in range(3)])
    assert np.abs(b - bref).max() <= 1e-12 * np.abs(bref).max()


@pytest.mark.parametrize("case", CASES)
def test_fp32_operator_matches_oracle(gpu_lib, case):
    """The FP32 V-cycle's operator at every level, to FP32 rounding of the oracle's FP64 result."""
    import torch
    g, t = _pair(gpu_lib, case, precision="fp32_pc")
    H = octree.Hierarchy(t)
    rng = np.random.default_rng(12)
    for l, m in enumerate(H.meshes):
        u = rng.standard_normal((2, m.ndof))
        got = g.apply_f32(torch.as_tensor(u, dtype=torch.float32).cuda().contiguous(), level=l).cpu().numpy()
        ref = np.stack([m.apply(u[k].astype(np.float32).astype(np.float64)) for k in range(2)])
        assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max(), l


@pytest.mark.parametrize("case,cheb", [(CASES[0], (6, 10)), (CASES[2], (8, 4)), (LARGE, (8, 4))])
def test_fp32_pc_solve_matches_the_fp64_solution(gpu_lib, case, cheb):
    """FP32 V-cycle under FP64 CG: the FP64 residual reaches the tolerance, and the solution agrees
    with the oracle's FP64 MG-PCG (or, at the large size, with the library's FP64 solve)."""
    ne, lo, hi, q, dq, depth = case
    rho = _molecule if case is LARGE else _two_centres
    kw = dict(rho=rho, delta_q=dq, max_depth=depth, rtol=1e-11, cheb_degree=cheb[0], cheb_degree_h=cheb[1])
    g32 = gpu_lib.Octree(ne, lo, hi, q=q, precision="fp32_pc", **kw)
    g64 = gpu_lib.Octree(ne, lo, hi, q=q, **kw)
    xyz = g32.nodes()
    bxyz = g32.boundary_points()
    f = np.stack([rho(*xyz), _gauss(3.0, (0.1, 0.0, 0.2))(*xyz)])
    gb = np.stack([np.zeros(bxyz.shape[1]), 0.05 * np.cos(bxyz[0] + bxyz[1])])
    b = g32.rhs(_t(f), _t(gb))
    x32, st32 = g32.solve(b)
    x64, st64 = g64.solve(b)
    x32, x64 = x32.cpu().numpy(), x64.cpu().numpy()
    for k in range(2):
        assert st32[k]["status"] == 0 and st32[k]["rel_residual"] <= 2e-11
        assert st32[k]["iters"] <= st64[k]["iters"] + 3, (st32[k]["iters"], st64[k]["iters"])
        assert np.abs(x32[k] - x64[k]).max() <= 1e-8 * np.abs(x64[k]).max()
    if case is not LARGE:
        t = octree.Octree(ne, lo, hi, q, rho=rho, delta_q=dq, max_depth=depth)
        H = octree.Hierarchy(t, degree=cheb[0], degree_h=cheb[1])
        bh = b.cpu().numpy()
        for k in range(2):
            xr, _, _, _ = pcg.pcg(H.levels[0].A, bh[k], H.vcycle, rtol=1e-12)
            assert np.abs(x32[k] - xr).max() <= 1e-8 * np.abs(xr).max()


@pytest.mark.parametrize("case,quadrature", [(CASES[0], False), (CASES[1], True)])
def test_exchange_matches_oracle(gpu_lib, case, quadrature):
    """W_k, K_ij and E_x on the octree grid (Dirichlet data closed-form or by quadrature) against
    the oracle's exchange with its own MG-PCG solves at the same tolerance."""
    from workloads import gaussians
    prims = gaussians.Primitives([0.9, 1.6, 0.7, 2.5], [[0.3, 0.1, 0.0], [-0.4, 0.0, 0.2], [0.1, -0.3, -0.1],
                                                        [0.5, 0.2, -0.2]])
    orb = gaussians.Orbitals(prims, gaussians.lowdin(np.array([[1.0, 0.3, 0.1], [0.2, -1.0, 0.4], [0.5, 0.4, -0.6],
                                                               [0.1, 0.2, 1.0]]), prims.overlap()))
    g, t = _pair(gpu_lib, case, rtol=1e-12)
    H = octree.Hierarchy(t)
    m = H.meshes[0]
    psi = list(orb.values(*m.nodes()))
    gp = None if quadrature else orb.pair_potentials(*m.boundary_points())
    W, K, EX, st, v = g.exchange(_t(np.stack(psi)), None if gp is None else _t(gp), keep_potentials=True)
    assert all(x["status"] == 0 for x in st)
    pairs = [(i, j) for i in range(3) for j in range(i, 3)]
    gref = [m.boundary_data(psi[i] * psi[j]) for i, j in pairs] if quadrature else list(gp)
    vr, Wr, Kr, EXr = octree.exchange(m, psi, gref, lambda b: pcg.pcg(H.levels[0].A, b, H.vcycle, rtol=1e-12)[0])
    assert np.abs(K - Kr).max() <= 1e-9 * np.abs(Kr).max()
    assert abs(EX - EXr) <= 1e-9 * abs(EXr)
    W = W.cpu().numpy()
    for k in range(3):
        assert np.abs(W[k] - Wr[k]).max() <= 1e-8 * np.abs(Wr[k]).max()
    v = v.cpu().numpy()
    for k in range(len(pairs)):
        assert np.abs(v[k] - vr[k]).max() <= 1e-8 * np.abs(vr[k]).max()


@pytest.mark.parametrize("q,rho", [(1, None), (2, None), (1, "refined")])
def test_degenerate_hierarchies(gpu_lib, q, rho):
    """A single level (q = 1, no refinement: the V-cycle is the exact base-mesh solve, so PCG ends
    in one iteration), degree steps only (no refinement), and refinement at q = 1 (mesh steps
    only): solves against the oracle's dense solution."""
    ne, lo, hi = (3, 2, 2), (-1.5, -1.0, -1.0), (1.5, 1.0, 1.0)
    dens = _two_centres if rho else None
    g = gpu_lib.Octree(ne, lo, hi, q=q, rho=dens, delta_q=1e-4, max_depth=2, rtol=1e-12)
    t = octree.Octree(ne, lo, hi, q, rho=dens, delta_q=1e-4, max_depth=2)
    m = t.mesh()
    assert g.n_elements == len(m.cells) and g.n_levels == len(octree.Hierarchy(t).meshes)
    X, Y, Z = m.nodes()
    bx, by, bz = m.boundary_points()
    b = m.rhs(_gauss(4.0, (0.2, 0.1, -0.1))(X, Y, Z), 0.1 * np.cos(bx + 2 * by) * bz)
    x, st = g.solve(_t(b[None]))
    A, _ = m.dense()
    ref = np.linalg.solve(A, b)
    assert st[0]["status"] == 0
    if g.n_levels == 1:
        assert st[0]["iters"] == 1
    assert np.abs(x.cpu().numpy()[0] - ref).max() <= 1e-9 * np.abs(ref).max()


def test_octree_arguments_are_checked(gpu_lib):
    with pytest.raises(gpu_lib.DgError):
        gpu_lib.Octree((9, 1, 1), (0, 0, 0), (1, 1, 1), q=2)          # more than 8 base elements per axis
    with pytest.raises(gpu_lib.DgError):
        gpu_lib.Octree((1, 1, 1), (0, 0, 0), (1, 1, 1), q=5)          # degree above 4
    with pytest.raises(gpu_lib.DgError):
        gpu_lib.Octree((1, 1, 1), (0, 0, 0), (1, 1, 1), q=2, precision="bf16f_pc")
    with pytest.raises(gpu_lib.DgError, match="max_elements"):
        gpu_lib.Octree((2, 2, 2), (-2, -2, -2), (2, 2, 2), q=2, rho=_two_centres, delta_q=1e-9, max_depth=4,
                       max_elements=100)
    with pytest.raises(gpu_lib.DgError, match="finite"):
        gpu_lib.Octree((1, 1, 1), (0, 0, 0), (1, 1, 1), q=2, rho=lambda x, y, z: np.nan * x)
    # no refinement without a density: the base mesh, and its operator equals the uniform GL mesh's
    o = gpu_lib.Octree((2, 3, 2), (-1.0, 0.0, -2.0), (1.5, 2.0, 1.0), q=3)
    assert o.n_elements == 12 and o.max_generation == 0
