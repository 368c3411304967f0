"""GPU parity of the Gauss-Legendre node family (dg_opts.node_family = 1, the nodes Sec. 6.2
names) against the oracle's GL construction, through the C ABI.

Bars as for the Gauss-Lobatto path: operator, right-hand side, transfers and coarsest solve to
FP64 rounding (1e-12; the coarsest solve 1e-11), the FP32 operator to 2e-5, smoother bounds and
one V-cycle to 1e-9, full solves against the exact solve at the parity tolerance (potential bar
1e-8).  The restrictions of the family (no fused solve, no learned guess, no quadrature
Dirichlet data) are argument errors.
"""
import numpy as np
import pytest

from oracle import fdm, layout, mg, sipdg
from workloads import configs

from _cases import PARITY_RTOL, POT_BAR

pytestmark = pytest.mark.gpu

CASES = [
    # (E, p, lo, hi, n_levels)
    ((4, 6, 2), 4, (-2.0, -3.0, -1.0), (2.0, 3.0, 1.0), 0),     # degree steps 4 -> 2 -> 1
    ((5, 3, 7), 3, (-2.5, -1.0, -3.0), (2.5, 2.0, 4.0), 0),     # N = 4, partial bricks
    ((6, 5, 3), 2, (0.0, 0.0, 0.0), (3.0, 2.5, 1.5), 0),        # N = 3
    ((3, 2, 2), 6, (-1.0, -1.0, -1.0), (2.0, 1.0, 1.0), 0),     # N = 7, one-element bricks
    ((8, 8, 8), 1, (-4.0, -4.0, -4.0), (4.0, 4.0, 4.0), 2),     # p = 1, a mesh-coarsening step
]
IDS = [f"E{c[0]}p{c[1]}" for c in CASES]


def _t(a, dtype=np.float64):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _n(t):
    return t.detach().cpu().numpy()


def _ctx(gpu_lib, case, **kw):
    E, p, lo, hi, nl = case
    return gpu_lib.Context([(E, p, lo, hi)], n_levels=nl, node_family="gl", **kw)


def _hier(case):
    E, p, lo, hi, nl = case
    return mg.Hierarchy(E, p, lo, hi, n_levels=nl or None, family="gl")


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_gl_operator_apply_all_levels_fp64_and_fp32(gpu_lib, case):
    ctx = _ctx(gpu_lib, case)
    H = _hier(case)
    assert ctx.info[0]["n_levels"] == len(H.levels)
    rng = np.random.default_rng(31)
    for level, L in enumerate(H.levels):
        u = rng.standard_normal((2,) + L.shape)
        uem = np.stack([layout.to_element_major(u[r], L.E, L.n) for r in range(2)])
        ref = np.stack([layout.to_element_major(L.A(u[r]), L.E, L.n) for r in range(2)])
        y = _n(ctx.operator_apply(_t(uem), level=level)).reshape(2, -1)
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max(), level
        y32 = _n(ctx.operator_apply(_t(uem, np.float32), level=level)).reshape(2, -1)
        assert np.abs(y32 - ref).max() <= 2e-5 * np.abs(ref).max(), level


@pytest.mark.parametrize("case", CASES[:3], ids=IDS[:3])
def test_gl_rhs_assembly(gpu_lib, case):
    ctx = _ctx(gpu_lib, case)
    axes = _hier(case).levels[0].axes
    NX, NY, NZ = (axes[d].N for d in range(3))
    rng = np.random.default_rng(32)
    rho = rng.standard_normal((NZ, NY, NX))
    faces = [rng.standard_normal(s) for s in [(NZ, NY)] * 2 + [(NZ, NX)] * 2 + [(NY, NX)] * 2]
    E, n = case[0], case[1] + 1
    b = _n(ctx.rhs_assemble(_t(layout.to_element_major(rho, E, n)), _t(layout.join_faces(faces))))
    ref = layout.to_element_major(sipdg.rhs(axes, rho, faces), E, n)
    assert np.abs(b.reshape(-1) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_gl_transfers_coarse_solve_and_vcycle(gpu_lib, case):
    ctx = _ctx(gpu_lib, case)
    H = _hier(case)
    rng = np.random.default_rng(33)
    Lc = H.levels[-1]
    r = rng.standard_normal(Lc.shape)
    z = _n(ctx.coarse_solve(_t(layout.to_element_major(r, Lc.E, Lc.n))))
    ref = layout.to_element_major(H.coarse.solve(r), Lc.E, Lc.n)
    assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()
    for l in range(len(H.levels) - 1):
        F, C = H.levels[l], H.levels[l + 1]
        rf = rng.standard_normal(F.shape)
        rc = _n(ctx.restrict(_t(layout.to_element_major(rf, F.E, F.n)), level=l))
        ref = layout.to_element_major(H.restrict(l, rf), C.E, C.n)
        assert np.abs(rc - ref).max() <= 1e-12 * np.abs(ref).max(), l
        zc, zf0 = rng.standard_normal(C.shape), rng.standard_normal(F.shape)
        zf = _n(ctx.prolong_add(_t(layout.to_element_major(zc, C.E, C.n)),
                                _t(layout.to_element_major(zf0, F.E, F.n)), level=l))
        ref = layout.to_element_major(zf0 + H.prolong(l, zc), F.E, F.n)
        assert np.abs(zf - ref).max() <= 1e-12 * np.abs(ref).max(), l
        li = ctx.level_info(0, l)
        assert abs(li["lam_hi"] - H.lam[l][1]) <= 1e-9 * H.lam[l][1], l
    L0 = H.levels[0]
    r = rng.standard_normal(L0.shape)
    z = _n(ctx.vcycle(_t(layout.to_element_major(r, L0.E, L0.n))))
    ref = layout.to_element_major(H.vcycle(r), L0.E, L0.n)
    assert np.abs(z - ref).max() <= 1e-9 * np.abs(ref).max()


def _gaussian_problem(ctx, case, dens):
    """rho and g of a closed-form density at the library's nodes and face points, and the oracle's
    exact solution with the same data at its own nodes and face points."""
    xyz, fxyz = ctx.mesh_coords(0)
    rho = dens.density(xyz[0], xyz[1], xyz[2])
    g = dens.potential(fxyz[0], fxyz[1], fxyz[2])
    axes = _hier(case).levels[0].axes
    X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
    faces = [dens.potential(*fp) for fp in sipdg.face_points(axes)]
    ex = fdm.FDM(axes).solve(sipdg.rhs(axes, dens.density(X, Y, Z), faces))
    return rho, g, axes, ex


@pytest.mark.parametrize("precision", ["fp64", "fp32_pc", "bf16f_pc", "fp32_ir"])
def test_gl_full_solves_match_the_exact_solve(gpu_lib, precision):
    """Two Gaussian densities on the degree-4 GL mesh (3 levels) in one call: every potential
    against the oracle's exact GL solve (BF16F_PC runs as FP32_PC on these levels; FP32_IR at the
    tighter FP32 refinement tolerance)."""
    case = ((6, 4, 4), 4, (-3.0, -2.0, -2.0), (3.0, 2.0, 2.0), 0)
    rtol = 1e-12 if precision == "fp32_ir" else PARITY_RTOL
    ctx = _ctx(gpu_lib, case, rtol=rtol, precision=precision)
    dens = [configs.scaled(4, 4, 2, seed=3).batch.densities[k] for k in range(2)]
    probs = [_gaussian_problem(ctx, case, d) for d in dens]
    v, st = ctx.solve_batch(_t(np.concatenate([p[0] for p in probs])), _t(np.concatenate([p[1] for p in probs])))
    assert all(s["status"] == 0 and s["rel_residual"] <= rtol for s in st)
    v = _n(v).reshape(2, -1)
    E, n = case[0], case[1] + 1
    for k, (_, _, axes, ex) in enumerate(probs):
        M = sipdg.mass(axes)
        got = layout.to_global(v[k], E, n)
        assert np.sqrt(np.sum(M * (got - ex) ** 2) / np.sum(M * ex ** 2)) <= POT_BAR, k


def test_gl_restrictions_are_argument_errors(gpu_lib):
    case = CASES[0]
    with pytest.raises(gpu_lib.DgError, match="invalid argument"):
        _ctx(gpu_lib, case, fused=1)
    ctx = _ctx(gpu_lib, case)
    net = gpu_lib.Net(4, 8, 125, 27)
    with pytest.raises(gpu_lib.DgError, match="Gauss-Lobatto"):
        ctx.attach_guess(net)
    nd = ctx.info[0]["n_dofs"]
    rho = _t(np.ones(nd))
    with pytest.raises(gpu_lib.DgError, match="quadrature"):
        ctx.solve_batch(rho, None)
