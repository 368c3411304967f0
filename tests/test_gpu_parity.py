"""GPU parity: every step of the HIP path against the FP64 oracle, through the C ABI.

Bars: operator, transfers, right-hand side and coarsest solve agree with the
oracle to FP64 rounding (relative 1e-12); smoother bounds and one V-cycle to
1e-9 (Lanczos in a different summation order); full solves are compared with
the exact (fast-diagonalisation) solution at the parity tolerance 1e-11:
relative M-weighted L2 error <= 1e-8 and pair energies within 1e-10 Ha.
"""
import numpy as np
import pytest

from oracle import exchange as ox, fdm, layout, mg, pcg, sipdg
from workloads import configs, gaussians

from _cases import (ENERGY_BAR, PARITY_RTOL, PARITY_RTOL_FP32, POT_BAR, from_em, gpu_sample, level_axes, oracle_axes,
                    oracle_density_problem, oracle_faces, oracle_grid, rel_l2_M, to_em)

pytestmark = pytest.mark.gpu

CASES = [
    # (E, p, lo, hi, n_levels)
    ((4, 6, 2), 4, (-2.0, -3.0, -1.0), (2.0, 3.0, 1.0), 0),     # N=5, bricks 2^3
    ((5, 3, 7), 3, (-2.5, -1.0, -3.0), (2.5, 2.0, 4.0), 0),     # N=4, partial bricks
    ((6, 5, 3), 2, (0.0, 0.0, 0.0), (3.0, 2.5, 1.5), 0),        # N=3, bricks 4^3, partial
    ((3, 2, 2), 6, (-1.0, -1.0, -1.0), (2.0, 1.0, 1.0), 0),     # N=7, one-element bricks
    ((2, 2, 1), 7, (-1.0, -1.0, -0.5), (1.0, 1.0, 0.5), 0),     # N=8, single element along z
    ((8, 8, 8), 1, (-4.0, -4.0, -4.0), (4.0, 4.0, 4.0), 2),     # p=1 fine level, mesh coarsening
]


def _mesh(c):
    E, p, lo, hi, _ = c
    return configs.Mesh(E, p, lo, hi)


def _ctx(gpu_lib, cases, **kw):
    return gpu_lib.Context([(c[0], c[1], c[2], c[3]) for c in cases], n_levels=cases[0][4], **kw)


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _n(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=[f"E{c[0]}p{c[1]}" for c in CASES])
def test_operator_apply_all_levels(gpu_lib, case):
    mesh = _mesh(case)
    ctx = _ctx(gpu_lib, [case])
    nl = ctx.info[0]["n_levels"]
    assert nl == len(mg.hierarchy(mesh.E, mesh.p, case[4] or None))
    rng = np.random.default_rng(11)
    for level in range(nl):
        axes, E, p = level_axes(mesh, case[4] or None, level)
        n = p + 1
        nrhs = 3
        u = rng.standard_normal((nrhs, int(np.prod(E)) * n ** 3))
        y = _n(ctx.operator_apply(_t(u), level=level)).reshape(nrhs, -1)
        for r in range(nrhs):
            ref = layout.to_element_major(sipdg.apply(axes, layout.to_global(u[r], E, n)), E, n)
            assert np.abs(y[r] - ref).max() <= 1e-12 * np.abs(ref).max(), (level, r)


def _t32(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("case", CASES, ids=[f"E{c[0]}p{c[1]}" for c in CASES])
def test_operator_apply_fp32_all_levels(gpu_lib, case):
    """The FP32 kernels of the mixed-precision inner solve (tiles, ghosts and coefficients in
    FP32) against the FP64 oracle, to FP32 rounding: an indexing or coefficient slip gives
    O(1) relative errors, far above this bar."""
    mesh = _mesh(case)
    ctx = _ctx(gpu_lib, [case])
    nl = ctx.info[0]["n_levels"]
    rng = np.random.default_rng(21)
    for level in range(nl):
        axes, E, p = level_axes(mesh, case[4] or None, level)
        n = p + 1
        nrhs = 2
        u = rng.standard_normal((nrhs, int(np.prod(E)) * n ** 3)).astype(np.float32)
        y = _n(ctx.operator_apply(_t32(u), level=level)).reshape(nrhs, -1)
        for r in range(nrhs):
            ref = layout.to_element_major(sipdg.apply(axes, layout.to_global(u[r].astype(np.float64), E, n)), E, n)
            assert np.abs(y[r] - ref).max() <= 2e-5 * np.abs(ref).max(), (level, r)


@pytest.mark.parametrize("case", CASES, ids=[f"E{c[0]}p{c[1]}" for c in CASES])
def test_vcycle_fp32(gpu_lib, case):
    """One FP32 V-cycle (FP32 smoothing, transfers and restriction epilogue, FP64 coarsest
    solve) against the oracle's FP64 V-cycle, to FP32 rounding."""
    mesh = _mesh(case)
    ctx = _ctx(gpu_lib, [case])
    H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi, n_levels=case[4] or None)
    L0 = H.levels[0]
    r = np.random.default_rng(22).standard_normal(L0.shape)
    z = _n(ctx.vcycle(_t32(layout.to_element_major(r, L0.E, L0.n))))
    ref = layout.to_element_major(H.vcycle(r), L0.E, L0.n)
    assert np.abs(z - ref).max() <= 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("case", CASES[:3], ids=[f"E{c[0]}p{c[1]}" for c in CASES[:3]])
def test_rhs_assembly(gpu_lib, case):
    mesh = _mesh(case)
    ctx = _ctx(gpu_lib, [case])
    axes = oracle_axes(mesh)
    rng = np.random.default_rng(12)
    nrhs = 2
    NX, NY, NZ = (axes[d].N for d in range(3))
    rho = rng.standard_normal((nrhs, NZ, NY, NX))
    faces = [[rng.standard_normal(s) for s in [(NZ, NY)] * 2 + [(NZ, NX)] * 2 + [(NY, NX)] * 2] for _ in range(nrhs)]
    rho_em = np.concatenate([to_em(rho[r], mesh) for r in range(nrhs)])
    g = np.concatenate([layout.join_faces(faces[r]) for r in range(nrhs)])
    b = _n(ctx.rhs_assemble(_t(rho_em), _t(g))).reshape(nrhs, -1)
    for r in range(nrhs):
        ref = to_em(sipdg.rhs(axes, rho[r], faces[r]), mesh)
        assert np.abs(b[r] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("case", CASES, ids=[f"E{c[0]}p{c[1]}" for c in CASES])
def test_coarse_solve_and_transfers(gpu_lib, case):
    mesh = _mesh(case)
    ctx = _ctx(gpu_lib, [case])
    H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi, n_levels=case[4] or None)
    rng = np.random.default_rng(13)
    # coarsest exact solve
    Lc = H.levels[-1]
    r = rng.standard_normal(Lc.shape)
    z = _n(ctx.coarse_solve(_t(layout.to_element_major(r, Lc.E, Lc.n))))
    ref = layout.to_element_major(H.coarse.solve(r), Lc.E, Lc.n)
    assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()
    # restriction and prolongation between every pair of levels
    for l in range(len(H.levels) - 1):
        F, C = H.levels[l], H.levels[l + 1]
        rf = rng.standard_normal(F.shape)
        rc = _n(ctx.restrict(_t(layout.to_element_major(rf, F.E, F.n)), level=l))
        ref = layout.to_element_major(H.restrict(l, rf), C.E, C.n)
        assert np.abs(rc - ref).max() <= 1e-12 * np.abs(ref).max()
        zc = rng.standard_normal(C.shape)
        zf0 = rng.standard_normal(F.shape)
        zf = _n(ctx.prolong_add(_t(layout.to_element_major(zc, C.E, C.n)),
                                _t(layout.to_element_major(zf0, F.E, F.n)), level=l))
        ref = layout.to_element_major(zf0 + H.prolong(l, zc), F.E, F.n)
        assert np.abs(zf - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("case", CASES, ids=[f"E{c[0]}p{c[1]}" for c in CASES])
def test_smoother_bounds_and_vcycle(gpu_lib, case):
    mesh = _mesh(case)
    ctx = _ctx(gpu_lib, [case])
    H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi, n_levels=case[4] or None)
    for l in range(len(H.levels) - 1):
        li = ctx.level_info(0, l)
        assert abs(li["lam_hi"] - H.lam[l][1]) <= 1e-9 * H.lam[l][1]
        assert abs(li["lam_lo"] - H.lam[l][0]) <= 1e-9 * H.lam[l][0]
    L0 = H.levels[0]
    r = np.random.default_rng(14).standard_normal(L0.shape)
    z = _n(ctx.vcycle(_t(layout.to_element_major(r, L0.E, L0.n))))
    ref = layout.to_element_major(H.vcycle(r), L0.E, L0.n)
    assert np.abs(z - ref).max() <= 1e-9 * np.abs(ref).max()


def test_single_gaussian_solve_matches_exact_and_closed_form(gpu_lib):
    wl = configs.single()
    mesh, dens = wl.meshes[0], wl.batch.densities[0]
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=wl.rtol)
    rho, g = gpu_sample(ctx, 0, dens)
    v, st = ctx.solve_batch(_t(rho), _t(g))
    axes, rho_o, faces, b = oracle_density_problem(mesh, dens)
    v_ex = fdm.FDM(axes).solve(b)
    assert rel_l2_M(axes, mesh, _n(v), v_ex) <= POT_BAR
    assert st[0]["status"] == 0 and st[0]["rel_residual"] <= wl.rtol
    H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi, n_levels=wl.n_levels)
    _, it_o, _, _ = pcg.solve(H, b, rtol=wl.rtol)
    assert abs(st[0]["iters"] - it_o) <= 1
    X, Y, Z = oracle_grid(axes)
    err = rel_l2_M(axes, mesh, _n(v), dens.potential(X, Y, Z))
    assert 1e-2 < err < 4e-2   # discretisation error against erf(sqrt(a) r)/r


def test_batch_over_two_meshes_interleaved(gpu_lib):
    wl = configs.scaled(4, 4, 3, seed=21)
    m0 = wl.meshes[0]
    m1 = configs.Mesh((6, 4, 4), 3, (-3.0, -2.0, -2.0), (3.0, 2.0, 2.0))
    ctx = gpu_lib.Context([(m.E, m.p, m.lo, m.hi) for m in (m0, m1)], rtol=PARITY_RTOL)
    ids = [0, 1, 0, 1, 1]
    dens = [wl.batch.densities[k % 3] for k in range(len(ids))]
    rho, g = [], []
    for k, mid in enumerate(ids):
        r_, g_ = gpu_sample(ctx, mid, dens[k])
        rho.append(r_); g.append(g_)
    v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)), mesh_ids=ids)
    v = _n(v)
    off = 0
    for k, mid in enumerate(ids):
        mesh = (m0, m1)[mid]
        axes, _, _, b = oracle_density_problem(mesh, dens[k])
        n = ctx.info[mid]["n_dofs"]
        assert rel_l2_M(axes, mesh, v[off:off + n], fdm.FDM(axes).solve(b)) <= POT_BAR
        assert st[k]["status"] == 0
        off += n


def test_uneven_batch_three_meshes_matches_oracle_and_per_mesh_solves(gpu_lib):
    """Interleaved right-hand sides of three meshes (degrees 4, 3 and 2) in one call, mixed
    precision: every potential against the exact solve, and bitwise equal to solving each
    mesh's right-hand sides on their own (the batch only regroups and overlaps them)."""
    meshes = [configs.Mesh((4, 4, 4), 4, (-2.0,) * 3, (2.0,) * 3),
              configs.Mesh((6, 4, 4), 3, (-3.0, -2.0, -2.0), (3.0, 2.0, 2.0)),
              configs.Mesh((4, 6, 4), 2, (-2.0, -3.0, -2.0), (2.0, 3.0, 2.0))]
    wl = configs.scaled(4, 4, 7, seed=33)
    ids = [2, 0, 1, 2, 0, 1, 1]
    dens = [wl.batch.densities[k] for k in range(len(ids))]
    ctx = gpu_lib.Context([(m.E, m.p, m.lo, m.hi) for m in meshes], rtol=PARITY_RTOL_FP32, precision="fp32_ir")
    rho, g = [], []
    for k, mid in enumerate(ids):
        r_, g_ = gpu_sample(ctx, mid, dens[k])
        rho.append(r_); g.append(g_)
    v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)), mesh_ids=ids)
    v = _n(v)
    offs = np.cumsum([0] + [ctx.info[mid]["n_dofs"] for mid in ids])
    for k, mid in enumerate(ids):
        axes, _, _, b = oracle_density_problem(meshes[mid], dens[k])
        assert rel_l2_M(axes, meshes[mid], v[offs[k]:offs[k + 1]], fdm.FDM(axes).solve(b)) <= POT_BAR
        assert st[k]["status"] == 0
    # the converged potentials as initial guesses (gathered like rho): nothing left to do
    v2, st2 = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)), mesh_ids=ids, x0=_t(v))
    assert np.array_equal(_n(v2), v) and all(s["iters"] == 0 and s["guess_used"] == 1 for s in st2)
    for mid in range(3):
        ks = [k for k, m in enumerate(ids) if m == mid]
        vm, sm = ctx.solve_batch(_t(np.concatenate([rho[k] for k in ks])), _t(np.concatenate([g[k] for k in ks])),
                                 mesh_ids=[mid] * len(ks))
        vm = _n(vm)
        n = ctx.info[mid]["n_dofs"]
        for q, k in enumerate(ks):
            assert np.array_equal(vm[q * n:(q + 1) * n], v[offs[k]:offs[k + 1]])
            assert sm[q]["iters"] == st[k]["iters"]


def test_solver_lanes_match_one_lane_bitwise(gpu_lib):
    """A batch of 36 right-hand sides of one mesh is split over 2 (default), 3 or 4 concurrent
    solver lanes (parts of 18, 12 and 9) or solved as one group (lanes=1): the potentials and
    iteration counts agree bit for bit, in every precision."""
    wl = configs.scaled(4, 4, 36, seed=41)
    mesh = wl.meshes[0]
    m = (mesh.E, mesh.p, mesh.lo, mesh.hi)
    for prec in ("fp64", "fp32_ir", "fp32_pc", "bf16_pc", "bf16f_pc"):
        out = []
        for lanes in (1, 2, 3, 4):
            ctx = gpu_lib.Context([m], precision=prec, lanes=lanes)
            rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
            v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)))
            out.append((_n(v), [s["iters"] for s in st]))
            ctx.close()
        for k in range(1, 4):
            assert np.array_equal(out[0][0], out[k][0]) and out[0][1] == out[k][1], (prec, k + 1)


def test_zero_and_empty_right_hand_sides(gpu_lib):
    mesh = configs.Mesh((4, 4, 4), 2, (-1.0,) * 3, (1.0,) * 3)
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)])
    nd, nf = ctx.info[0]["n_dofs"], ctx.info[0]["n_face"]
    v, st = ctx.solve_batch(_t(np.zeros(nd)), _t(np.zeros(nf)))
    assert np.all(_n(v) == 0.0) and st[0]["iters"] == 0
    v, st = ctx.solve_batch(_t(np.zeros(0)), _t(np.zeros(0)), mesh_ids=[])
    assert v.numel() == 0 and st == []


def test_invalid_arguments_are_rejected(gpu_lib):
    with pytest.raises(gpu_lib.DgError):
        gpu_lib.Context([((4, 4, 4), 9, (0,) * 3, (1,) * 3)])
    with pytest.raises(gpu_lib.DgError):
        gpu_lib.Context([((4, 4, 4), 2, (0,) * 3, (0,) * 3)])
    ctx = gpu_lib.Context([((4, 4, 4), 2, (0,) * 3, (1,) * 3)])
    code = gpu_lib.lib.dg_mesh_info(ctx._h, 5, None, None, None)
    assert code == -1


def test_every_compiled_tile_gives_the_same_operator(gpu_lib):
    """The operator and a V-cycle do not depend on the work-group tile: every compiled tile of
    the degree-4 slab kernel (4x2, 4x4, 2x2; 1 to 4 layers per chunk) reproduces the default
    tile's A u to 1e-13, in FP64 and FP32 (a context takes the tiles set before its set-up)."""
    mesh = configs.Mesh((5, 3, 6), 4, (-2.0, -1.0, -3.0), (2.5, 2.0, 3.0))
    m = (mesh.E, mesh.p, mesh.lo, mesh.hi)
    ref = gpu_lib.Context([m])
    nd = ref.info[0]["n_dofs"]
    u = np.random.default_rng(3).standard_normal(3 * nd)
    y64 = _n(ref.operator_apply(_t(u)))
    import torch
    u32 = torch.as_tensor(u.astype(np.float32)).cuda()
    y32 = ref.operator_apply(u32).cpu().numpy().astype(np.float64)
    saved = {(fp, st): gpu_lib.tile_get(fp, 5, st) for fp in (4, 8) for st in ("APPLY",)}
    try:
        for tx, ty in ((4, 2), (4, 4), (2, 2)):
            for z in (1, 2, 3, 4):
                for fp in (4, 8):
                    gpu_lib.tile_set(fp, 5, "APPLY", tx, ty, z)
                ctx = gpu_lib.Context([m])
                assert gpu_lib.tile_get(8, 5, "APPLY") == (tx, ty, z)
                d64 = np.max(np.abs(_n(ctx.operator_apply(_t(u))) - y64))
                d32 = np.max(np.abs(ctx.operator_apply(u32).cpu().numpy().astype(np.float64) - y32))
                assert d64 <= 1e-13 * np.max(np.abs(y64)), (tx, ty, z)
                assert d32 <= 1e-6 * np.max(np.abs(y32)), (tx, ty, z)
                ctx.close()
    finally:
        for (fp, st), t in saved.items():
            gpu_lib.tile_set(fp, 5, st, *t)


def test_full_solves_agree_on_every_compiled_tile(gpu_lib):
    """Full solves with every step of the degree-4 level on another compiled tile (both
    arithmetics, FP64 and mixed precision, two solver lanes) reach the same potentials as with
    the default tiles: only the order of the partial dot products changes."""
    wl = configs.scaled(4, 4, 18, seed=53)
    mesh = wl.meshes[0]
    m = (mesh.E, mesh.p, mesh.lo, mesh.hi)
    steps = list(gpu_lib.STEPS)
    saved = {(fp, st): gpu_lib.tile_get(fp, 5, st) for fp in (4, 8) for st in steps}

    def solve(prec):
        ctx = gpu_lib.Context([m], precision=prec, rtol=1e-11)
        rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
        v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)))
        assert all(s["status"] == 0 for s in st)
        ctx.close()
        return _n(v)

    ref = {prec: solve(prec) for prec in ("fp64", "fp32_ir")}
    try:
        for tile in ((4, 2, 4), (4, 4, 2), (2, 2, 3)):
            for fp in (4, 8):
                for st in steps:
                    gpu_lib.tile_set(fp, 5, st, *tile)
            for prec in ("fp64", "fp32_ir"):
                v = solve(prec)
                assert np.max(np.abs(v - ref[prec])) <= 1e-8 * np.max(np.abs(ref[prec])), (tile, prec)
    finally:
        for (fp, st), t in saved.items():
            gpu_lib.tile_set(fp, 5, st, *t)


def test_non_finite_inputs_are_rejected(gpu_lib):
    """A NaN or Inf in a source, its Dirichlet data or a caller's initial guess is reported as
    an argument error, in every precision and over two solver lanes (20 right-hand sides); the
    context solves normally afterwards."""
    wl = configs.scaled(4, 2, 20, seed=43)
    mesh = wl.meshes[0]
    for prec in ("fp64", "fp32_ir", "fp32_pc"):
        ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], precision=prec)
        assert ctx.opts.lanes == 2
        rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
        rho, g = np.concatenate(rho), np.concatenate(g)
        nd, nf = ctx.info[0]["n_dofs"], ctx.info[0]["n_face"]
        bad = rho.copy()
        bad[5 * nd + 17] = np.nan
        with pytest.raises(gpu_lib.DgError, match="non-finite"):
            ctx.solve_batch(_t(bad), _t(g))
        bad = g.copy()
        bad[13 * nf + 3] = np.inf
        with pytest.raises(gpu_lib.DgError, match="non-finite"):
            ctx.solve_batch(_t(rho), _t(bad))
        x0 = np.zeros_like(rho)
        x0[2 * nd] = np.nan
        with pytest.raises(gpu_lib.DgError, match="non-finite"):
            ctx.solve_batch(_t(rho), _t(g), x0=_t(x0))
        v, st = ctx.solve_batch(_t(rho), _t(g))
        assert all(s["status"] == 0 for s in st) and np.all(np.isfinite(_n(v))), prec


def test_mixed_precision_falls_back_to_fp64(gpu_lib):
    """With a single refinement step the FP32 inner solves (to 1e-4) cannot reach 1e-11: the
    FP64 fallback finishes every right-hand side from its current iterate (one more outer
    step counted), and the potentials agree with the plain FP64 solver's."""
    wl = configs.scaled(4, 4, 20, seed=47)
    mesh = wl.meshes[0]
    m = (mesh.E, mesh.p, mesh.lo, mesh.hi)
    ctx = gpu_lib.Context([m], precision="fp32_ir", max_outer=1, rtol=1e-11)
    rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
    rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
    v, st = ctx.solve_batch(rho, g)
    assert all(s["status"] == 0 and s["rel_residual"] <= 1e-11 and s["outer_iters"] == 2 for s in st)
    ref = gpu_lib.Context([m], precision="fp64", rtol=1e-11)
    v64, _ = ref.solve_batch(rho, g)
    v, v64 = _n(v), _n(v64)
    assert np.max(np.abs(v - v64)) <= 1e-8 * np.max(np.abs(v64))
    # with the default number of steps no right-hand side needs the fallback
    ctx8 = gpu_lib.Context([m], precision="fp32_ir", rtol=1e-11)
    _, st8 = ctx8.solve_batch(rho, g)
    assert all(s["status"] == 0 and s["outer_iters"] <= 8 for s in st8)


def _small_exchange_case():
    prims = gaussians.Primitives([0.6, 1.4, 0.9, 0.45, 2.0],
                                 [[0.4, 0, 0], [0.4, 0, 0], [-0.5, 0.2, 0.1], [-0.5, 0.2, 0.1], [0.1, -0.6, 0.3]])
    rng = np.random.default_rng(5)
    C = gaussians.lowdin(rng.standard_normal((5, 3)), prims.overlap())
    return gaussians.Orbitals(prims, C), configs.Mesh((6, 6, 6), 4, (-5.0,) * 3, (5.0,) * 3)


def test_exchange_matches_oracle(gpu_lib):
    orb, mesh = _small_exchange_case()
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], rtol=PARITY_RTOL)
    xyz, fxyz = ctx.mesh_coords(0)
    phi = orb.values(xyz[0], xyz[1], xyz[2])
    g = orb.pair_potentials(fxyz[0], fxyz[1], fxyz[2])
    W, K, EX, st, v = ctx.exchange(_t(phi.reshape(-1)), _t(g.reshape(-1)), keep_potentials=True)
    axes = oracle_axes(mesh)
    X, Y, Z = oracle_grid(axes)
    phi_o = list(orb.values(X, Y, Z))
    fp = [[None] * 6 for _ in orb.pairs()]
    for f, vals in enumerate(oracle_faces(axes, lambda a, b_, c: orb.pair_potentials(a.reshape(-1), b_.reshape(-1), c.reshape(-1)))):
        for q in range(len(vals)):
            fp[q][f] = vals[q].reshape(axes[2].N if f < 4 else axes[1].N, -1)
    F = fdm.FDM(axes)
    v_o, W_o, K_o, EX_o = ox.exchange(axes, phi_o, fp, F.solve)
    K = _n(K)
    assert np.abs(K - K_o).max() <= ENERGY_BAR
    assert abs(EX - EX_o) <= 3 * ENERGY_BAR
    W = _n(W).reshape(3, -1)
    v = _n(v).reshape(len(K), -1)
    for q in range(len(K)):
        assert rel_l2_M(axes, mesh, v[q], v_o[q]) <= POT_BAR
    for k in range(3):
        assert rel_l2_M(axes, mesh, W[k], W_o[k]) <= POT_BAR
    assert all(s["status"] == 0 for s in st)


def test_mixed_precision_refinement_reaches_fp64_accuracy(gpu_lib):
    wl = configs.scaled(6, 4, 2, seed=31)
    mesh = wl.meshes[0]
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], rtol=PARITY_RTOL_FP32, precision="fp32_ir")
    rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
    v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)))
    v = _n(v).reshape(2, -1)
    for k, d in enumerate(wl.batch.densities):
        axes, _, _, b = oracle_density_problem(mesh, d)
        assert rel_l2_M(axes, mesh, v[k], fdm.FDM(axes).solve(b)) <= POT_BAR
        assert st[k]["status"] == 0 and st[k]["outer_iters"] >= 2


def test_graph_replay_matches_eager_launches_bitwise(gpu_lib):
    """The captured PCG iteration, replayed several times per solve and across
    solves with eager work in between, gives bitwise the eager result."""
    import torch
    wl = configs.scaled(6, 4, 3, seed=41)
    mesh = wl.meshes[0]
    m = (mesh.E, mesh.p, mesh.lo, mesh.hi)
    outs = []
    for use_graph in (0, 1):
        for prec in ("fp64", "fp32_ir", "fp32_pc", "bf16_pc"):
            ctx = gpu_lib.Context([m], rtol=1e-10, use_graph=use_graph, precision=prec, check_every=2)
            rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
            rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
            v1, st1 = ctx.solve_batch(rho, g)
            ctx.operator_apply(v1)           # eager work between graph replays
            torch.cuda.synchronize()
            v2, st2 = ctx.solve_batch(rho, g)
            assert torch.equal(v1, v2)
            assert [s["iters"] for s in st1] == [s["iters"] for s in st2]
            outs.append((prec, _n(v1), [s["iters"] for s in st1]))
    for prec in ("fp64", "fp32_ir", "fp32_pc", "bf16_pc"):
        a, b = [o for o in outs if o[0] == prec]
        assert np.array_equal(a[1], b[1]) and a[2] == b[2]


def _box_density(mesh, seed):
    """Two or three normalised Gaussians inside the central half of a mesh's box."""
    rng = np.random.default_rng(seed)
    lo, hi = np.array(mesh.lo), np.array(mesh.hi)
    c, w = 0.5 * (lo + hi), 0.25 * (hi - lo)
    K = int(rng.integers(2, 4))
    h = float(np.min((hi - lo) / np.array(mesh.E)))
    alpha = rng.uniform(0.5, 1.5, K) / h ** 2
    return gaussians.GaussianDensity(rng.uniform(0.5, 1.5, K), alpha, c + rng.uniform(-1, 1, (K, 3)) * w)


@pytest.mark.parametrize("case", CASES, ids=[f"E{c[0]}p{c[1]}" for c in CASES])
def test_fp32_preconditioned_fp64_pcg_matches_exact(gpu_lib, case):
    """FP32_PC (FP64 PCG, FP32 V-cycle) on every operator case, the degrees without a mixed
    operator kernel included (their FP32 direction is widened first): the potential meets the
    bar against the exact solve at the parity tolerance, with the iteration count of the FP64
    solver (+-1) and a potential within FP64 CG's own error of the FP64 solver's."""
    mesh = _mesh(case)
    dens = [_box_density(mesh, 60 + k) for k in range(2)]
    out = {}
    for prec in ("fp64", "fp32_pc"):
        ctx = _ctx(gpu_lib, [case], rtol=PARITY_RTOL, precision=prec)
        rho, g = zip(*[gpu_sample(ctx, 0, d) for d in dens])
        v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)))
        assert all(s_["status"] == 0 and s_["rel_residual"] <= PARITY_RTOL for s_ in st), prec
        out[prec] = (_n(v).reshape(len(dens), -1), [s_["iters"] for s_ in st])
    for k, d in enumerate(dens):
        axes, _, _, b = oracle_density_problem(mesh, d)
        ref = fdm.FDM(axes).solve(b)
        assert rel_l2_M(axes, mesh, out["fp32_pc"][0][k], ref) <= POT_BAR, k
        assert abs(out["fp32_pc"][1][k] - out["fp64"][1][k]) <= 1, k


P4_CASES = [
    ((4, 6, 2), 4, (-2.0, -3.0, -1.0), (2.0, 3.0, 1.0), 0),      # every 4 x 2 tile at a face, 2 levels:
                                                                 # BF16 fields on the finest level only
    ((10, 6, 4), 4, (-5.0, -3.0, -2.0), (5.0, 3.0, 2.0), 0),     # interior and ragged tiles, 3 levels: BF16
                                                                 # on the degree-2 level, restricted into the
                                                                 # coarsest
    ((8, 8, 8), 4, (-4.0, -4.0, -4.0), (4.0, 4.0, 4.0), 0),      # 4 levels (degree steps, then a mesh step)
]


@pytest.mark.parametrize("case", P4_CASES, ids=[f"E{c[0]}" for c in P4_CASES])
def test_bf16_field_vcycle_pcg_matches_exact(gpu_lib, case):
    """BF16F_PC: FP64 CG (search direction stored in FP32) preconditioned by the V-cycle whose
    fields (source, smoother iterates) on the finest level and, below it, on its degree-2 step are
    stored in BF16: the potentials meet the bar against the exact solve at the parity tolerance,
    with FP32_PC's iteration count (+-1); the mode also runs in an interleaved batch over two lanes
    and a second call from the converged potentials does no iteration."""
    mesh = _mesh(case)
    dens = [_box_density(mesh, 160 + k) for k in range(20)]
    out = {}
    for prec in ("fp32_pc", "bf16f_pc"):
        ctx = _ctx(gpu_lib, [case], rtol=PARITY_RTOL, precision=prec)
        rho, g = zip(*[gpu_sample(ctx, 0, d) for d in dens])
        rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
        v, st = ctx.solve_batch(rho, g)
        assert all(s_["status"] == 0 and s_["rel_residual"] <= PARITY_RTOL for s_ in st), prec
        v2, st2 = ctx.solve_batch(rho, g, x0=v)
        assert all(s_["iters"] == 0 and s_["guess_used"] == 1 for s_ in st2), prec
        out[prec] = (_n(v).reshape(len(dens), -1), [s_["iters"] for s_ in st])
    for k in (0, 9, 19):
        axes, _, _, b = oracle_density_problem(mesh, dens[k])
        assert rel_l2_M(axes, mesh, out["bf16f_pc"][0][k], fdm.FDM(axes).solve(b)) <= POT_BAR, k
    assert max(abs(a - b_) for a, b_ in zip(out["bf16f_pc"][1], out["fp32_pc"][1])) <= 1
    # the BF16 fields were used (the mode did not fall back to FP32_PC): the potentials differ
    assert not np.array_equal(out["bf16f_pc"][0], out["fp32_pc"][0])


def test_single_level_hierarchy(gpu_lib):
    """A degree-1 mesh of at most 16 nodes per axis has a single multigrid level with default
    options: PCG is preconditioned by the exact solve alone and converges at once, in every
    precision, to the exact solution."""
    mesh = configs.Mesh((8, 8, 8), 1, (-4.0,) * 3, (4.0,) * 3)
    dens = _box_density(mesh, 71)
    axes, _, _, b = oracle_density_problem(mesh, dens)
    ref = fdm.FDM(axes).solve(b)
    for prec in ("fp64", "fp32_pc", "fp32_ir", "bf16f_pc"):
        ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], rtol=PARITY_RTOL, precision=prec)
        assert ctx.info[0]["n_levels"] == 1
        rho, g = gpu_sample(ctx, 0, dens)
        v, st = ctx.solve_batch(_t(rho), _t(g))
        assert st[0]["status"] == 0 and st[0]["iters"] <= (2 if prec != "fp32_ir" else 8), (prec, st)
        assert rel_l2_M(axes, mesh, _n(v), ref) <= POT_BAR, prec


def test_call_status_without_statistics(gpu_lib):
    """A caller that passes no statistics array still learns that a right-hand side missed its
    tolerance: the call returns DG_WARN_NOT_CONVERGED (one PCG iteration cannot reach 1e-12)."""
    import ctypes
    wl = configs.scaled(4, 4, 2, seed=73)
    mesh = wl.meshes[0]
    for prec in ("fp64", "fp32_pc", "fp32_ir"):
        ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], rtol=1e-12, max_iter=1, max_outer=1,
                              precision=prec)
        rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
        rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
        v = torch_empty_like(rho)
        ids = (ctypes.c_int * 2)(0, 0)
        code = gpu_lib.lib.dg_poisson_solve_batch(ctx._h, 2, ids, ctypes.c_void_p(rho.data_ptr()),
                                                  ctypes.c_void_p(g.data_ptr()), None,
                                                  ctypes.c_void_p(v.data_ptr()), None, gpu_lib._stream())
        assert code == gpu_lib.DG_WARN_NOT_CONVERGED, (prec, code)


def torch_empty_like(t):
    import torch
    return torch.empty_like(t)


def test_pair_densities_every_pair_and_subranges(gpu_lib):
    """dg_pair_densities forms phi_i phi_j bitwise (one FP64 product per node) in row-major pair
    order, for the whole triangle and for sub-ranges that start and end inside a row; bad
    ranges are argument errors."""
    rng = np.random.default_rng(81)
    norb, nd = 7, 3001
    phi = rng.standard_normal((norb, nd))
    pairs = [(i, j) for i in range(norb) for j in range(i, norb)]
    ref = np.stack([phi[i] * phi[j] for i, j in pairs])
    tphi = _t(phi.reshape(-1))
    assert np.array_equal(_n(gpu_lib.pair_densities(tphi, norb)).reshape(len(pairs), nd), ref)
    for first, count in ((0, 1), (5, 9), (13, 15), (27, 1)):
        got = _n(gpu_lib.pair_densities(tphi, norb, first, count)).reshape(count, nd)
        assert np.array_equal(got, ref[first:first + count]), (first, count)
    for first, count in ((-1, 2), (20, 9), (0, 29)):
        with pytest.raises(gpu_lib.DgError):
            gpu_lib.pair_densities(tphi, norb, first, count)


@pytest.mark.parametrize("case", [c for c in CASES if np.prod(c[0]) * (c[1] + 1) ** 3 <= 8192],
                         ids=[f"E{c[0]}p{c[1]}" for c in CASES if np.prod(c[0]) * (c[1] + 1) ** 3 <= 8192])
def test_fused_small_mesh_solve_matches_level_kernels(gpu_lib, case):
    """With fused = 1, a mesh whose levels all have at most 8,192 nodes is solved in FP64 by one
    launch, one work-group per right-hand side (the whole PCG and V-cycle in the kernel, fields in
    LDS when they fit, else in global work space; both forms occur among these cases): the
    potentials meet the bar against the exact solve at the parity tolerance, with the
    level-by-level solver's iteration counts (+-1), for a batch of 20 over two lanes and with an
    initial guess."""
    mesh = _mesh(case)
    dens = [_box_density(mesh, 90 + k) for k in range(20)]
    out = {}
    for fused in (1, 0):
        ctx = _ctx(gpu_lib, [case], rtol=PARITY_RTOL, fused=fused)
        rho, g = zip(*[gpu_sample(ctx, 0, d) for d in dens])
        rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
        v, st = ctx.solve_batch(rho, g)
        assert all(s_["status"] == 0 and s_["rel_residual"] <= PARITY_RTOL for s_ in st), fused
        # the converged potentials as guesses: nothing left to do
        v2, st2 = ctx.solve_batch(rho, g, x0=v)
        assert all(s_["iters"] == 0 and s_["guess_used"] == 1 for s_ in st2), fused
        out[fused] = (_n(v).reshape(len(dens), -1), [s_["iters"] for s_ in st])
    for k in (0, 7, 19):
        axes, _, _, b = oracle_density_problem(mesh, dens[k])
        assert rel_l2_M(axes, mesh, out[1][0][k], fdm.FDM(axes).solve(b)) <= POT_BAR, k
    assert max(abs(a - b_) for a, b_ in zip(out[1][1], out[0][1])) <= 1


GROUP_CASES = [c for c in CASES if c[1] <= 4] + [
    ((4, 4, 4), 1, (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0), 0),    # one level: the exact solve preconditions
]


@pytest.mark.parametrize("K", [1, 4])
@pytest.mark.parametrize("case", GROUP_CASES, ids=[f"E{c[0]}p{c[1]}" for c in GROUP_CASES])
def test_group_persistent_solve_matches_exact(gpu_lib, case, K):
    """With fused = 2 the whole FP64 PCG runs in one launch, a group of K work-groups per
    right-hand side separated by group barriers (operator evaluated per node, transfers by
    gather, coarsest solve in three group phases): the potentials meet the bar against the exact
    solve at the parity tolerance, with the level-by-level solver's iteration counts (+-1), for a
    batch of 20 over two lanes, and converged potentials given back as guesses need no iteration."""
    mesh = _mesh(case)
    dens = [_box_density(mesh, 190 + k) for k in range(20)]
    out = {}
    for fused in (2, 0):
        ctx = _ctx(gpu_lib, [case], rtol=PARITY_RTOL, fused=fused, fused_wgs=K)
        rho, g = zip(*[gpu_sample(ctx, 0, d) for d in dens])
        rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
        v, st = ctx.solve_batch(rho, g)
        assert all(s_["status"] == 0 and s_["rel_residual"] <= PARITY_RTOL for s_ in st), fused
        v2, st2 = ctx.solve_batch(rho, g, x0=v)
        assert all(s_["iters"] == 0 and s_["guess_used"] == 1 for s_ in st2), fused
        assert ctx.fused_fallbacks() == 0
        out[fused] = (_n(v).reshape(len(dens), -1), [s_["iters"] for s_ in st])
    for k in (0, 11, 19):
        axes, _, _, b = oracle_density_problem(mesh, dens[k])
        assert rel_l2_M(axes, mesh, out[2][0][k], fdm.FDM(axes).solve(b)) <= POT_BAR, k
    assert max(abs(a - b_) for a, b_ in zip(out[2][1], out[0][1])) <= 1


def test_group_persistent_single_gaussian(gpu_lib):
    """The single-Gaussian workload (4^3 elements, p = 3, two levels) by the group-persistent
    solve with the automatic group size, against the exact solve."""
    wl = configs.single()
    mesh, dens = wl.meshes[0], wl.batch.densities[0]
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=wl.rtol, fused=2)
    rho, g = gpu_sample(ctx, 0, dens)
    v, st = ctx.solve_batch(_t(rho), _t(g))
    assert st[0]["status"] == 0 and st[0]["rel_residual"] <= wl.rtol
    axes, _, _, b = oracle_density_problem(mesh, dens)
    assert rel_l2_M(axes, mesh, _n(v), fdm.FDM(axes).solve(b)) <= POT_BAR
    assert ctx.fused_fallbacks() == 0


def test_group_persistent_fallback_when_a_barrier_gives_up(gpu_lib):
    """fused_spin < 0 makes every group barrier give up at its first incomplete poll (every wave
    still leaves the kernel); the call then solves the batch again with the level kernels, so the
    results still meet the bar and the context counts the fallback."""
    case = GROUP_CASES[0]
    mesh = _mesh(case)
    dens = [_box_density(mesh, 290 + k) for k in range(6)]
    ctx = _ctx(gpu_lib, [case], rtol=PARITY_RTOL, fused=2, fused_wgs=4, fused_spin=-1)
    rho, g = zip(*[gpu_sample(ctx, 0, d) for d in dens])
    v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)))
    assert all(s_["status"] == 0 and s_["rel_residual"] <= PARITY_RTOL for s_ in st)
    assert ctx.fused_fallbacks() >= 1
    v = _n(v).reshape(len(dens), -1)
    for k in (0, 5):
        axes, _, _, b = oracle_density_problem(mesh, dens[k])
        assert rel_l2_M(axes, mesh, v[k], fdm.FDM(axes).solve(b)) <= POT_BAR, k


MF_CASES = [
    ((4, 6, 2), 4, (-2.0, -3.0, -1.0), (2.0, 3.0, 1.0), 0),      # whole 4 x 2 tiles, every tile at a face
    ((10, 6, 2), 4, (-5.0, -3.0, -1.0), (5.0, 3.0, 1.0), 0),     # interior tiles, ragged tiles at the x face
]


@pytest.mark.parametrize("case", MF_CASES, ids=[f"E{c[0]}" for c in MF_CASES])
def test_matrix_core_operator_matches_oracle(gpu_lib, case):
    """The degree-4 operator with its x and y line contractions on the matrix cores (BF16 operands,
    FP32 accumulation; ghost lines at the domain faces) against the oracle's FP64 apply: each x or
    y output sums at most 15 products whose two BF16 factors are each rounded to 2^-9 relative, so
    its error is below 4e-3 of the sum of the absolute products; for random inputs that sum stays
    within a few times max|y|, and the bar is 2e-2 max|y|.  The same inputs through the FP32
    vector-unit kernel stay at FP32 rounding (2e-5), so the difference is the BF16 rounding alone."""
    mesh = _mesh(case)
    ctx = _ctx(gpu_lib, [case])
    axes = oracle_axes(mesh)
    u = np.random.default_rng(17).standard_normal((axes[2].N, axes[1].N, axes[0].N))
    ref = layout.to_element_major(sipdg.apply(axes, u), mesh.E, mesh.p + 1)
    import torch
    ut = torch.as_tensor(layout.to_element_major(u, mesh.E, mesh.p + 1), dtype=torch.float32).cuda()
    y_mf = ctx.operator_apply_mfma(ut).double().cpu().numpy()
    y_32 = ctx.operator_apply(ut).double().cpu().numpy()
    scale = np.abs(ref).max()
    err_mf = np.abs(y_mf - ref).max() / scale
    err_32 = np.abs(y_32 - ref).max() / scale
    print(f"matrix-core operator: rel. max error {err_mf:.2e} (FP32 vector units {err_32:.2e})")
    assert err_32 <= 2e-5
    assert 1e-5 < err_mf <= 2e-2
    # levels without a matrix-core kernel are refused
    with pytest.raises(gpu_lib.DgError):
        ctx.operator_apply_mfma(torch.zeros(ctx._level_dofs(0, 1), dtype=torch.float32, device="cuda"), level=1)


def test_bf16_preconditioned_fp64_pcg_matches_exact(gpu_lib):
    """BF16_PC (FP64 flexible CG, the finest-level smoothing steps on the matrix cores) reaches the
    parity tolerance and the exact solution, with at most a few more iterations than FP64."""
    wl = configs.scaled(8, 4, 6, seed=57)
    mesh = wl.meshes[0]
    out = {}
    for prec in ("fp64", "bf16_pc"):
        ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], rtol=PARITY_RTOL, precision=prec)
        rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
        v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)))
        assert all(s_["status"] == 0 and s_["rel_residual"] <= PARITY_RTOL for s_ in st), prec
        out[prec] = (_n(v).reshape(6, -1), [s_["iters"] for s_ in st])
    print("iterations fp64", out["fp64"][1], "bf16_pc", out["bf16_pc"][1])
    for k in (0, 5):
        axes, _, _, b = oracle_density_problem(mesh, wl.batch.densities[k])
        assert rel_l2_M(axes, mesh, out["bf16_pc"][0][k], fdm.FDM(axes).solve(b)) <= POT_BAR, k
    assert max(a - b_ for a, b_ in zip(out["bf16_pc"][1], out["fp64"][1])) <= 4
