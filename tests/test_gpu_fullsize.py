"""Full-size parity in the benchmark's launch configuration.

The exchange workload of 8 orbitals on the 16^3-element, p = 4 mesh (36 pair
densities, 512,000 nodes each) is solved the way the benchmark times it: FP32
inner solves inside FP64 refinement, the trained initial-guess network, two
solver lanes, captured graphs.  The oracle solves a sample of the pair
problems exactly (fast diagonalisation), one by one.  At the parity tolerance
(1e-12 for FP32 refinement, 1e-11 for the plain FP64 solver) the sampled
potentials and pair energies meet the parity bars; at the
benchmark's tolerance 1e-8 their error stays within what such a residual
leaves (an oracle study on these pairs found potential errors up to 9.7e-8
and pair-energy errors up to 2.4e-8 Ha, the first-order part coming from the
Dirichlet lift).
"""
import os

import numpy as np
import pytest

from oracle import exchange as ox, fdm
from workloads import configs

from _cases import (ENERGY_BAR, PARITY_RTOL, PARITY_RTOL_FP32, POT_BAR, oracle_axes, oracle_faces, oracle_grid,
                    rel_l2_M)

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2510_21213_amd", "weights", "guess_16e_p4.bin")
SAMPLE = [(0, 5), (3, 7)]      # orbital pairs (i, j): the pairs ii, ij and jj are checked
BENCH_POT_BAR = 3e-7           # at residual 1e-8 (observed <= 9.7e-8)
BENCH_ENERGY_BAR = 1e-7        # hartree, at residual 1e-8 (observed <= 2.4e-8)


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def workload():
    return configs.exchange8()


@pytest.fixture(scope="module")
def oracle_sample(workload):
    """Oracle potentials and pair energies of the sampled pairs (its own nodes and inputs)."""
    mesh, orb = workload.meshes[0], workload.orbitals
    axes = oracle_axes(mesh)
    X, Y, Z = oracle_grid(axes)
    phi = orb.values(X, Y, Z)
    faces = oracle_faces(axes, lambda a, b, c: orb.pair_potentials(a.reshape(-1), b.reshape(-1), c.reshape(-1)))
    F = fdm.FDM(axes)
    out = {}
    for i, j in SAMPLE:
        # the oracle's exchange on the two orbitals i, j: pairs (i,i), (i,j), (j,j)
        qs = [ox.pair_index(a, b, orb.norb) for a, b in ((i, i), (i, j), (j, j))]
        fp = [[faces[f][q].reshape(axes[2].N if f < 4 else axes[1].N, -1) for f in range(6)] for q in qs]
        v, _, K, _ = ox.exchange(axes, [phi[i], phi[j]], fp, F.solve)
        for q, vq, Kq in zip(qs, v, K):
            out[q] = (vq, Kq)
    return axes, out


def _solve(gpu_lib, workload, rtol, precision="fp32_ir", learned=True):
    mesh, orb = workload.meshes[0], workload.orbitals
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=workload.n_levels, rtol=rtol,
                          precision=precision)
    assert ctx.opts.lanes == 2 and ctx.opts.use_graph == 1
    net = None
    if learned:
        net = gpu_lib.Net(4, 32, 125, 27)
        net.load(WEIGHTS)
        ctx.attach_guess(net)
    xyz, fxyz = ctx.mesh_coords(0)
    phi = _t(orb.values(xyz[0], xyz[1], xyz[2]).reshape(-1))
    g = _t(orb.pair_potentials(fxyz[0], fxyz[1], fxyz[2]).reshape(-1))
    ctx.exchange(phi, g)                          # warm: the timed configuration replays graphs
    W, K, EX, st, v = ctx.exchange(phi, g, keep_potentials=True)
    npairs = orb.norb * (orb.norb + 1) // 2
    return K.cpu().numpy(), EX, st, v.cpu().numpy().reshape(npairs, -1), net


def _check(gpu_lib, workload, oracle_sample, rtol, pot_bar, energy_bar, precision="fp32_ir", learned=True):
    mesh, orb = workload.meshes[0], workload.orbitals
    K, EX, st, v, _ = _solve(gpu_lib, workload, rtol, precision, learned)
    assert all(s["status"] == 0 and s["rel_residual"] <= rtol for s in st)
    assert all(s["guess_used"] in (0, 1) for s in st)
    assert any(s["guess_used"] for s in st) if learned else not any(s["guess_used"] for s in st)
    # E_x is the ordered-pair sum of the returned pair energies
    n = orb.norb
    ex = sum(K[ox.pair_index(i, i, n)] for i in range(n)) + \
        2.0 * sum(K[ox.pair_index(i, j, n)] for i in range(n) for j in range(i + 1, n))
    assert abs(EX - ex) <= 1e-12 * abs(ex)
    axes, ref = oracle_sample
    for q, (vq, Kq) in ref.items():
        assert rel_l2_M(axes, mesh, v[q], vq) <= pot_bar, q
        assert abs(K[q] - Kq) <= energy_bar, q


def test_exchange8_parity_tolerance_bench_configuration(gpu_lib, workload, oracle_sample):
    _check(gpu_lib, workload, oracle_sample, PARITY_RTOL_FP32, POT_BAR, ENERGY_BAR)


def test_exchange8_parity_tolerance_fp64(gpu_lib, workload, oracle_sample):
    """The plain FP64 solver (no guess) meets both bars at the oracle's parity tolerance."""
    _check(gpu_lib, workload, oracle_sample, PARITY_RTOL, POT_BAR, ENERGY_BAR, precision="fp64", learned=False)


def test_exchange8_bench_tolerance_bench_configuration(gpu_lib, workload, oracle_sample):
    _check(gpu_lib, workload, oracle_sample, workload.rtol, BENCH_POT_BAR, BENCH_ENERGY_BAR)


def test_trained_guess_saves_iterations_on_a_molecule_outside_its_training_set(gpu_lib, workload):
    """The benchmark molecule (seed 2) is not among the training molecules (seeds 10000+i):
    with the trained network every guess passes the guard and the mean iteration count at
    the benchmark tolerance drops by at least one against the same solver without it."""
    K_g, _, st_g, _, _ = _solve(gpu_lib, workload, workload.rtol)
    K_0, _, st_0, _, _ = _solve(gpu_lib, workload, workload.rtol, learned=False)
    assert all(s["guess_used"] == 1 for s in st_g) and not any(s["guess_used"] for s in st_0)
    it_g = np.mean([s["iters"] for s in st_g])
    it_0 = np.mean([s["iters"] for s in st_0])
    assert it_g <= it_0 - 1.0, (it_g, it_0)
    assert np.abs(K_g - K_0).max() <= BENCH_ENERGY_BAR


def test_large_mesh_five_levels_sampled_sources(gpu_lib):
    """The 32^3-element, p = 4 mesh with 5 levels (two mesh-coarsening levels below the degree
    steps), 16 Gaussian-sum sources in one call (two solver lanes), FP32 refinement with the
    guess network trained for this mesh: two sampled potentials against the oracle's exact
    solve at the parity tolerance."""
    from oracle import fdm
    from _cases import gpu_sample, oracle_density_problem
    wl = configs.scaled(32, 4, 16, seed=71, n_levels=5)
    mesh = wl.meshes[0]
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=5, rtol=PARITY_RTOL_FP32, precision="fp32_ir")
    assert ctx.opts.lanes == 2
    net = gpu_lib.Net(4, 32, 125, 27)
    net.load(WEIGHTS.replace("guess_16e_p4", "guess_32e_p4"))
    ctx.attach_guess(net)
    rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
    v, st = ctx.solve_batch(_t(np.concatenate(rho)), _t(np.concatenate(g)))
    assert all(s["status"] == 0 and s["rel_residual"] <= PARITY_RTOL_FP32 for s in st)
    v = v.cpu().numpy().reshape(16, -1)
    for k in (3, 12):      # one source of each lane
        axes, _, _, b = oracle_density_problem(mesh, wl.batch.densities[k])
        assert rel_l2_M(axes, mesh, v[k], fdm.FDM(axes).solve(b)) <= POT_BAR, k


def test_exchange16_largest_batch_bench_tolerance(gpu_lib):
    """The largest batch of the workloads: 16 orbitals, 136 pair densities on the 16^3, p = 4
    mesh in one call (two lanes of 68, FP32 refinement, trained guess) at the benchmark
    tolerance: sampled pairs against the oracle's exact solve, E_x from the returned energies."""
    wl = configs.exchange16()
    mesh, orb = wl.meshes[0], wl.orbitals
    K, EX, st, v, _ = _solve(gpu_lib, wl, wl.rtol)
    n = orb.norb
    assert len(st) == n * (n + 1) // 2 == 136
    assert all(s["status"] == 0 and s["rel_residual"] <= wl.rtol for s in st)
    ex = sum(K[ox.pair_index(i, i, n)] for i in range(n)) + \
        2.0 * sum(K[ox.pair_index(i, j, n)] for i in range(n) for j in range(i + 1, n))
    assert abs(EX - ex) <= 1e-12 * abs(ex)
    axes = oracle_axes(mesh)
    X, Y, Z = oracle_grid(axes)
    phi = orb.values(X, Y, Z)
    faces = oracle_faces(axes, lambda a, b, c: orb.pair_potentials(a.reshape(-1), b.reshape(-1), c.reshape(-1)))
    i, j = 2, 13
    qs = [ox.pair_index(a, b, n) for a, b in ((i, i), (i, j), (j, j))]
    fp = [[faces[f][q].reshape(axes[2].N if f < 4 else axes[1].N, -1) for f in range(6)] for q in qs]
    v_o, _, K_o, _ = ox.exchange(axes, [phi[i], phi[j]], fp, fdm.FDM(axes).solve)
    for q, vq, Kq in zip(qs, v_o, K_o):
        assert rel_l2_M(axes, mesh, v[q], vq) <= BENCH_POT_BAR, q
        assert abs(K[q] - Kq) <= BENCH_ENERGY_BAR, q
