"""GPU parity of the learned-guess network against the oracle U-Net.

Forward and backward of the HIP kernels (FP32) against oracle/convnet.py
(FP64) with the same parameters, one training step (A-norm loss through the
library's operator, gradient, Adam) against the oracle, and the guess path
of the solver (a guess never changes the converged answer; the guard keeps
only guesses whose residual is below ||b||).
"""
import numpy as np
import pytest

from oracle import convnet, layout, sipdg
from workloads import configs

from _cases import PARITY_RTOL_FP32, POT_BAR, gpu_sample, oracle_density_problem, rel_l2_M

pytestmark = pytest.mark.gpu


def _t(a, dtype=np.float64):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).cuda()


@pytest.mark.parametrize("levels,E", [(3, (6, 4, 5)), (1, (3, 3, 2)), (4, (8, 8, 8))])
def test_forward_backward_match_oracle(gpu_lib, levels, E):
    C, cin = 8, 27
    specs = convnet.layer_specs(levels, C, cin, cin)
    n = convnet.param_count(specs)
    rng = np.random.default_rng(levels)
    params = (0.3 * rng.standard_normal(n)).astype(np.float32)
    net = gpu_lib.Net(levels, C, cin, cin)
    assert net.num_params == n
    net.set_params(params)
    assert np.array_equal(net.get_params(), params)
    B = 2
    x = rng.standard_normal((B, E[2], E[1], E[0], cin)).astype(np.float32)
    y_ref, cache = convnet.forward(params.astype(np.float64), specs, levels, x.astype(np.float64))
    # matrix-core path: BF16 operands (8-bit mantissa), FP32 accumulation
    net.set_bf16(True)
    yb = net.forward(_t(x, np.float32), E, B).cpu().numpy().reshape(B, E[2], E[1], E[0], cin)
    assert np.abs(yb - y_ref).max() <= 3e-2 * np.abs(y_ref).max()
    assert np.abs(yb - y_ref).max() >= 1e-7 * np.abs(y_ref).max()   # it really ran in BF16
    # FP32 vector path: exact up to FP32 rounding
    net.set_bf16(False)
    y = net.forward(_t(x, np.float32), E, B).cpu().numpy().reshape(B, E[2], E[1], E[0], cin)
    assert np.abs(y - y_ref).max() <= 1e-4 * np.abs(y_ref).max()
    dy = rng.standard_normal(y.shape).astype(np.float32)
    g = net.backward(_t(dy, np.float32)).cpu().numpy()
    g_ref = convnet.backward(params.astype(np.float64), specs, levels, cache, dy.astype(np.float64))
    assert np.abs(g - g_ref).max() <= 2e-4 * np.abs(g_ref).max()


@pytest.mark.parametrize("levels,E,C,cin", [(3, (6, 4, 5), 8, 27), (4, (8, 8, 8), 32, 125), (2, (5, 3, 4), 16, 64)])
def test_inference_with_bf16_activations(gpu_lib, levels, E, C, cin):
    """The guess's forward stores every activation in BF16 (half the bytes of FP32).  The
    matrix-core convolutions round their FP32 operands to BF16 (nearest even) on load, so rounding
    them once when they are stored gives the same operands: the output equals the FP32-activation
    matrix-core forward bit for bit, and stays within the BF16 bound of the oracle network."""
    specs = convnet.layer_specs(levels, C, cin, 27)
    n = convnet.param_count(specs)
    rng = np.random.default_rng(100 + levels)
    params = (0.3 * rng.standard_normal(n) / np.sqrt(C)).astype(np.float32)
    net = gpu_lib.Net(levels, C, cin, 27)
    net.set_params(params)
    net.set_bf16(True)
    B = 2
    x = rng.standard_normal((B, E[2], E[1], E[0], cin)).astype(np.float32)
    y16 = net.infer(_t(x, np.float32), E, B).cpu().numpy()
    yb = net.forward(_t(x, np.float32), E, B).cpu().numpy()
    assert np.array_equal(y16, yb)
    y_ref, _ = convnet.forward(params.astype(np.float64), specs, levels, x.astype(np.float64))
    y16 = y16.reshape(y_ref.shape)
    assert np.abs(y16 - y_ref).max() <= 3e-2 * np.abs(y_ref).max()


def _continuize_1d(E, n):
    """1D averaging of the two copies of every node shared by neighbouring elements."""
    N = E * n
    Cm = np.eye(N)
    for e in range(E - 1):
        a, b = e * n + n - 1, (e + 1) * n
        Cm[a, a] = Cm[a, b] = Cm[b, a] = Cm[b, b] = 0.5
    return Cm


@pytest.mark.parametrize("mode", [0, 2])
def test_train_step_matches_oracle(gpu_lib, mode):
    import torch
    from oracle import mg
    mesh = configs.Mesh((4, 4, 4), 2, (-2.0,) * 3, (2.0,) * 3)
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)])
    levels, C, cin, cout = 2, 8, 27, 8       # level 1 of a p=2 mesh is p=1: 8 nodes per element
    specs = convnet.layer_specs(levels, C, cin, cout)
    n = convnet.param_count(specs)
    rng = np.random.default_rng(7)
    params = (0.2 * rng.standard_normal(n)).astype(np.float32)
    net = gpu_lib.Net(levels, C, cin, cout)
    net.set_bf16(False)
    net.set_params(params)
    B = 2
    nd = ctx.info[0]["n_dofs"]
    x = rng.standard_normal((B, nd)).astype(np.float32)
    t = rng.standard_normal((B, nd))
    lr = 1e-3
    loss = net.train_step(ctx, _t(x, np.float32), _t(t), B, lr, mode=mode)
    # oracle: output map (continuous projection, then interpolation to degree 2),
    # the same loss, gradient and Adam step
    H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi)
    axes = H.levels[0].axes
    Cx = _continuize_1d(4, 2)
    xs = x.reshape(B, 4, 4, 4, cin).astype(np.float64)
    y, cache = convnet.forward(params.astype(np.float64), specs, levels, xs)
    y = y.reshape(B, -1)
    dy = np.zeros_like(y)
    L = 0.0
    for b in range(B):
        yg = layout.to_global(y[b], mesh.E, 2)
        yc = np.einsum("Zc,Yb,Xa,cba->ZYX", Cx, Cx, Cx, yg)
        x0 = H.prolong(0, yc)
        e = x0 - layout.to_global(t[b], mesh.E, 3)
        Ae = sipdg.apply(axes, e)
        tg = layout.to_global(t[b], mesh.E, 3)
        tAt = float(np.sum(tg * sipdg.apply(axes, tg)))
        L += float(np.sum(e * Ae)) / tAt / B
        gx = 2.0 * (Ae if mode == 0 else H.vcycle(Ae)) / (tAt * B)
        gy = np.einsum("Zc,Yb,Xa,cba->ZYX", Cx, Cx, Cx, H.restrict(0, gx))
        dy[b] = layout.to_element_major(gy, mesh.E, 2)
    assert abs(loss - L) <= 1e-5 * abs(L)
    g = convnet.backward(params.astype(np.float64), specs, levels, cache, dy.reshape(B, 4, 4, 4, cout))
    p1, _, _ = convnet.adam(params.astype(np.float64), g, np.zeros(n), np.zeros(n), 1, lr)
    got = net.get_params()
    moved = np.abs(p1 - params) > 1e-5   # Adam's first step is lr * sign(g) where |g| is not tiny
    assert np.abs(got - p1)[moved].max() <= 1e-6 + 1e-3 * lr


def test_guess_path_keeps_converged_answer_and_guard(gpu_lib):
    import torch
    wl = configs.scaled(8, 4, 3, seed=51)
    mesh = wl.meshes[0]
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], rtol=1e-11)
    rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
    rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
    net = gpu_lib.Net(3, 8, 125, 27)
    rng = np.random.default_rng(3)
    net.set_params((0.05 * rng.standard_normal(net.num_params)).astype(np.float32))
    ctx.attach_guess(net)
    v, st = ctx.solve_batch(rho, g)
    v = v.cpu().numpy().reshape(3, -1)
    for k, d in enumerate(wl.batch.densities):
        axes, _, _, b = oracle_density_problem(mesh, d)
        from oracle import fdm
        assert rel_l2_M(axes, mesh, v[k], fdm.FDM(axes).solve(b)) <= POT_BAR
        assert st[k]["guess_used"] in (0, 1) and st[k]["status"] == 0
    # a zero network gives v0 = 0, whose residual equals ||b||: the guard rejects it
    net.set_params(np.zeros(net.num_params, dtype=np.float32))
    _, st0 = ctx.solve_batch(rho, g)
    assert all(s["guess_used"] == 0 for s in st0)
    ctx.attach_guess(None)
    _, st1 = ctx.solve_batch(rho, g)
    assert [s["iters"] for s in st1] == [s["iters"] for s in st0]


def test_training_reduces_loss_and_save_load_roundtrip(gpu_lib, tmp_path):
    import torch
    wl = configs.scaled(8, 4, 8, seed=61)
    mesh = wl.meshes[0]
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], rtol=1e-8)
    rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
    rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
    v, _ = ctx.solve_batch(rho, g)
    net = gpu_lib.Net(3, 16, 125, 27)
    rng = np.random.default_rng(9)
    net.set_params(_init(net, rng))
    B = 8
    nd = ctx.info[0]["n_dofs"]
    x, s = net.prepare_input(rho, B, nd)
    t = v / s.repeat_interleave(nd)
    losses = [net.train_step(ctx, x, t, B, 2e-3, mode=2) for _ in range(60)]
    assert losses[-1] < 0.5 * losses[0]
    path = tmp_path / "net.bin"
    net.save(path)
    net2 = gpu_lib.Net(3, 16, 125, 27)
    net2.load(path)
    assert np.array_equal(net2.get_params(), net.get_params())


def _init(net, rng):
    """He-style initial weights for the layer sizes of the architecture (biases zero)."""
    specs = convnet.layer_specs(net.levels, net.channels, net.in_channels, net.out_channels)
    out = []
    for name, k, s, ci, co in specs:
        fan_in = k ** 3 * ci
        scale = np.sqrt(2.0 / fan_in) if name != "out" else np.sqrt(1.0 / fan_in)
        out += [scale * rng.standard_normal(k ** 3 * ci * co), np.zeros(co)]
    return np.concatenate(out).astype(np.float32)


@pytest.mark.parametrize("precision", ["fp32_ir", "fp64"])
def test_guard_on_device_with_zero_source_in_the_batch(gpu_lib, precision):
    """The guard is taken from the solve's first FP64 residual.  A zero source gets a
    nonzero guess from the network's biases (its residual exceeds ||b|| = 0): it is
    dropped and the solution is exactly zero; the other sources converge to the exact
    solve whichever way their guess was judged, and a dropped guess leaves the iteration
    path of a solve without a guess."""
    from oracle import fdm
    wl = configs.scaled(8, 4, 3, seed=52)
    mesh = wl.meshes[0]
    ctx = gpu_lib.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], rtol=1e-11, precision=precision)
    rho, g = zip(*[gpu_sample(ctx, 0, d) for d in wl.batch.densities])
    nd, nf = len(rho[0]), len(g[0])
    rho = list(rho[:2]) + [np.zeros(nd)] + list(rho[2:])
    g = list(g[:2]) + [np.zeros(nf)] + list(g[2:])
    rho, g = _t(np.concatenate(rho)), _t(np.concatenate(g))
    net = gpu_lib.Net(3, 8, 125, 27)
    rng = np.random.default_rng(4)
    net.set_params((0.05 * rng.standard_normal(net.num_params)).astype(np.float32))
    ctx.attach_guess(net)
    v, st = ctx.solve_batch(rho, g)
    v = v.cpu().numpy().reshape(4, -1)
    assert st[2]["guess_used"] == 0 and st[2]["status"] == 0 and not np.any(v[2])
    for k, d in zip((0, 1, 3), wl.batch.densities):
        axes, _, _, b = oracle_density_problem(mesh, d)
        assert rel_l2_M(axes, mesh, v[k], fdm.FDM(axes).solve(b)) <= POT_BAR
        assert st[k]["guess_used"] in (0, 1) and st[k]["status"] == 0
    net.set_params(np.zeros(net.num_params, dtype=np.float32))   # v0 = 0: dropped everywhere
    v0, st0 = ctx.solve_batch(rho, g)
    assert all(s["guess_used"] == 0 for s in st0)
    ctx.attach_guess(None)
    v1, st1 = ctx.solve_batch(rho, g)
    assert [s["iters"] for s in st1] == [s["iters"] for s in st0]
    assert [s["outer_iters"] for s in st1] == [s["outer_iters"] for s in st0]


def test_guess_in_a_batch_over_two_meshes(gpu_lib):
    """A learned guess for an interleaved batch over two p = 4 meshes (the network runs once
    per mesh inside the call): every potential against the exact solve, and bitwise equal to
    one call per mesh with the same network."""
    import torch
    from oracle import fdm
    m0 = configs.Mesh((4, 4, 4), 4, (-2.0,) * 3, (2.0,) * 3)
    m1 = configs.Mesh((6, 4, 6), 4, (-3.0, -2.0, -3.0), (3.0, 2.0, 3.0))
    dens = configs.scaled(4, 4, 5, seed=53).batch.densities
    ctx = gpu_lib.Context([(m.E, m.p, m.lo, m.hi) for m in (m0, m1)], rtol=PARITY_RTOL_FP32, precision="fp32_ir")
    net = gpu_lib.Net(3, 8, 125, 27)
    net.set_params((0.05 * np.random.default_rng(6).standard_normal(net.num_params)).astype(np.float32))
    ctx.attach_guess(net)
    ids = [1, 0, 1, 0, 1]
    samples = [gpu_sample(ctx, mid, dens[k]) for k, mid in enumerate(ids)]
    v, st = ctx.solve_batch(_t(np.concatenate([s[0] for s in samples])), _t(np.concatenate([s[1] for s in samples])),
                            mesh_ids=ids)
    v = v.cpu().numpy()
    off, parts = 0, {0: [], 1: []}
    for k, mid in enumerate(ids):
        mesh = (m0, m1)[mid]
        n = ctx.info[mid]["n_dofs"]
        axes, _, _, b = oracle_density_problem(mesh, dens[k])
        assert rel_l2_M(axes, mesh, v[off:off + n], fdm.FDM(axes).solve(b)) <= POT_BAR
        assert st[k]["status"] == 0 and st[k]["guess_used"] in (0, 1)
        parts[mid].append((k, off, n))
        off += n
    for mid, ks in parts.items():
        r = _t(np.concatenate([samples[k][0] for k, _, _ in ks]))
        g = _t(np.concatenate([samples[k][1] for k, _, _ in ks]))
        vm, stm = ctx.solve_batch(r, g, mesh_ids=[mid] * len(ks))
        vm = vm.cpu().numpy()
        o2 = 0
        for (k, o, n), s in zip(ks, stm):
            assert np.array_equal(vm[o2:o2 + n], v[o:o + n])
            assert s["iters"] == st[k]["iters"] and s["guess_used"] == st[k]["guess_used"]
            o2 += n
