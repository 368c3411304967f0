#!/usr/bin/env python
"""Benchmark: Poisson right-hand sides solved per second, learned + mixed precision vs plain FP64 MG-PCG.

Default workload ``heldout32``: 128 held-out pair densities rho_ij = phi_i phi_j
(the first 128 pairs, in pair order, of four molecules of 16-32 atoms with 8
Loewdin orbitals each, seeds 90000-90003, none of them in the guess network's
training set) on the 32x32x32-element, degree-4 auxiliary mesh of [-16,16]^3
(4,096,000 nodes per right-hand side), closed-form Dirichlet data, 5-level
hp-multigrid PCG.  One step = one dg_poisson_solve_batch call over the 128
right-hand sides (right-hand-side assembly, learned guess, batched solve),
inputs resident in HBM.

Operating point: every arm stops at the same FP64 relative residual, 1e-11,
the loosest power of ten at which the FP64 solver meets the parity bars (1e-8
relative L2 on potentials, 1e-10 Ha on pair and exchange energies) on every
exchange pair; every potential of every arm is compared with the oracle's
exact solve (cpu leg).  The same comparison at the metric's residual 1e-8
is reported beside it (``at_metric_residual``).

Arms: ``fp32_pc+learned`` (the headline ``value``: FP64 CG preconditioned by
the FP32 V-cycle, trained initial guess), ``fp32_pc``, ``fp64+learned``,
``fp64`` (plain FP64 MG-PCG) and ``fp32_pc+untrained`` (the same network with
random weights, a control).

Prints one JSON line.  --gpus above 1 is refused: the measurement is of one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector
METRIC = "Poisson RHS solved/sec at 1e-8 rel. residual: learned+mixed vs plain FP64 MG-PCG"
OPERATING_RTOL = 1e-11
POT_BAR, ENERGY_BAR = 1e-8, 1e-10
HELDOUT_RHS = 128
# arithmetic each precision mode computes in (the "dtype" field of the JSON line)
DTYPE_OF = {"fp64": "f64", "fp32_ir": "f64 refinement + f32 inner PCG", "fp32_pc": "f64 CG + f32 V-cycle",
            "bf16_pc": "f64 flexible CG + f32 V-cycle, bf16 matrix-core x/y contractions in level-0 smoothing",
            "bf16f_pc": "f64 CG (f32-stored search direction) + f32-arithmetic V-cycle with bf16 fields on its two finest levels"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3,
                    help="untimed steps first: the first calls capture the PCG graphs and learn how many "
                         "iteration blocks to replay before a host check")
    ap.add_argument("--config", default="heldout32",
                    choices=["heldout32", "exchange8", "exchange16", "uneven", "single", "quadrature", "consumers",
                             "octree"],
                    help="heldout32: 128 held-out pair densities on 32^3 elements p=4 (default); "
                         "exchange8/16: the exchange step of 8/16 orbitals on 16^3 elements p=4; "
                         "uneven: 256 densities over 8^3, 12^3 and 16^3 meshes in one interleaved batch; "
                         "single: one two-Gaussian density on 4^3 elements p=3 (latency-bound); "
                         "quadrature: the exchange8 step with its Dirichlet data computed by quadrature; "
                         "consumers: Hartree/exchange actions projected on a 256-function basis and the "
                         "compressed exchange on the exchange8 mesh")
    ap.add_argument("--arms", default="bf16f_pc+learned,fp32_pc+learned,fp32_pc,fp64+learned,fp64,bf16f_pc+untrained",
                    help="precision fp32_pc, bf16f_pc, bf16_pc, fp32_ir or fp64, optionally +learned (trained guess) or "
                         "+untrained (the same network with random weights, a control); the first is the headline")
    ap.add_argument("--rtol", type=float, default=OPERATING_RTOL, help="FP64 relative residual of every arm")
    ap.add_argument("--metric-rtol", type=float, default=1e-8,
                    help="second comparison at this residual (0: skip)")
    ap.add_argument("--metric-arms", default="bf16f_pc+learned,fp64")
    ap.add_argument("--weights", default=None,
                    help="guess network (default: the weights trained for the workload's mesh)")
    ap.add_argument("--lanes", type=int, default=2, choices=[1, 2, 3, 4],
                    help="solver lanes per mesh: 2 solves a batch as two concurrent halves")
    ap.add_argument("--cheb-degree", type=int, default=None, help="smoothing steps (default: the library's)")
    ap.add_argument("--cheb-ratio", type=float, default=None, help="smoothing interval ratio (default: the library's)")
    ap.add_argument("--cheb-degree-h", type=int, default=None,
                    help="smoothing steps on the degree-1 coarse levels (default: the library's)")
    ap.add_argument("--inner-rtol", type=float, default=None, help="inner FP32 tolerance of fp32_ir")
    ap.add_argument("--fused", type=int, default=None, choices=[0, 1, 2],
                    help="FP64 small-mesh solve in one launch: 1 one work-group per RHS, 2 group-persistent")
    ap.add_argument("--fused-wgs", type=int, default=None, help="work-groups per RHS of the group-persistent solve")
    ap.add_argument("--learned-cgc", type=int, default=None,
                    help="PCG iterations that take the learned coarse-grid correction (FP64 arms with +learned, "
                         "--lanes 1)")
    ap.add_argument("--node-family", default=None, choices=["gll", "gl"],
                    help="element nodes: gll (default) or gl (Gauss-Legendre: general operator kernels, no learned "
                         "guess; the oracle legs are skipped)")
    ap.add_argument("--profile-solves", type=int, default=2,
                    help="eager solves of the headline arm that time the dominant kernel (0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=1, help="pair solves timed on the oracle (0: skip)")
    ap.add_argument("--check", type=int, default=-1,
                    help="right-hand sides compared with the oracle's exact solve (-1: all, 0: none)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run 3 device-to-device copies of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    args.solver_opts = {k: v for k, v in (("cheb_degree", args.cheb_degree), ("cheb_ratio", args.cheb_ratio),
                                          ("cheb_degree_h", args.cheb_degree_h), ("inner_rtol", args.inner_rtol),
                                          ("fused", args.fused), ("fused_wgs", args.fused_wgs),
                                          ("node_family", args.node_family), ("learned_cgc", args.learned_cgc))
                        if v is not None}
    if args.node_family == "gl":
        # the CPU legs compare with the oracle's Gauss-Lobatto solve; the GL parity lives in the tests
        args.check, args.cpu_sample, args.profile_solves, args.metric_rtol = 0, 0, 0, 0
    return args


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is measured here; run with --gpus 1"}))
        sys.exit(2)
    import torch

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.config == "uneven":
        return main_uneven(args)
    if args.config == "single":
        return main_single(args)
    if args.config == "quadrature":
        return main_quadrature(args)
    if args.config == "consumers":
        return main_consumers(args)
    if args.config == "octree":
        return main_octree(args)
    return main_pairs(args)


# ---------------------------------------------------------------------------
# pair-density workloads: heldout32 (solve_batch) and exchange8/16 (exchange step)

class PairWorkload:
    """Molecules and the pairs taken from each: [(orbitals, first pair, count)], one mesh."""

    def __init__(self, name, mesh, n_levels, mols, exchange, weights):
        self.name, self.mesh, self.n_levels, self.mols = name, mesh, n_levels, mols
        self.exchange = exchange          # True: one dg_exchange_apply call per step (one molecule)
        self.weights = weights
        self.nrhs = sum(c for _, _, c in mols)


def pair_workload(name):
    from workloads import configs
    wdir = os.path.join(ROOT, "paper_2510_21213_amd", "weights")
    if name == "heldout32":
        mols, left, m = [], HELDOUT_RHS, 0
        while left > 0:
            wl = configs.large_molecule(m, held_out=True)
            n = min(left, len(wl.orbitals.pairs()))
            mols.append((wl.orbitals, 0, n))
            left -= n
            m += 1
        return PairWorkload(name, wl.meshes[0], wl.n_levels, mols, False, os.path.join(wdir, "guess_32e_p4.bin"))
    wl = configs.exchange8() if name == "exchange8" else configs.exchange16()
    return PairWorkload(name, wl.meshes[0], wl.n_levels, [(wl.orbitals, 0, len(wl.orbitals.pairs()))], True,
                        os.path.join(wdir, "guess_16e_p4.bin"))


def gpu_inputs(W, ctx):
    """Orbitals, pair densities and Dirichlet data at the library's nodes (device tensors)."""
    import torch

    from paper_2510_21213_amd import binding
    xyz, fxyz = ctx.mesh_coords(0)
    phis, rhos, gs = [], [], []
    for orb, first, n in W.mols:
        phi = orb.values_torch(*xyz, device="cuda").reshape(-1).contiguous()
        phis.append(phi)
        rhos.append(binding.pair_densities(phi, orb.norb, first, n))
        gs.append(orb.pair_potentials_torch(*fxyz, device="cuda")[first:first + n].reshape(-1))
    return phis, torch.cat(rhos), torch.cat(gs).contiguous()


def make_ctx(W, prec, rtol, args, net_cache, learned, **kw):
    from paper_2510_21213_amd import binding
    opts = dict(n_levels=W.n_levels, rtol=rtol, precision=prec, lanes=args.lanes)
    opts.update(args.solver_opts)
    opts.update(kw)
    m = W.mesh
    ctx = binding.Context([(m.E, m.p, m.lo, m.hi)], **opts)
    if learned:
        if learned not in net_cache:
            net = binding.Net(4, 32, 125, 27)
            if learned == "learned":
                net.load(args.weights or W.weights)
            else:
                # control: the same architecture with random (He) weights, as in the training script
                import numpy as np

                from paper_2510_21213_amd.train_guess import he_init
                net.set_params(he_init(net, np.random.default_rng(12345)))
            net_cache[learned] = net
        ctx.attach_guess(net_cache[learned])
    return ctx


def run_arm(W, arm, rtol, args, inputs, net_cache):
    """Warm-up, then the timed steps of one arm; returns its record and the last potentials."""
    import numpy as np
    import torch
    prec, _, learned = arm.partition("+")
    if learned not in ("", "learned", "untrained"):
        raise SystemExit(f"unknown arm {arm}")
    ctx = make_ctx(W, prec, rtol, args, net_cache, learned)
    phis, rho, g = inputs

    def step():
        if W.exchange:
            Wk, K, EX, st, _ = ctx.exchange(phis[0], g)
            return st, EX
        v, st = ctx.solve_batch(rho, g)
        return st, None

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    step_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st, EX = step()                      # returns after its stream is synchronised
        step_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the potentials of the same solve, kept for the comparison with the exact solve
    if W.exchange:
        _, K, EX, st, v = ctx.exchange(phis[0], g, keep_potentials=True)
    else:
        v, st = ctx.solve_batch(rho, g)
    ctx.close()
    iters = [s["iters"] for s in st]
    rec = {
        "value": W.nrhs * args.steps / dt,
        "ms_per_step": 1e3 * dt / args.steps,
        "ms_per_step_median": 1e3 * float(np.median(step_s)),
        "rtol": rtol,
        "iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
        "outer_mean": float(np.mean([s["outer_iters"] for s in st])),
        "max_rel_residual": float(max(s["rel_residual"] for s in st)),
        "guess_used": float(np.mean([s["guess_used"] for s in st])),
        "status_ok": all(s["status"] == 0 for s in st),
    }
    if EX is not None:
        rec["E_x"] = EX
    log(f"{arm} rtol {rtol:g}: {rec['value']:.1f} RHS/s, {rec['iters_mean']:.2f} iterations, "
        f"guess used {rec['guess_used']:.2f}")
    return rec, v


def main_pairs(args):
    import torch
    W = pair_workload(args.config)
    arms = [a for a in args.arms.split(",") if a]
    net_cache = {}
    log(f"workload {W.name}: {W.nrhs} right-hand sides")
    probe = make_ctx(W, "fp64", args.rtol, args, net_cache, "")
    info = probe.info[0]
    inputs = gpu_inputs(W, probe)
    probe.close()
    results, pots = {}, {}
    for arm in arms:
        results[arm], pots[arm] = run_arm(W, arm, args.rtol, args, inputs, net_cache)
    metric_pass = None
    if args.metric_rtol > 0:
        metric_pass = {"rtol": args.metric_rtol, "arms": {}}
        for arm in [a for a in args.metric_arms.split(",") if a]:
            rec, pots[f"{arm}@{args.metric_rtol:g}"] = run_arm(W, arm, args.metric_rtol, args, inputs, net_cache)
            metric_pass["arms"][arm] = rec
        ma = list(metric_pass["arms"])
        if "fp64" in metric_pass["arms"] and len(ma) > 1:
            metric_pass["speedup_vs_plain_fp64"] = metric_pass["arms"][ma[0]]["value"] / metric_pass["arms"]["fp64"]["value"]
    head_arm = arms[0]
    roofline = measure_roofline(W, head_arm, args, inputs, net_cache) if args.profile_solves > 0 else None
    torch.cuda.synchronize()
    cpu = check = None
    if args.cpu_sample > 0 or args.check != 0:
        cpu, check = cpu_leg_pairs(args, W, pots)
    head = results[head_arm]
    prec = head_arm.partition("+")[0]
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_median": head["ms_per_step_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_OF[prec],
        "data": "synthetic",
        "config": {"workload": workload_name(W, info, args.rtol), "arm": head_arm, "rtol": args.rtol,
                   "equal_accuracy": "every arm stops at the same FP64 relative residual; cpu leg checks "
                                     "every potential against the exact solve",
                   "learned_guess": "learned" in head_arm, "parallelism": "single GPU", "solver_lanes": args.lanes},
        "arms": results,
        "speedup_vs_plain_fp64": (head["value"] / results["fp64"]["value"]) if "fp64" in results else None,
        "at_metric_residual": metric_pass,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "check_vs_exact": check,
    }
    print(json.dumps(line))


def workload_name(W, info, rtol):
    m = W.mesh
    if W.name == "heldout32":
        return (f"heldout32: {W.nrhs} held-out pair-density RHS (first {W.nrhs} pairs of {len(W.mols)} molecules of "
                f"16-32 atoms, 8 orbitals each), {m.E[0]}^3 elements p={m.p} ({info['n_dofs']} DOFs/RHS), "
                f"{W.n_levels}-level MG-PCG to FP64 relative residual {rtol:g}")
    return (f"{W.name}: exchange step, {W.nrhs} pair-density RHS, {m.E[0]}^3 elements p={m.p} "
            f"({info['n_dofs']} DOFs/RHS), {W.n_levels}-level MG-PCG to FP64 relative residual {rtol:g}")


def measure_roofline(W, arm, args, inputs, net_cache):
    """The dominant kernel (the finest-level Chebyshev smoothing step) timed by HIP events on the
    solver's stream, in a pass of its own after the timed steps: events recorded inside captured
    graphs cannot be timed on this runtime, so the same solves run on eager launches on one lane,
    where every launch has the whole batch to itself."""
    prec, _, learned = arm.partition("+")
    ctx = make_ctx(W, prec, args.rtol, args, net_cache, learned, use_graph=0, lanes=1)
    phis, rho, g = inputs

    def solve():
        if W.exchange:
            ctx.exchange(phis[0], g)
        else:
            ctx.solve_batch(rho, g)

    solve()
    ctx.profile(True)
    for _ in range(args.profile_solves):
        solve()
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    if prof["launches"] <= 0 or prof["seconds"] <= 0:
        return None
    achieved = prof["bytes"] / prof["seconds"] / 1e9
    copy_gbs = copy_bandwidth()
    fp = "float" if prec != "fp64" else "double"
    if prec == "bf16f_pc":
        fp = "float, ..., __bf16"  # FP32 arithmetic on BF16 fields
    traffic_file = {"heldout32": "cheb_step_heldout32.md", "exchange8": "cheb_step_exchange8.md"}.get(W.name)
    return {
        "bound": "hbm",
        "kernel": f"finest-level Chebyshev smoothing step (k_slab<{fp},5,...,BM_CHEB/BM_CHEBDOT>)",
        "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
        "traffic": measured_traffic(traffic_file, "dg_kernels.hip", prec) if traffic_file else None,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, copy-calibrated)",
        "valu_busy": measured_traffic(traffic_file, "dg_kernels.hip", prec, "valu_busy") if traffic_file else None,
        "valu_busy_note": "fraction of the isolated launch the vector ALUs issue (SQ_ACTIVE_INST_VALU x 4 cycles / "
                          "1024 SIMDs at 2.4 GHz, committed counter summary): the step is bound by issue and "
                          "barrier latency when this is high while frac is low",
        "algorithmic_bytes_per_launch": prof["bytes"] / prof["launches"],
        "bytes_counted": "per step and right-hand side still iterating: read z, f (and z_prev after the first "
                         "step), write z': 3 or 4 fields of the finest level, at the size of their storage type",
        "avg_launch_us": 1e6 * prof["seconds"] / prof["launches"],
        "launches": prof["launches"],
        "timing_source": "HIP events on the solver's stream around each launch, eager launches on one lane, "
                         "a separate pass after the timed steps",
        "copy_gbs": copy_gbs,
        "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
        "copy_note": "device-to-device copy of 2 GiB (read + write bytes over its duration), timed in the same "
                     "process: the streaming rate this GPU reaches with the runtime's own copy kernel",
    }


def copy_bandwidth(mib=2048, reps=5):
    """Bytes read plus written per second by a device-to-device copy of mib MiB (best of reps), GB/s."""
    import torch

    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        dt = e0.elapsed_time(e1) * 1e-3
        best = dt if best is None else min(best, dt)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / best / 1e9


def measured_traffic(profile_name, kernel_source, prec, key="traffic_bytes_per_launch"):
    """HBM bytes per launch (or another field of the record, `key`) from the committed rocprofv3
    counter summary, or None.

    None when the summary is missing, was taken for another arithmetic, or on a different kernel source.
    """
    import hashlib
    path = os.path.join(ROOT, "profiles", profile_name)
    src = os.path.join(ROOT, "paper_2510_21213_amd", "csrc", kernel_source)
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        if line.startswith("traffic-json:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel_source_sha256_16") == digest and rec.get("precision", prec) == prec:
                return rec.get(key)
    return None


def _host():
    """The host the oracle ran on: logical CPUs and the CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"host_cpus": os.cpu_count(), "host_cpu_model": model}


def _threads():
    from threadpoolctl import threadpool_info
    return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])


def cpu_leg_pairs(args, W, pots):
    """Oracle timing on the host cores (a bounded sample), and every kept GPU potential against
    the oracle's exact solve (fast diagonalisation) of the same pair problem at the oracle's own
    nodes, with its pair energy K_ij = sum M rho v."""
    import numpy as np

    from oracle import exchange as ox
    from oracle import fdm, layout, mg, pcg, sipdg
    mesh = W.mesh
    axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
    X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
    fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
    Mw = sipdg.mass(axes)
    F = fdm.FDM(axes)
    t_in = time.perf_counter()

    def problems():
        """(rhs index, rho, b) of every pair, molecule by molecule (closed forms at the oracle's nodes)."""
        q = 0
        for m, (orb, first, n) in enumerate(W.mols):
            log(f"oracle inputs of molecule {m} ({time.perf_counter() - t_in:.0f} s into the cpu leg)")
            phi = orb.values_torch(X, Y, Z).numpy().reshape((orb.norb,) + X.shape)
            faces = [orb.pair_potentials_torch(fx[f], fy[f], fz[f])[first:first + n].numpy() for f in range(6)]
            pairs = orb.pairs()[first:first + n]
            for k, (i, j) in enumerate(pairs):
                rho = phi[i] * phi[j]
                fk = [faces[f][k].reshape(fx[f].shape) for f in range(6)]
                yield q, rho, sipdg.rhs(axes, rho, fk)
                q += 1

    cpu = None
    if args.cpu_sample > 0:
        H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi, n_levels=W.n_levels)
        sample = []
        for q, rho, b in problems():
            sample.append(b)
            if len(sample) >= args.cpu_sample:
                break
        t0 = time.perf_counter()
        its = []
        for b in sample:
            _, it, _, _ = pcg.solve(H, b, rtol=args.rtol)
            its.append(it)
        dt = time.perf_counter() - t0
        t1 = time.perf_counter()
        for b in sample:
            F.solve(b)
        dtf = time.perf_counter() - t1
        cpu = {"value": len(sample) / dt, "unit": "RHS/s", "cores": _threads(), "kind": "oracle", **_host(),
               "sample": f"the first {len(sample)} of the {W.nrhs} pair problems, oracle MG-PCG FP64 (NumPy) to "
                         f"{args.rtol:g}, iterations {its}, {dt:.1f} s; hierarchy set-up excluded",
               "exact_fdm_value": len(sample) / dtf}
        log(f"oracle MG-PCG {cpu['value']:.3f} RHS/s")
    check = None
    if args.check != 0:
        limit = W.nrhs if args.check < 0 else args.check
        import torch

        # the norms are taken on the GPU in the library's element-major order (the oracle's exact
        # solution, its source and the mass are reordered once per pair; no GPU result reaches the oracle)
        def em(a):
            return torch.as_tensor(layout.to_element_major(a, mesh.E, mesh.p + 1)).cuda()
        Mw_t = em(Mw)
        errs = {name: [] for name in pots}
        dks = {name: [] for name in pots}
        nd = int(np.prod(X.shape))
        for q, rho, b in problems():
            if q >= limit:
                break
            ref = F.solve(b)
            Kref = float(np.sum(Mw * rho * ref))
            ref_t, mrho_t = em(ref), Mw_t * em(rho)
            rn = float(torch.sum(Mw_t * ref_t * ref_t))
            for name, v in pots.items():
                got = v[q * nd:(q + 1) * nd]
                d = got - ref_t
                errs[name].append(float(torch.sqrt(torch.sum(Mw_t * d * d) / rn)))
                dks[name].append(abs(float(torch.sum(mrho_t * got)) - Kref))
        check = {}
        for name in pots:
            e, d = np.array(errs[name]), np.array(dks[name])
            check[name] = {"rhs_checked": int(len(e)), "max_rel_L2_err_vs_exact": float(e.max()),
                           "mean_rel_L2_err_vs_exact": float(e.mean()), "max_abs_dK_Ha": float(d.max()),
                           "meets_bars": bool(e.max() <= POT_BAR and d.max() <= ENERGY_BAR)}
            if W.exchange and len(e) == W.nrhs:
                orb = W.mols[0][0]
                n = orb.norb
                # E_x error from the pair-energy errors' signed sums is not recoverable from |dK|; report
                # the bound sum_i dK_ii + 2 sum_{i<j} dK_ij
                check[name]["E_x_err_bound_Ha"] = float(sum((1.0 if i == j else 2.0) * d[ox.pair_index(i, j, n)]
                                                            for i in range(n) for j in range(i, n)))
        log(f"exact check of {limit} right-hand sides done ({time.perf_counter() - t_in:.0f} s in the cpu leg)")
    return cpu, check


# ---------------------------------------------------------------------------
# uneven batch over three meshes

def main_uneven(args):
    """Uneven batch: one solve_batch call over right-hand sides of three meshes, interleaved
    in the caller's order, against one call per mesh (the same work without the overlap)."""
    import numpy as np
    import torch

    from paper_2510_21213_amd import binding
    from workloads import configs

    wl = configs.uneven()
    ids = [int(m) for m in wl.batch.mesh_ids]
    meshes = [(m.E, m.p, m.lo, m.hi) for m in wl.meshes]
    arms = [a for a in args.arms.split(",") if a and "learned" not in a and "untrained" not in a] or ["fp32_pc"]
    results, pots = {}, {}
    rho = g = None
    for arm in arms:
        ctx = binding.Context(meshes, n_levels=wl.n_levels, rtol=args.rtol, precision=arm, lanes=args.lanes,
                              **args.solver_opts)
        if rho is None:
            rs, gs = [], []
            coords = [ctx.mesh_coords(m) for m in range(len(meshes))]
            for k, mid in enumerate(ids):
                xyz, fxyz = coords[mid]
                d = wl.batch.densities[k]
                rs.append(d.density(xyz[0], xyz[1], xyz[2]))
                gs.append(d.potential(fxyz[0], fxyz[1], fxyz[2]))
            rho = torch.as_tensor(np.concatenate(rs)).cuda()
            g = torch.as_tensor(np.concatenate(gs)).cuda()
            offs = np.cumsum([0] + [ctx.info[m]["n_dofs"] for m in ids])
            foffs = np.cumsum([0] + [ctx.info[m]["n_face"] for m in ids])
            per = {m: [k for k in range(len(ids)) if ids[k] == m] for m in range(len(meshes))}
            rho_m = {m: torch.cat([rho[offs[k]:offs[k + 1]] for k in ks]) for m, ks in per.items()}
            g_m = {m: torch.cat([g[foffs[k]:foffs[k + 1]] for k in ks]) for m, ks in per.items()}
        for _ in range(args.warmup):
            ctx.solve_batch(rho, g, mesh_ids=ids)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            v, st = ctx.solve_batch(rho, g, mesh_ids=ids)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        # the same work as one call per mesh, one after the other
        for m in per:
            ctx.solve_batch(rho_m[m], g_m[m], mesh_ids=[m] * len(per[m]))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            for m in per:
                ctx.solve_batch(rho_m[m], g_m[m], mesh_ids=[m] * len(per[m]))
        torch.cuda.synchronize()
        dts = (time.perf_counter() - t1) / args.steps
        its = np.array([s["iters"] for s in st])
        results[arm] = {
            "value": len(ids) / dt, "ms_per_step": 1e3 * dt,
            "one_call_per_mesh_value": len(ids) / dts,
            "max_rel_residual": float(max(s["rel_residual"] for s in st)),
            "per_mesh": {f"{wl.meshes[m].E[0]}^3": {"rhs": len(ks), "iters_mean": float(its[ks].mean()),
                                                    "iters_min": int(its[ks].min()), "iters_max": int(its[ks].max())}
                         for m, ks in per.items()},
        }
        pots[arm] = v
        ctx.close()
    cpu = check = None
    if args.check != 0 or args.cpu_sample > 0:
        cpu, check = cpu_leg_uneven(args, wl, ids, offs, per, pots)
    head_arm = arms[0]
    head = results[head_arm]
    line = {
        "metric": "Poisson RHS solved/sec (uneven batch over three meshes)",
        "value": head["value"], "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE_OF[head_arm.split("+")[0]], "data": "synthetic",
        "config": {"workload": f"uneven: 256 Gaussian-sum densities over 8^3, 12^3, 16^3 elements p=4 "
                               f"(86/85/85, interleaved), 4-level MG-PCG to {args.rtol:g}", "arm": head_arm,
                   "parallelism": "single GPU"},
        "arms": results,
        "cpu_baseline": cpu,
        "check_vs_exact": check,
    }
    print(json.dumps(line))


def cpu_leg_uneven(args, wl, ids, offs, per, pots):
    """Oracle MG-PCG timing on one density of the largest mesh, and sampled potentials of every
    mesh against the oracle's exact solve."""
    import numpy as np

    from oracle import fdm, layout, mg, pcg, sipdg

    def problem(m, k):
        mesh = wl.meshes[m]
        axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
        X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
        d = wl.batch.densities[k]
        fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
        return axes, sipdg.rhs(axes, d.density(X, Y, Z), [d.potential(fx[f], fy[f], fz[f]) for f in range(6)])

    cpu = None
    if args.cpu_sample > 0:
        m = len(wl.meshes) - 1
        mesh = wl.meshes[m]
        H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi, n_levels=wl.n_levels)
        axes, b = problem(m, per[m][0])
        t0 = time.perf_counter()
        _, it, _, _ = pcg.solve(H, b, rtol=args.rtol)
        dt = time.perf_counter() - t0
        cpu = {"value": 1.0 / dt, "unit": "RHS/s", "cores": _threads(), "kind": "oracle", **_host(),
               "sample": f"one density of the {mesh.E[0]}^3 mesh, oracle MG-PCG FP64 to {args.rtol:g}, {it} "
                         f"iterations; set-up excluded (the smaller meshes are faster)"}
    check = None
    if args.check != 0:
        check = {}
        for arm, v in pots.items():
            errs = []
            for m, ks in per.items():
                mesh = wl.meshes[m]
                for k in (ks[0], ks[len(ks) // 2], ks[-1]):
                    axes, b = problem(m, k)
                    ref = fdm.FDM(axes).solve(b)
                    Mw = sipdg.mass(axes)
                    got = layout.to_global(v[offs[k]:offs[k + 1]].cpu().numpy(), mesh.E, mesh.p + 1)
                    errs.append(float(np.sqrt(np.sum(Mw * (got - ref) ** 2) / np.sum(Mw * ref ** 2))))
            check[arm] = {"rhs_checked": len(errs), "max_rel_L2_err_vs_exact": max(errs)}
    return cpu, check


# ---------------------------------------------------------------------------
# single small right-hand side (latency-bound)

def main_single(args):
    """One right-hand side on the 4^3-element, p = 3 mesh (4,096 nodes, 2 levels, tolerance 1e-10):
    the vectors stay in cache, so the solve is bound by launch latency; reported as us per solve."""
    import torch

    from paper_2510_21213_amd import binding
    from workloads import configs

    wl = configs.single()
    mesh = wl.meshes[0]
    d = wl.batch.densities[0]
    # arms: a precision, optionally +fused (one work-group per RHS runs the whole FP64 solve) or
    # +group (the group-persistent launch: fused_wgs work-groups per RHS, group barriers)
    arms = [a for a in args.arms.split(",") if a and "learned" not in a and "untrained" not in a] or ["fp64"]
    results, pots = {}, {}
    for arm in arms:
        opts = dict(args.solver_opts)
        if arm.endswith("+fused"):
            opts["fused"] = 1
        elif arm.endswith("+group"):
            opts["fused"] = 2
        ctx = binding.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=wl.rtol,
                              precision=arm.split("+")[0], **opts)
        xyz, fxyz = ctx.mesh_coords(0)
        rho = torch.as_tensor(d.density(xyz[0], xyz[1], xyz[2])).cuda()
        g = torch.as_tensor(d.potential(fxyz[0], fxyz[1], fxyz[2])).cuda()
        for _ in range(args.warmup):
            ctx.solve_batch(rho, g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            v, st = ctx.solve_batch(rho, g)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        results[arm] = {"value": 1.0 / dt, "us_per_solve": 1e6 * dt, "iters": st[0]["iters"],
                        "outer_iters": st[0]["outer_iters"], "rel_residual": st[0]["rel_residual"],
                        "fused": opts.get("fused", 0), "fused_wgs": opts.get("fused_wgs", 0),
                        "fused_fallbacks": ctx.fused_fallbacks()}
        pots[arm] = v
        ctx.close()
    check = cpu = None
    if args.check != 0 or args.cpu_sample > 0:
        cpu, check = cpu_leg_single(args, wl, pots)
    head_arm = arms[0]
    head = results[head_arm]
    line = {
        "metric": "Poisson RHS solved/sec at 1e-10 rel. residual (single RHS, latency-bound)",
        "value": head["value"], "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e-3 * head["us_per_solve"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE_OF[head_arm.split("+")[0]], "data": "synthetic",
        "config": {"workload": "single: two-Gaussian density, 4^3 elements p=3 (4096 DOFs), 2-level MG-PCG to 1e-10",
                   "arm": head_arm, "parallelism": "single GPU"},
        "arms": results,
        "roofline": None,
        "roofline_note": "4,096 nodes per vector stay in cache: bound by launch latency, reported as us per solve",
        "cpu_baseline": cpu,
        "check_vs_exact": check,
    }
    print(json.dumps(line))


def cpu_leg_single(args, wl, pots):
    import numpy as np

    from oracle import fdm, layout, mg, pcg, sipdg
    mesh = wl.meshes[0]
    d = wl.batch.densities[0]
    axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
    X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
    fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
    b = sipdg.rhs(axes, d.density(X, Y, Z), [d.potential(fx[f], fy[f], fz[f]) for f in range(6)])
    Mw = sipdg.mass(axes)
    ref = fdm.FDM(axes).solve(b)
    cont = d.potential(X, Y, Z)                   # the full-space potential the discretisation approximates

    def err(a, r):
        return float(np.sqrt(np.sum(Mw * (a - r) ** 2) / np.sum(Mw * r ** 2)))
    check = None
    if args.check != 0:
        check = {arm: {"rel_L2_err_vs_exact": err(layout.to_global(v.cpu().numpy(), mesh.E, mesh.p + 1), ref),
                       "rel_L2_err_vs_continuum": err(layout.to_global(v.cpu().numpy(), mesh.E, mesh.p + 1), cont)}
                 for arm, v in pots.items()}
    cpu = None
    if args.cpu_sample > 0:
        H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi, n_levels=wl.n_levels)
        pcg.solve(H, b, rtol=wl.rtol)
        n = 20
        t0 = time.perf_counter()
        for _ in range(n):
            _, it, _, _ = pcg.solve(H, b, rtol=wl.rtol)
        dt = (time.perf_counter() - t0) / n
        cpu = {"value": 1.0 / dt, "unit": "RHS/s", "us_per_solve": 1e6 * dt, "cores": _threads(), "kind": "oracle",
               **_host(),
               "sample": f"{n} solves of the single-Gaussian problem, oracle MG-PCG FP64 to {wl.rtol}, "
                         f"{it} iterations; set-up excluded"}
    return cpu, check


# ---------------------------------------------------------------------------
# adaptive octree auxiliary mesh

# Chebyshev steps on the octree's degree-4 and degree-2 levels, and on its degree-1 levels: on this
# mesh the iteration count follows the first alone (6: 30-32 iterations, 8: 23-26, 10: 19-23) and
# the degree-1 levels' steps only cost time; (8, 4) was the fastest measured on MI355X
OCTREE_CHEB = (8, 4)


def main_octree(args):
    """The 36 pair densities of the exchange8 molecule on its adaptive octree mesh (8^3 base
    elements on [-8, 8]^3, q = 4, refined on the electron density with delta_q = 1e-8, at most 3
    refinements): a step assembles the right-hand sides and solves them by MG-PCG to an FP64
    relative residual of 1e-8 over the refinement hierarchy.  Arms: the V-cycle in FP32 under
    the FP64 CG (fp32_pc, the line's value) and in FP64 (fp64)."""
    import numpy as np
    import torch

    from paper_2510_21213_amd import binding
    from workloads import configs

    wl = configs.octree()
    mesh, orb = wl.meshes[0], wl.orbitals
    arms = {}
    f = g = None
    for prec in ("fp32_pc", "fp64"):
        t0 = time.perf_counter()
        o = binding.Octree(mesh.E, mesh.lo, mesh.hi, q=mesh.p, rho=wl.density, delta_q=wl.delta_q,
                           max_depth=wl.max_depth, rtol=wl.rtol, max_iter=500, cheb_degree=OCTREE_CHEB[0],
                           cheb_degree_h=OCTREE_CHEB[1], precision=prec)
        t_setup = time.perf_counter() - t0
        log(f"octree {prec}: {o.n_elements} elements, {o.n_dofs} nodes, {o.n_levels} levels, set-up {t_setup:.2f} s")
        if f is None:
            xyz = o.nodes()
            bxyz = o.boundary_points()
            pairs = orb.pairs()                   # the order of Orbitals.pair_potentials
            psi = np.asarray(orb.values(xyz[0], xyz[1], xyz[2]))
            f = torch.as_tensor(np.stack([psi[i] * psi[j] for i, j in pairs])).cuda().contiguous()
            g = torch.as_tensor(orb.pair_potentials(bxyz[0], bxyz[1], bxyz[2])).cuda().contiguous()
            nrhs = len(pairs)

        def step():
            b = o.rhs(f, g)
            return o.solve(b)
        for _ in range(args.warmup):
            x, st = step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x, st = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        iters = [s["iters"] for s in st]
        log(f"octree {prec}: {dt * 1e3:.1f} ms per step, iterations {min(iters)}..{max(iters)}")
        arms[prec] = {"o": o, "x": x, "dt": dt, "iters": iters, "setup_s": t_setup,
                      "max_rel_residual": max(s["rel_residual"] for s in st)}
    o = arms["fp64"]["o"]
    # dominant kernel family of each arm: the finest-level operator (k_oct_op<5, ...>), APPLY form
    # timed on the binding's stream with HIP events; algorithmic bytes: read u, write y (geometry
    # and pieces are < 1 %)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20

    def timed(fn, arg):
        for _ in range(3):
            fn(arg)
        e0.record()
        for _ in range(reps):
            fn(arg)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3
    u = torch.randn(nrhs * o.n_dofs, dtype=torch.float64, device="cuda")
    t_op64 = timed(o.apply, u)
    t_op32 = timed(arms["fp32_pc"]["o"].apply_f32, u.float())
    algo32, algo64 = 8.0 * o.n_dofs * nrhs, 16.0 * o.n_dofs * nrhs

    def roofline(kernel, algo, t):
        return {"kernel": kernel, "bound": "hbm", "achieved": algo / t / 1e9, "peak": 8000.0, "unit": "GB/s",
                "frac": algo / t / 8e12, "traffic": None, "us_per_launch": t * 1e6, "algorithmic_bytes_per_launch": algo}
    roof = roofline("k_oct_op<5, APPLY, float> (finest-level operator of the FP32 V-cycle, 36 RHS)", algo32, t_op32)
    roof["traffic"] = measured_traffic("octree_step_exchange8.md", "dg_octree.hip", "fp32_pc")
    roof["fp64_arm"] = roofline("k_oct_op<5, APPLY, double> (36 RHS)", algo64, t_op64)
    roof["fp64_arm"]["traffic"] = measured_traffic("octree_step_exchange8.md", "dg_octree.hip", "fp64")
    # accuracy against the closed-form continuum potentials at the nodes (discretisation error),
    # and of the FP32-V-cycle arm against the FP64 one
    vall = orb.pair_potentials(xyz[0], xyz[1], xyz[2])
    res = {}
    x64 = arms["fp64"]["x"].cpu().numpy().reshape(nrhs, -1)
    for prec, A in arms.items():
        xs = A["x"].cpu().numpy().reshape(nrhs, -1)
        errs = [float(np.linalg.norm(xs[k] - vall[k]) / np.linalg.norm(vall[k])) for k in range(nrhs)]
        dev = max(float(np.linalg.norm(xs[k] - x64[k]) / np.linalg.norm(x64[k])) for k in range(nrhs))
        res[prec] = {"value": nrhs / A["dt"], "ms_per_step": A["dt"] * 1e3,
                     "iters": {"min": min(A["iters"]), "max": max(A["iters"]), "mean": float(np.mean(A["iters"]))},
                     "max_rel_residual": A["max_rel_residual"], "setup_s": A["setup_s"],
                     "rel_L2_err_vs_continuum": {"max": max(errs), "median": float(np.median(errs))},
                     "max_rel_L2_dev_vs_fp64_arm": dev}
    # Dirichlet data by quadrature of the pair densities (Sec. 6.3) against the closed forms
    gq = o.boundary_data(f)
    torch.cuda.synchronize()
    e0.record()
    gq = o.boundary_data(f)
    e1.record()
    torch.cuda.synchronize()
    t_q = e0.elapsed_time(e1) * 1e-3
    gq_err = float(((gq - g).abs().max() / g.abs().max()).item())
    log(f"octree: quadrature Dirichlet data {t_q * 1e3:.2f} ms, max rel. deviation from closed form {gq_err:.2e}")
    cpu = cpu_leg_octree(args, wl, pairs, arms["fp64"]["iters"]) if args.cpu_sample > 0 else None
    head = res["fp32_pc"]
    line = {
        "metric": "Poisson RHS solved/sec on the adaptive octree auxiliary mesh (MG-PCG to FP64 residual 1e-8)",
        "value": head["value"], "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE_OF["fp32_pc"], "data": "synthetic",
        "config": {"workload": f"octree: exchange8 molecule, 36 pair densities, {mesh.E[0]}^3 base elements q={mesh.p} "
                               f"refined on the electron density (delta_q {wl.delta_q}, depth {wl.max_depth}): "
                               f"{o.n_elements} elements, {o.n_dofs} nodes, {o.n_levels} levels; Chebyshev "
                               f"steps {OCTREE_CHEB[0]} (degree 4, 2), {OCTREE_CHEB[1]} (degree 1)",
                   "arm": "fp32_pc", "parallelism": "single GPU"},
        "arms": res,
        "speedup_vs_fp64": head["value"] / res["fp64"]["value"],
        "roofline": roof,
        "quadrature_data": {"ms": t_q * 1e3, "points": o.n_boundary, "sources": nrhs,
                            "max_rel_dev_vs_closed_form": gq_err,
                            "note": "Dirichlet data by quadrature of the 36 pair densities over the octree's "
                                    "nodes (Sec. 6.3), not in the timed step (which uses the closed forms)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def cpu_leg_octree(args, wl, pairs, gpu_iters):
    """The oracle's octree MG-PCG on one pair (set-up excluded): a few iterations timed, scaled by
    the iteration count of the GPU solve of that pair."""
    import numpy as np

    from oracle import octree, pcg
    mesh, orb = wl.meshes[0], wl.orbitals
    tree = octree.Octree(mesh.E, mesh.lo, mesh.hi, mesh.p, rho=wl.density, delta_q=wl.delta_q,
                         max_depth=wl.max_depth)
    H = octree.Hierarchy(tree, degree=OCTREE_CHEB[0], degree_h=OCTREE_CHEB[1])
    m = H.meshes[0]
    X, Y, Z = m.nodes()
    bx, by, bz = m.boundary_points()
    i, j = pairs[0]
    psi = np.asarray(orb.values(X, Y, Z))
    g = orb.pair_potentials(bx, by, bz)[0]
    b = m.rhs(psi[i] * psi[j], g)
    n_it = 3
    t0 = time.perf_counter()
    pcg.pcg(H.levels[0].A, b, H.vcycle, rtol=1e-30, maxit=n_it)
    per_it = (time.perf_counter() - t0) / n_it
    solve_s = per_it * gpu_iters[0]
    return {"value": 1.0 / solve_s, "unit": "RHS/s", "cores": _threads(), "kind": "oracle", **_host(),
            "sample": f"{n_it} oracle PCG iterations on pair {pairs[0]} of the same mesh ({per_it:.2f} s each), "
                      f"scaled by the GPU solve's {gpu_iters[0]} iterations; octree and multigrid set-up excluded"}


# ---------------------------------------------------------------------------
# Dirichlet data by quadrature

def main_consumers(args):
    """Consumers of the potentials on the exchange8 mesh (16^3 elements, p = 4, 512,000 nodes):
    the Hartree action of the 8 orbitals projected on a basis of 256 grid functions (one
    quadrature pass: each basis function read once), the exchange action of the 8 orbitals on
    the same basis (64 pair solves, W, projection), the compressed-exchange build from the
    orbitals' W and the compressed operator projected on the basis.  The projection kernel is
    timed with HIP events on the stream it runs on, against the HBM peak."""
    import numpy as np
    import torch

    from oracle import consumers, layout, sipdg
    from paper_2510_21213_amd import binding
    from workloads import configs

    wl = configs.exchange8()
    mesh, orb = wl.meshes[0], wl.orbitals
    arm = [a for a in args.arms.split(",") if a][0]
    prec, _, learned = arm.partition("+")
    ctx = binding.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=args.rtol,
                          precision=prec, lanes=args.lanes, **args.solver_opts)
    if learned == "learned":
        net = binding.Net(4, 32, 125, 27)
        net.load(args.weights or os.path.join(ROOT, "paper_2510_21213_amd", "weights", "guess_16e_p4.bin"))
        ctx.attach_guess(net)
    xyz, fxyz = ctx.mesh_coords(0)
    nd = ctx.info[0]["n_dofs"]
    n = orb.norb
    nbasis = 256
    psi = orb.values_torch(*xyz, device="cuda").reshape(-1).contiguous()
    gen = torch.Generator(device="cuda").manual_seed(11)
    phi = torch.randn(nbasis * nd, dtype=torch.float64, device="cuda", generator=gen)
    vH = torch.randn(nd, dtype=torch.float64, device="cuda", generator=gen)
    pairs_g = orb.pair_potentials_torch(*fxyz, device="cuda")            # [npairs(i<=j), nface]
    idx = [min(a, s) * n - min(a, s) * (min(a, s) - 1) // 2 + abs(a - s) for a in range(n) for s in range(n)]
    g_as = pairs_g[idx].reshape(-1).contiguous()                        # pair (a, s) at a*n + s

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        out = None
        for a, b in ev:
            a.record()
            out = fn()
            b.record()
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev])) * 1e-3, out

    dt_h, J = timed(lambda: ctx.hartree_action(phi, psi, vH), max(args.steps, 20))
    dt_x, (Kx, W, st) = timed(lambda: ctx.exchange_action(phi, psi, psi, g_pairs=g_as, keep_w=True), args.steps)
    dt_b, xi = timed(lambda: ctx.ace_build(psi, W), max(args.steps, 20))
    dt_a, Ka = timed(lambda: ctx.ace_action(phi, psi, xi), max(args.steps, 20))
    bytes_h = float(nbasis + n + 1) * nd * 8
    achieved = bytes_h / dt_h / 1e9
    ace_err = float((Ka - Kx).abs().max() / Kx.abs().max())
    check = cpu = None
    if args.check != 0 or args.cpu_sample > 0:
        # oracle projection of a sample of basis rows (the same seeded fields, moved to the host)
        axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
        w = consumers.weights(axes)
        rows = [0, 101, 255]
        ph = [layout.to_global(phi[r * nd:(r + 1) * nd].cpu().numpy(), mesh.E, mesh.p + 1) for r in rows]
        ps = [layout.to_global(x, mesh.E, mesh.p + 1) for x in psi.cpu().numpy().reshape(n, -1)]
        vh = layout.to_global(vH.cpu().numpy(), mesh.E, mesh.p + 1)
        t0 = time.perf_counter()
        ref = consumers.hartree_action(w, ph, ps, vh)
        dt_cpu = time.perf_counter() - t0
        got = J.cpu().numpy()[rows]
        check = {"hartree_rows_checked": len(rows),
                 "max_rel_err": float(np.abs(got - ref).max() / np.abs(ref).max())}
        cpu = {"value": len(rows) / dt_cpu, "unit": "basis rows projected/s (8 vectors)",
               "cores": os.cpu_count(), "kind": "oracle",
               "sample": f"oracle hartree_action of {len(rows)} basis rows against the 8 orbitals"}
    ctx.close()
    line = {
        "metric": "Hartree action of 8 orbitals projected on a 256-function basis, calls/sec",
        "value": 1.0 / dt_h, "unit": "calls/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt_h, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"consumers: exchange8 mesh {mesh.E[0]}^3 elements p={mesh.p} ({nd} nodes), "
                               f"{n} orbitals, {nbasis} seeded random basis fields",
                   "arm": arm, "parallelism": "single GPU"},
        "exchange_action": {"ms_per_call": 1e3 * dt_x, "pair_solves": n * n, "rhs_per_s": n * n / dt_x,
                            "max_rel_residual": float(max(s["rel_residual"] for s in st))},
        "ace_build_ms": 1e3 * dt_b, "ace_action_ms": 1e3 * dt_a,
        "ace_vs_exchange_on_occupied_max_rel": ace_err,
        "roofline": {"bound": "hbm", "kernel": "k_project (quadrature projection) with its chunk reduction",
                     "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": None, "algorithmic_bytes_per_launch": bytes_h,
                     "bytes_counted": "each basis field, each orbital and the potential read once (8 B per node)",
                     "timing_source": "HIP events on the current torch stream around each call"},
        "cpu_baseline": cpu,
        "check_vs_oracle": check,
    }
    print(json.dumps(line))


def main_quadrature(args):
    """The exchange step of the 8-orbital workload (36 pair densities, 16^3 elements, p = 4) with
    its Dirichlet data computed on the GPU by quadrature of the pair densities over the grid
    (g left to the library), against the same step given closed-form data; and the quadrature
    kernel alone, timed with HIP events on the stream it runs on, against the FP64 vector peak."""
    import numpy as np
    import torch

    from paper_2510_21213_amd import binding
    from workloads import configs

    wl = configs.exchange8()
    mesh, orb = wl.meshes[0], wl.orbitals
    n = orb.norb
    pairs = orb.pairs()
    npairs = len(pairs)
    arm = [a for a in args.arms.split(",") if a][0]
    prec, _, learned = arm.partition("+")
    ctx = binding.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=args.rtol,
                          precision=prec, lanes=args.lanes, **args.solver_opts)
    net = None
    if learned == "learned":
        net = binding.Net(4, 32, 125, 27)
        net.load(args.weights or os.path.join(ROOT, "paper_2510_21213_amd", "weights", "guess_16e_p4.bin"))
        ctx.attach_guess(net)
    xyz, fxyz = ctx.mesh_coords(0)
    phi = orb.values_torch(*xyz, device="cuda").reshape(-1).contiguous()
    rho = binding.pair_densities(phi, n)
    g_cf = orb.pair_potentials_torch(*fxyz, device="cuda").reshape(-1).contiguous()
    nface, ndof = ctx.info[0]["n_face"], ctx.info[0]["n_dofs"]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, out

    dt_q, (W, K, EX, st, _) = timed(lambda: ctx.exchange(phi, None))
    dt_c, (_, K_c, EX_c, _, _) = timed(lambda: ctx.exchange(phi, g_cf))
    # the quadrature entry point alone (pack, sum over the grid, split reduction), timed by events
    # on the current torch stream, which is the stream the library enqueues on
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    g = ctx.boundary_data(rho)
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        g = ctx.boundary_data(rho)
        b.record()
    torch.cuda.synchronize()
    dt_g = float(np.mean([a.elapsed_time(b) for a, b in ev])) * 1e-3
    flops = float(nface) * ndof * (9 + 2 * npairs)
    achieved = flops / dt_g / 1e12
    g_h = g.cpu().numpy().reshape(npairs, nface)
    g_cf_h = g_cf.cpu().numpy().reshape(npairs, nface)
    cpu = check = None
    if args.cpu_sample > 0:
        cpu, check = cpu_leg_quadrature(args, mesh, orb, pairs, nface, g_h)
    ctx.close()
    line = {
        "metric": "Poisson RHS solved/sec, Dirichlet data by quadrature on the GPU",
        "value": npairs / dt_q, "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt_q, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 data, " + DTYPE_OF[prec] + " solve", "data": "synthetic",
        "config": {"workload": f"quadrature: exchange8 step, {npairs} pair-density RHS, {mesh.E[0]}^3 elements "
                               f"p={mesh.p} ({ndof} DOFs, {nface} boundary nodes per RHS), Dirichlet data by "
                               f"quadrature, residual {args.rtol:g}", "arm": arm, "parallelism": "single GPU"},
        "step_with_closed_form_data": {"value": npairs / dt_c, "ms_per_step": 1e3 * dt_c},
        "boundary_data": {"ms_per_call": 1e3 * dt_g, "rhs_per_s": npairs / dt_g,
                          "pair_terms_per_s": float(nface) * ndof * npairs / dt_g},
        "quadrature_vs_closed_form": {
            "max_abs_diff_g": float(np.abs(g_h - g_cf_h).max()),
            "max_abs_diff_K_Ha": float(np.abs(K.cpu().numpy() - K_c.cpu().numpy()).max()),
            "E_x": EX, "E_x_closed_form_data": EX_c},
        "max_rel_residual": float(max(s["rel_residual"] for s in st)),
        "roofline": {"bound": "alu", "kernel": "k_quad (FP64 boundary-by-grid sum), bracketed with the pack "
                                               "and reduction launches of the same call",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic("boundary_quadrature_exchange8.md", "dg_boundary.hip", "fp64"),
                     "traffic_unit": "bytes per launch of k_quad (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                     "algorithmic_flops_per_launch": flops,
                     "flop_count": "per boundary-node/grid-node pair 9 (distance 8, reciprocal root 1) "
                                   "plus 2 per source",
                     "avg_launch_us": 1e6 * dt_g, "timing_source": "HIP events on the call's stream"},
        "cpu_baseline": cpu,
        "check_vs_oracle": check,
    }
    print(json.dumps(line))


def cpu_leg_quadrature(args, mesh, orb, pairs, nface, g_h):
    import numpy as np

    from oracle import boundary, sipdg
    axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
    X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
    po = orb.values(X, Y, Z)
    fo = np.stack([po[i] * po[j] for i, j in pairs])
    pts = boundary.boundary_points(axes)
    idx = np.arange(0, nface, max(1, nface // 384))
    t0 = time.perf_counter()
    go = boundary.potential_at(axes, fo, pts[idx])
    dt_o = time.perf_counter() - t0
    per_rhs = dt_o * (nface / len(idx)) / len(pairs)
    cpu = {"value": 1.0 / per_rhs, "unit": "RHS/s", "cores": _threads(), "kind": "oracle", **_host(),
           "sample": f"oracle direct sum for all {len(pairs)} pair densities at {len(idx)} of the {nface} "
                     f"boundary nodes ({dt_o:.1f} s), scaled to whole boundary-data sets per second"}
    check = {"max_rel_diff_vs_oracle": float(max(np.abs(g_h[q, idx] - go[q]).max() / np.abs(go[q]).max()
                                                 for q in range(len(pairs))))}
    return cpu, check


if __name__ == "__main__":
    main()
