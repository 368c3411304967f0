#!/usr/bin/env python
"""Benchmark: Poisson right-hand sides solved per second at FP64 relative residual 1e-8.

Workload (default ``exchange8``): the exchange step of 8 Loewdin-orthonormal
orbitals on a 16x16x16-element, degree-4 auxiliary mesh (512,000 nodes) --
all 36 pair densities rho_ij = phi_i phi_j as Poisson right-hand sides with
closed-form Dirichlet data, solved to 1e-8 by 4-level hp-multigrid PCG, then
W_k, K_ij and E_x.  One step = one dg_exchange_apply call (RHS assembly, the
batched solve and the exchange reductions) with all inputs resident in HBM.

Arms: ``fp32_ir`` (FP32 inner PCG inside FP64 iterative refinement; the
headline ``value``) and ``fp64`` (plain FP64 MG-PCG; reported beside it).

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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=6,
                    help="untimed steps first: the first calls capture the PCG graphs and learn how many "
                         "iteration blocks to replay before a host check (about five calls to settle)")
    ap.add_argument("--config", default="exchange8",
                    choices=["exchange8", "exchange16", "large", "uneven", "single", "quadrature"],
                    help="uneven: 256 densities over 8^3, 12^3 and 16^3 meshes in one interleaved batch; "
                         "single: one two-Gaussian density on 4^3 elements p=3 (latency-bound); "
                         "quadrature: the exchange8 step with its Dirichlet data computed by quadrature")
    ap.add_argument("--arms", default="fp32_ir+learned,fp32_ir,fp64+learned,fp64",
                    help="precision fp32_ir or fp64, optionally +learned (trained guess) or +untrained "
                         "(the same network with random weights, a control)")
    ap.add_argument("--weights", default=None,
                    help="guess network (default: the weights trained for the workload's mesh)")
    ap.add_argument("--lanes", type=int, default=2, choices=[1, 2],
                    help="solver lanes per mesh: 2 solves a batch as two concurrent halves")
    ap.add_argument("--cheb-degree", type=int, default=None, help="smoothing steps (default: the library's)")
    ap.add_argument("--cheb-ratio", type=float, default=None, help="smoothing interval ratio (default: the library's)")
    ap.add_argument("--cheb-degree-h", type=int, default=None,
                    help="smoothing steps on the degree-1 coarse levels (default: the library's)")
    ap.add_argument("--inner-rtol", type=float, default=None, help="inner FP32 tolerance (default: the library's)")
    ap.add_argument("--cpu-sample", type=int, default=12, help="pair solves timed on the oracle (0: skip)")
    ap.add_argument("--check-sample", type=int, default=4, help="pairs compared with the exact solve (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run 3 device-to-device copies of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    args.solver_opts = {k: v for k, v in (("cheb_degree", args.cheb_degree), ("cheb_ratio", args.cheb_ratio),
                                          ("cheb_degree_h", args.cheb_degree_h), ("inner_rtol", args.inner_rtol))
                        if v is not None}
    return args


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is measured; run with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2510_21213_amd import binding
    from workloads import configs

    torch.cuda.set_device(0)
    if args.config == "uneven":
        return main_uneven(args)
    if args.config == "single":
        return main_single(args)
    if args.config == "quadrature":
        return main_quadrature(args)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    wl = {"exchange8": configs.exchange8, "exchange16": configs.exchange16,
          "large": lambda: configs.large_molecule(0, held_out=True)}[args.config]()
    if args.weights is None:
        name = "guess_32e_p4.bin" if args.config == "large" else "guess_16e_p4.bin"
        args.weights = os.path.join(ROOT, "paper_2510_21213_amd", "weights", name)
    mesh = wl.meshes[0]
    orb = wl.orbitals
    norb = orb.norb
    npairs = norb * (norb + 1) // 2
    arms = [a for a in args.arms.split(",") if a]
    results = {}
    first_ctx = None
    net = None
    for arm in arms:
        prec, _, learned = arm.partition("+")
        if learned not in ("", "learned", "untrained"):
            raise SystemExit(f"unknown arm {arm}")
        ctx = binding.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=wl.rtol,
                              precision=prec, lanes=args.lanes, **args.solver_opts)
        if learned == "learned":
            if net is None:
                net = binding.Net(4, 32, 125, 27)
                net.load(args.weights)
            ctx.attach_guess(net)
        elif learned == "untrained":
            # control: the same architecture with random (He) weights, as in the training script
            from paper_2510_21213_amd.train_guess import he_init
            control = binding.Net(4, 32, 125, 27)
            control.set_params(he_init(control, np.random.default_rng(12345)))
            ctx.attach_guess(control)
        if first_ctx is None:
            xyz, fxyz = ctx.mesh_coords(0)
            phi = torch.as_tensor(orb.values(xyz[0], xyz[1], xyz[2]).reshape(-1)).cuda()
            g = torch.as_tensor(orb.pair_potentials(fxyz[0], fxyz[1], fxyz[2]).reshape(-1)).cuda()
            first_ctx = ctx
        for _ in range(args.warmup):
            ctx.exchange(phi, g)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        iters, outer, res, used, step_s = [], [], [], [], []
        for _ in range(args.steps):
            ts = time.perf_counter()
            W, K, EX, st, _ = ctx.exchange(phi, g)   # returns after its stream is synchronised
            step_s.append(time.perf_counter() - ts)
            iters += [s["iters"] for s in st]
            outer += [s["outer_iters"] for s in st]
            res += [s["rel_residual"] for s in st]
            used += [s["guess_used"] for s in st]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = ctx.profile_read()
        ctx.profile(False)
        if prof["launches"] < 0:
            # the runtime could not time events recorded inside the captured graph: time the
            # same steps on eager launches instead (same kernels, same inputs), on one solver
            # lane so that every timed launch runs alone (two lanes overlap their launches)
            ectx = binding.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=wl.rtol,
                                   precision=prec, use_graph=0, lanes=1, **args.solver_opts)
            if learned == "learned":
                ectx.attach_guess(net)
            elif learned == "untrained":
                ectx.attach_guess(control)
            ectx.exchange(phi, g)
            ectx.profile(True)
            for _ in range(args.steps):
                ectx.exchange(phi, g)
            prof = ectx.profile_read()
            prof["source"] = "eager launches on one solver lane (graph events not timeable)"
            ectx.profile(False)
            ectx.close()
        else:
            prof["source"] = "events inside the timed region"
        dt = t1 - t0
        results[arm] = {
            "value": npairs * args.steps / dt,
            "ms_per_step": 1e3 * dt / args.steps,
            "ms_per_step_median": 1e3 * float(np.median(step_s)),
            "iters_mean": float(np.mean(iters)), "iters_max": int(np.max(iters)),
            "outer_mean": float(np.mean(outer)),
            "max_rel_residual": float(np.max(res)),
            "guess_used": float(np.mean(used)) if learned else 0.0,
            "E_x": EX,
            "prof": prof,
            "ctx": ctx,
        }

    head_arm = arms[0]
    head = results[head_arm]
    prof = head["prof"]
    achieved = prof["bytes"] / prof["seconds"] / 1e9 if prof["seconds"] > 0 else None
    roofline = {
        "bound": "hbm",
        "kernel": "finest-level Chebyshev smoothing step (k_slab, N=5, BM_CHEB/BM_CHEBDOT, "
                  + ("float" if head_arm.startswith("fp32_ir") else "double") + ")",
        "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": (achieved / PEAK_HBM_GBS) if achieved else None,
        "traffic": measured_traffic("cheb_step_exchange8.md", "dg_kernels.hip")
        if (head_arm.startswith("fp32_ir") and args.config == "exchange8") else None,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
        "algorithmic_bytes_per_launch": prof["bytes"] / max(1, prof["launches"]),
        "avg_launch_us": 1e6 * prof["seconds"] / max(1, prof["launches"]),
        "launches": prof["launches"],
        "timing_source": prof.get("source"),
    }

    cpu = None
    check = None
    if args.cpu_sample > 0 or args.check_sample > 0:
        cpu, check = cpu_leg(args, wl, results, phi, g, npairs)

    arms_out = {a: {k: v for k, v in r.items() if k not in ("prof", "ctx")} for a, r in results.items()}
    for a, r in results.items():
        p = r["prof"]
        arms_out[a]["cheb_step_GBs"] = p["bytes"] / p["seconds"] / 1e9 if p["seconds"] > 0 else None
    line = {
        "metric": "Poisson RHS solved/sec at 1e-8 rel. residual: learned+mixed vs plain FP64 MG-PCG",
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
        "dtype": "f32" if head_arm.startswith("fp32_ir") else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {npairs} pair-density RHS, {mesh.E[0]}^3 elements p={mesh.p} "
                               f"({first_ctx.info[0]['n_dofs']} DOFs/RHS), {wl.n_levels}-level MG-PCG to {wl.rtol}",
                   "arm": head_arm, "learned_guess": "learned" in head_arm, "parallelism": "single GPU",
                   "solver_lanes": args.lanes},
        "arms": arms_out,
        "speedup_vs_plain_fp64": (head["value"] / results["fp64"]["value"]) if "fp64" in results else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "check_vs_exact": check,
    }
    print(json.dumps(line))


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
    arms = [a for a in args.arms.split(",") if a and "learned" not in a] or ["fp32_ir"]
    results = {}
    rho = g = None
    for arm in arms:
        ctx = binding.Context(meshes, n_levels=wl.n_levels, rtol=wl.rtol, precision=arm, lanes=args.lanes, **args.solver_opts)
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
            "v": v, "ctx": ctx,
        }
    check = None
    if args.check_sample > 0:
        from oracle import fdm, layout, sipdg
        check = {}
        for arm, r in results.items():
            v = r["v"].cpu().numpy()
            errs = []
            for m, ks in per.items():
                mesh = wl.meshes[m]
                axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
                X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
                M = sipdg.mass(axes)
                F = fdm.FDM(axes)
                for k in ks[:max(1, args.check_sample // len(per))]:
                    d = wl.batch.densities[k]
                    fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
                    fvals = [d.potential(fx[f], fy[f], fz[f]) for f in range(6)]
                    ref = F.solve(sipdg.rhs(axes, d.density(X, Y, Z), fvals))
                    got = layout.to_global(v[offs[k]:offs[k + 1]], mesh.E, mesh.p + 1)
                    errs.append(float(np.sqrt(np.sum(M * (got - ref) ** 2) / np.sum(M * ref ** 2))))
            check[arm] = {"rhs_checked": len(errs), "max_rel_L2_err_vs_exact": max(errs)}
    head_arm = arms[0]
    head = results[head_arm]
    line = {
        "metric": "Poisson RHS solved/sec at 1e-8 rel. residual (uneven batch)",
        "value": head["value"], "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if head_arm.startswith("fp32_ir") else "f64", "data": "synthetic",
        "config": {"workload": "uneven: 256 Gaussian-sum densities over 8^3, 12^3, 16^3 elements p=4 "
                               "(86/85/85, interleaved), 4-level MG-PCG to 1e-08", "arm": head_arm,
                   "parallelism": "single GPU"},
        "arms": {a: {k: v for k, v in r.items() if k not in ("v", "ctx")} for a, r in results.items()},
        "check_vs_exact": check,
    }
    print(json.dumps(line))


def main_single(args):
    """One right-hand side on the 4^3-element, p = 3 mesh (4,096 nodes, 2 levels, tolerance 1e-10):
    the vectors stay in cache, so the solve is bound by launch latency; reported as us per solve."""
    import numpy as np
    import torch

    from paper_2510_21213_amd import binding
    from workloads import configs

    wl = configs.single()
    mesh = wl.meshes[0]
    d = wl.batch.densities[0]
    arms = [a for a in args.arms.split(",") if a and "learned" not in a] or ["fp64"]
    results = {}
    for arm in arms:
        ctx = binding.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=wl.rtol,
                              precision=arm, **args.solver_opts)
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
                        "outer_iters": st[0]["outer_iters"], "rel_residual": st[0]["rel_residual"], "v": v}
    check = cpu = None
    if args.check_sample > 0 or args.cpu_sample > 0:
        from oracle import fdm, layout, mg, pcg, sipdg
        axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
        X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
        fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
        b = sipdg.rhs(axes, d.density(X, Y, Z), [d.potential(fx[f], fy[f], fz[f]) for f in range(6)])
        M = sipdg.mass(axes)
        ref = fdm.FDM(axes).solve(b)
        cont = d.potential(X, Y, Z)                   # the full-space potential the discretisation approximates

        def err(a, r):
            return float(np.sqrt(np.sum(M * (a - r) ** 2) / np.sum(M * r ** 2)))
        check = {arm: {"rel_L2_err_vs_exact": err(layout.to_global(r["v"].cpu().numpy(), mesh.E, mesh.p + 1), ref),
                       "rel_L2_err_vs_continuum": err(layout.to_global(r["v"].cpu().numpy(), mesh.E, mesh.p + 1), cont)}
                 for arm, r in results.items()}
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
    head_arm = arms[0]
    head = results[head_arm]
    line = {
        "metric": "Poisson RHS solved/sec at 1e-10 rel. residual (single RHS, latency-bound)",
        "value": head["value"], "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e-3 * head["us_per_solve"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if head_arm.startswith("fp32_ir") else "f64", "data": "synthetic",
        "config": {"workload": "single: two-Gaussian density, 4^3 elements p=3 (4096 DOFs), 2-level MG-PCG to 1e-10",
                   "arm": head_arm, "parallelism": "single GPU"},
        "arms": {a: {k: v for k, v in r.items() if k != "v"} for a, r in results.items()},
        "roofline": None,
        "roofline_note": "4,096 nodes per vector stay in cache: bound by launch latency, reported as us per solve",
        "cpu_baseline": cpu,
        "check_vs_exact": check,
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
    ctx = binding.Context([(mesh.E, mesh.p, mesh.lo, mesh.hi)], n_levels=wl.n_levels, rtol=wl.rtol,
                          precision=prec, lanes=args.lanes, **args.solver_opts)
    net = None
    if learned == "learned":
        net = binding.Net(4, 32, 125, 27)
        net.load(args.weights or os.path.join(ROOT, "paper_2510_21213_amd", "weights", "guess_16e_p4.bin"))
        ctx.attach_guess(net)
    xyz, fxyz = ctx.mesh_coords(0)
    phi_h = orb.values(xyz[0], xyz[1], xyz[2]).reshape(n, -1)
    phi = torch.as_tensor(phi_h.reshape(-1)).cuda()
    rho = torch.as_tensor(np.stack([phi_h[i] * phi_h[j] for i, j in pairs]).reshape(-1)).cuda()
    g_cf = torch.as_tensor(orb.pair_potentials(fxyz[0], fxyz[1], fxyz[2]).reshape(-1)).cuda()
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
    # the quadrature entry point alone (pack, sum over the grid, split reduction)
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
        from oracle import boundary, sipdg
        axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
        X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
        po = orb.values(X, Y, Z)
        fo = np.stack([po[i] * po[j] for i, j in pairs])
        pts = boundary.boundary_points(axes)
        idx = np.arange(0, nface, max(1, nface // (32 * args.cpu_sample)))
        t0 = time.perf_counter()
        go = boundary.potential_at(axes, fo, pts[idx])
        dt_o = time.perf_counter() - t0
        per_rhs = dt_o * (nface / len(idx)) / npairs
        cpu = {"value": 1.0 / per_rhs, "unit": "RHS/s", "cores": _threads(), "kind": "oracle", **_host(),
               "sample": f"oracle direct sum for all {npairs} pair densities at {len(idx)} of the {nface} "
                         f"boundary nodes ({dt_o:.1f} s), scaled to whole boundary-data sets per second"}
        check = {"max_rel_diff_vs_oracle": float(max(np.abs(g_h[q, idx] - go[q]).max() / np.abs(go[q]).max()
                                                     for q in range(npairs)))}
    line = {
        "metric": "Poisson RHS solved/sec at 1e-8 rel. residual, Dirichlet data by quadrature on the GPU",
        "value": npairs / dt_q, "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt_q, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 data, " + ("f32" if prec == "fp32_ir" else "f64") + " inner solve", "data": "synthetic",
        "config": {"workload": f"quadrature: exchange8 step, {npairs} pair-density RHS, {mesh.E[0]}^3 elements "
                               f"p={mesh.p} ({ndof} DOFs, {nface} boundary nodes per RHS), Dirichlet data by "
                               f"quadrature", "arm": arm, "parallelism": "single GPU"},
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
                     "traffic": measured_traffic("boundary_quadrature_exchange8.md", "dg_boundary.hip"),
                     "traffic_unit": "bytes per launch of k_quad (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                     "algorithmic_flops_per_launch": flops,
                     "flop_count": "per boundary-node/grid-node pair 9 (distance 8, reciprocal root 1) "
                                   "plus 2 per source",
                     "avg_launch_us": 1e6 * dt_g, "timing_source": "HIP events on the call's stream"},
        "cpu_baseline": cpu,
        "check_vs_oracle": check,
    }
    print(json.dumps(line))


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


def measured_traffic(profile_name, kernel_source):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None.

    None when the summary is missing or was taken on a different kernel source.
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
            if rec.get("kernel_source_sha256_16") == digest:
                return rec["traffic_bytes_per_launch"]
    return None


def cpu_leg(args, wl, results, phi, g, npairs):
    """Oracle timing on the host cores, and the GPU potentials against the exact solve."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_info

    from oracle import fdm, layout, mg, pcg, sipdg

    mesh = wl.meshes[0]
    orb = wl.orbitals
    axes = sipdg.make_axes(mesh.E, mesh.p, mesh.lo, mesh.hi)
    X, Y, Z = np.broadcast_arrays(*sipdg.node_grid(axes))
    fx, fy, fz = (layout.boundary_faces_of(A) for A in (X, Y, Z))
    phi_o = orb.values(X, Y, Z)
    pairs = orb.pairs()
    sample = list(range(0, npairs, max(1, npairs // max(1, max(args.cpu_sample, args.check_sample)))))

    def problem(q):
        i, j = pairs[q]
        faces = []
        for f in range(6):
            vals = orb.pair_potentials(fx[f].reshape(-1), fy[f].reshape(-1), fz[f].reshape(-1))[q]
            faces.append(vals.reshape(fx[f].shape))
        return sipdg.rhs(axes, phi_o[i] * phi_o[j], faces)

    cpu = None
    if args.cpu_sample > 0:
        H = mg.Hierarchy(mesh.E, mesh.p, mesh.lo, mesh.hi, n_levels=wl.n_levels)
        qs = sample[:args.cpu_sample]
        bs = [problem(q) for q in qs]
        t0 = time.perf_counter()
        its = []
        for b in bs:
            _, it, _, _ = pcg.solve(H, b, rtol=wl.rtol)
            its.append(it)
        dt = time.perf_counter() - t0
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        # the same solves on one host thread (a shorter sample), and the exact solve (fast diagonalisation)
        from threadpoolctl import threadpool_limits
        q1 = bs[:max(1, len(bs) // 6)]
        with threadpool_limits(1):
            t1 = time.perf_counter()
            for b in q1:
                pcg.solve(H, b, rtol=wl.rtol)
            dt1 = time.perf_counter() - t1
        F = fdm.FDM(axes)
        t2 = time.perf_counter()
        for b in bs:
            F.solve(b)
        dtf = time.perf_counter() - t2
        cpu = {"value": len(qs) / dt, "unit": "RHS/s", "cores": threads, "kind": "oracle", **_host(),
               "sample": f"{len(qs)} of {npairs} pair solves (pairs {qs}), oracle MG-PCG FP64 to {wl.rtol}, "
                         f"iterations {its}; set-up excluded",
               "value_1thread": len(q1) / dt1, "sample_1thread": f"the first {len(q1)} of those solves, one thread",
               "exact_fdm_value": len(bs) / dtf}
    check = None
    if args.check_sample > 0:
        out = {}
        for arm, r in results.items():
            ctx = r["ctx"]
            _, _, _, _, v = ctx.exchange(phi, g, keep_potentials=True)
            v = v.cpu().numpy().reshape(npairs, -1)
            M = sipdg.mass(axes)
            F = fdm.FDM(axes)
            errs = []
            for q in sample[:args.check_sample]:
                ref = F.solve(problem(q))
                got = layout.to_global(v[q], mesh.E, mesh.p + 1)
                errs.append(float(np.sqrt(np.sum(M * (got - ref) ** 2) / np.sum(M * ref ** 2))))
            out[arm] = {"pairs": sample[:args.check_sample], "max_rel_L2_err_vs_exact": max(errs)}
        check = out
    return cpu, check


if __name__ == "__main__":
    main()
