#!/usr/bin/env python
"""Pick the operator kernels' work-group tiles by timing the exchange step on the GPU.

The operator steps run as a slab kernel whose work-group owns tx x ty elements of the x-y plane
and zlen element layers (dg_tile_set lists the compiled shapes).  The steps are grouped (the
FP32 smoothing steps and restriction of the degree-4 level; its other FP32 steps; its FP64
steps; the degree-2 and degree-1 levels in each arithmetic) and every compiled tile of a group
is tried in turn, coordinate descent from the current table, with an exchange step timed end to
end.  Workload exchange8 (36 pair densities of 8 orbitals, 16^3 elements, p = 4): the FP32
refinement arm with the trained guess for FP32 tiles, the plain FP64 arm for FP64 tiles.
Workload large (the 36 pair densities of the first held-out molecule on 32^3 elements, p = 4,
5 levels): the FP32_PC arm with its trained guess for every group it runs (its V-cycle is FP32,
its search-direction and residual steps FP64).  A tile replaces the current one only when its
median step time is lower by more than the noise margin.  Writes the table (tiles_gfx950.json
next to this file by default), which the binding applies on import.

    python paper_2510_21213_amd/tune_tiles.py [--workload large] [--steps 8] [--warmup 4] [--margin 0.02]
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2510_21213_amd import binding  # noqa: E402
from workloads import configs  # noqa: E402

ALL = list(binding.STEPS)
SHAPES5 = [(4, 2), (4, 4), (2, 2)]
GROUPS = [
    # name, fp_bytes, n, steps, shapes, zlens, arm timed
    ("fp32 degree-4 smoothing and restriction", 4, 5, ["CHEB", "CHEBDOT", "RESTRICT"], SHAPES5, [1, 2, 3, 4],
     "fp32_ir+learned"),
    ("fp32 degree-4 other steps", 4, 5, ["APPLY", "RESID", "PQ", "RESIDDOT"], SHAPES5, [1, 2, 3, 4],
     "fp32_ir+learned"),
    ("fp32 degree-2", 4, 3, ALL, [(4, 4)], [1, 2, 3, 4], "fp32_ir+learned"),
    ("fp32 degree-1", 4, 2, ALL, [(8, 8)], [1, 2], "fp32_ir+learned"),
    ("fp64 degree-4", 8, 5, ALL, SHAPES5, [1, 2, 3, 4], "fp64"),
    ("fp64 degree-2", 8, 3, ALL, [(4, 4)], [1, 2, 3, 4], "fp64"),
    ("fp64 degree-1", 8, 2, ALL, [(8, 8)], [1, 2], "fp64"),
]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--margin", type=float, default=0.02, help="relative gain a new tile must show")
    ap.add_argument("--out", default=binding.TILE_TABLE)
    ap.add_argument("--workload", default="exchange8", choices=["exchange8", "large"])
    ap.add_argument("--rtol", type=float, default=None, help="residual of the timed solves (default: the workload's)")
    ap.add_argument("--arm", default="fp32_pc+learned", help="arm timed on the large workload")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    large = args.workload == "large"
    wl = configs.large_molecule(0, held_out=True) if large else configs.exchange8()
    rtol = args.rtol or (1e-11 if large else wl.rtol)
    mesh, orb = wl.meshes[0], wl.orbitals
    m = (mesh.E, mesh.p, mesh.lo, mesh.hi)
    net = binding.Net(4, 32, 125, 27)
    net.load(os.path.join(ROOT, "paper_2510_21213_amd", "weights",
                          "guess_32e_p4.bin" if large else "guess_16e_p4.bin"))
    probe = binding.Context([m], n_levels=wl.n_levels)
    xyz, fxyz = probe.mesh_coords(0)
    probe.close()
    phi = orb.values_torch(*xyz, device="cuda").reshape(-1).contiguous()
    g = orb.pair_potentials_torch(*fxyz, device="cuda").reshape(-1).contiguous()
    groups = GROUPS
    if large:  # the FP32_PC arm: FP32 V-cycle steps and the FP64 degree-4 steps
        groups = [(nm, fp, n, st, sh, zl, args.arm) for nm, fp, n, st, sh, zl, _ in GROUPS if fp == 4 or n == 5]

    def measure(arm):
        prec = arm.split("+")[0]
        ctx = binding.Context([m], n_levels=wl.n_levels, rtol=rtol, precision=prec)
        if "learned" in arm:
            ctx.attach_guess(net)
        for _ in range(args.warmup):
            ctx.exchange(phi, g)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            ctx.exchange(phi, g)
            ts.append(time.perf_counter() - t0)
        ctx.close()
        return float(np.median(ts))

    def set_group(fp, n, steps, tile):
        for st in steps:
            binding.tile_set(fp, n, st, *tile)

    trials = []
    t_start = time.time()
    for name, fp, n, steps, shapes, zlens, arm in groups:
        current = {st: binding.tile_get(fp, n, st) for st in steps}
        base = measure(arm)
        best, best_t = None, base
        for tx, ty in shapes:
            for z in zlens:
                tile = (tx, ty, z)
                if all(current[st] == tile for st in steps):
                    continue
                set_group(fp, n, steps, tile)
                t = measure(arm)
                trials.append({"group": name, "tile": list(tile), "ms": 1e3 * t, "current_ms": 1e3 * base})
                print(f"{name}: tile {tile} {1e3 * t:.2f} ms (current {1e3 * base:.2f} ms) "
                      f"[{time.time() - t_start:.0f}s]", flush=True)
                if t < best_t:
                    best, best_t = tile, t
        for st in steps:
            binding.tile_set(fp, n, st, *current[st])
        if best is not None and best_t < base * (1.0 - args.margin):
            set_group(fp, n, steps, best)
            print(f"{name}: chose {best} ({1e3 * best_t:.2f} ms against {1e3 * base:.2f} ms)", flush=True)
        else:
            print(f"{name}: kept the current tiles", flush=True)

    tiles = []
    for fp in (4, 8):
        for n in (2, 3, 5):
            for st in ALL:
                tx, ty, z = binding.tile_get(fp, n, st)
                tiles.append({"fp_bytes": fp, "n": n, "step": st, "tx": tx, "ty": ty, "zlen": z})
    wname = (f"large: 36 pair densities of the first held-out molecule, 32^3 elements, p = 4, 5 levels, {args.arm}"
             if large else "exchange8: 36 pair densities, 16^3 elements, p = 4, 4 levels")
    report = {"arch": "gfx950", "workload": f"{wname}, residual {rtol:g}",
              "timing": f"median of {args.steps} exchange steps after {args.warmup} warm-up steps",
              "margin": args.margin, "tiles": tiles, "trials": trials, "seconds": time.time() - t_start}
    with open(args.out, "w") as f:
        json.dump(report, f, indent=1)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
