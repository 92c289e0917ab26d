#!/usr/bin/env python3
"""Throughput of the MLS-MPM substep on one MI355X.

A step is one call of mpm_step_n advancing every particle of the workload
by `--substeps-per-step` substeps (the whole hot path: cell sort, stress,
P2G, grid update, G2P, return map).  The timed region holds exactly
`--steps` steps between two device synchronisations, with the particle
state resident in HBM.  Prints one JSON line on stdout; progress goes to
stderr.

Workload (default): 2,000,000 particles on twelve ellipsoid instances,
128^3 grid, dt = 5e-5, fixed-corotated / von Mises / Drucker-Prager
materials, FP32 state with FP64 SVD.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one particle-substep in the fused kernel: read x (12),
# F (36), params (16) and material id (4); write x (12) and F (36)
BYTES_PER_PARTICLE = 116
# per active grid node: its accumulated (mv, m) written once and read once
BYTES_PER_ACTIVE_NODE = 32


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(sc, n_sub=2):
    """The FP64 oracle on `n_sub` substeps of the full workload, on the host."""
    import torch

    from oracle import mpm_oracle as O
    params = O.Params.from_scene(sc)
    state = O.state_from_scene(sc)
    t0 = time.perf_counter()
    for _ in range(n_sub):
        state = O.substep(state, params)
    dt = time.perf_counter() - t0
    return dict(value=sc.n * n_sub / dt, unit="particle-substeps/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{n_sub} substeps of the full {sc.n}-particle workload from its initial state "
                       f"({dt:.1f} s, float64 PyTorch CPU)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--substeps-per-step", type=int, default=20)
    ap.add_argument("--sort-every", type=int, default=0)
    ap.add_argument("--item", type=int, default=0, help="particles per work item (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-total", type=int, default=2_000_000)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the workload would shard by scene or by grid slab; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    log("generating workload ...")
    t = time.perf_counter()
    sc = scenes.make_scene("large_scene", n_total=args.n_total)
    log(f"  {sc.n} particles, {sc.grid_res}^3 grid, generated in {time.perf_counter() - t:.1f} s")

    ctx = B.init_from_scene(sc, sort_every=args.sort_every)
    if args.item:
        B.mpm_set_tuning(ctx, chunk=args.item)
    p = B.Particles.from_scene(sc)
    S = args.substeps_per_step
    for w in range(args.warmup):
        B.mpm_step_n(ctx, p, S)
        torch.cuda.synchronize()
        log(f"  warmup step {w + 1}/{args.warmup} done")

    B.mpm_profile(ctx, True)
    B.mpm_profile_read(ctx)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        B.mpm_step_n(ctx, p, S)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.mpm_profile_read(ctx)
    B.mpm_profile(ctx, False)
    elapsed = t1 - t0
    log(f"  timed {args.steps} steps x {S} substeps in {elapsed:.3f} s")

    diag = B.mpm_get_diagnostics(ctx)
    m, _, _ = B.grid_state(ctx)
    active = int((m > 0).sum().item())
    torch.cuda.synchronize()

    value = sc.n * S * args.steps / elapsed
    fused_ms, fused_n = prof["fused_substep"]
    fused_avg_s = fused_ms / max(fused_n, 1) / 1e3
    bytes_launch = BYTES_PER_PARTICLE * sc.n + BYTES_PER_ACTIVE_NODE * active
    achieved = bytes_launch / fused_avg_s / 1e9 if fused_n else None
    roofline = dict(bound="hbm", kernel="k_substep<fused>", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=(achieved / HBM_PEAK_GBS) if achieved else None, traffic=None,
                    bytes_per_launch=bytes_launch, avg_launch_us=fused_avg_s * 1e6, launches=fused_n,
                    active_nodes=active)
    breakdown = {k: dict(ms=round(v[0], 3), launches=v[1]) for k, v in prof.items() if v[1]}
    log("  kernel time by class:", json.dumps(breakdown))
    log("  diagnostics:", diag)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline(scenes.make_scene("large_scene", n_total=args.n_total))
        log(f"  oracle: {cpu['value']:.3e} particle-substeps/s on {cpu['cores']} threads")

    out = {
        "metric": "particle-substeps/s (forward MLS-MPM substep)",
        "value": value,
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "large_scene: 2M particles (12 ellipsoids, shell + MCIS interior), 128^3 grid, dt 5e-5, "
                        "fixed-corotated / von Mises / Drucker-Prager, FP32 state, FP64 SVD",
            "particles": sc.n, "grid_res": sc.grid_res, "substeps_per_step": S, "sort_every": args.sort_every,
            "item": args.item,
            "kernel_time_by_class_ms": breakdown,
            "diagnostics": {k: diag[k] for k in ("nonfinite", "out_of_grid", "tile_overflow", "tile_escapes")},
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
