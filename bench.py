#!/usr/bin/env python3
"""Throughput of the MLS-MPM substep on one MI355X.

A step is one render frame: every particle of the workload advances by
`--substeps-per-step` substeps (the whole hot path: cell sorts, stress,
P2G, grid update, G2P, return map) through mpm_advance on the scene held in
the context, and mpm_export_frame then writes the frame's positions and
Gaussian covariances in the caller's order.  The scene is copied into the
context (mpm_load) before warm-up.  The timed region holds exactly
`--steps` steps between two device synchronisations.  The same frames
through mpm_step_n (caller-order arrays in and out at every call) are timed
after it and reported beside the headline.  Prints one JSON line on stdout;
progress goes to stderr.

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
# LDS atomic adds of the P2G tile per particle-substep: 27 nodes x 4 channels
LDS_ADDS_PER_PARTICLE = 108
# algorithmic bytes of the adjoint kernels per particle-substep:
#   k_adj_g2p reads x 12, F 36 and the adjoints of x, v, C, F (96); writes
#     those of x and F (48)
#   k_adj_p2g reads x, v, C, F (96), params 16, material 4, log E 4, nu 4,
#     the adjoints of x and F (48) and the parameter gradients (8); writes
#     the adjoints of x, v, C, F (96) and the parameter gradients (8)
ADJ_G2P_BYTES = 192
ADJ_P2G_BYTES = 284
# one particle-substep of the taped forward + backward: the forward's fused
# kernel (116), its recompute that also writes v and C (164) and the two
# adjoint kernels
FWD_BWD_BYTES = 116 + 164 + ADJ_G2P_BYTES + ADJ_P2G_BYTES


KERNEL_SOURCES = ("paper_2602_01723_amd/csrc/mpm_kernels.hpp", "paper_2602_01723_amd/csrc/mpm_math.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_substep_large_scene_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The default-mode fused kernel's name in rocprofv3 records (the template
# arguments: fused mode, no deterministic variant, dense grid clearing).
FUSED_KERNEL = "k_substep<1, 0, false>"


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n_particles):
    """HBM bytes per fused-kernel launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for
    a plain copy of known size), or None if the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("particles") != n_particles:
        return None
    f_scale = t["copy_bytes"] / (t["copy_fetch_kib"] * 1024.0)
    w_scale = t["copy_bytes"] / (t["copy_write_kib"] * 1024.0)
    return t["fused_fetch_kib"] * 1024.0 * f_scale + t["fused_write_kib"] * 1024.0 * w_scale


# VALU issue of the fused kernel: one wave64 VALU instruction per SIMD every
# 4 clocks (16 lanes), 4 SIMDs per CU, 256 CUs at 2.4 GHz = 39.32e12 lane
# instructions/s.  The same issue rate gives the 78.6 TFLOP/s FP32 (unpacked)
# and FP64 FMA peaks.
VALU_PEAK_LANE_INSTR = 256 * 4 * 16 * 2.4e9
VALU_FILE = os.path.join(ROOT, "profiles", "fused_substep_large_scene_valu.json")
VALU_COMMAND = ("cd /tmp && rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
                "SQ_INSTS_LDS SQ_WAIT_INST_ANY SQ_INSTS_SALU --kernel-include-regex k_substep -f csv -d <out>/pmc_p1 "
                "-o p1 -- python3 <repo>/bench.py --steps 1 --warmup 1 --substeps-per-step 10 --no-autotune "
                "--no-step-n --no-cpu-baseline --no-batched --no-bgdo --no-models --no-mcis --no-ipf --no-det --no-configs --no-atomics")


def write_valu(p1_csv, n_particles=2_000_000):
    """Summarise the p1 instruction-mix pass (SQ_INSTS_VALU) of the fused
    kernel into VALU_FILE, stamped with the kernel source hash."""
    c = summarize_counters([p1_csv], n_particles=n_particles)
    out = {"kernel": FUSED_KERNEL, "particles": n_particles, "dispatches": c["dispatches"],
           "valu_instructions_per_particle": c["valu_instructions_per_particle"],
           "kernel_source_hash": kernel_source_hash(),
           "command": VALU_COMMAND}
    with open(VALU_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def measured_valu(n_particles):
    """VALU lane instructions per particle of the fused kernel from the
    committed counter summary, or None if the kernel sources changed since."""
    try:
        with open(VALU_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("particles") != n_particles:
        return None
    return t["valu_instructions_per_particle"]


ATOMICS_FILE = os.path.join(ROOT, "profiles", "fused_substep_large_scene_atomics.json")
ATOMICS_COMMAND = ("cd /tmp && rocprofv3 --pmc TCC_EA0_ATOMIC_sum TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum TCC_ATOMIC_sum "
                   "-f csv -d <out>/pmc_eaw -o eaw -- python3 <repo>/bench.py --steps 1 --warmup 1 "
                   "--substeps-per-step 10 --no-autotune --no-step-n --no-cpu-baseline --no-batched --no-bgdo "
                   "--no-models --no-mcis --no-ipf --no-det --no-configs --no-atomics")


def write_atomics(eaw_csv, n_particles=2_000_000):
    """Summarise the memory-side request pass of the fused kernel (global
    atomics and write requests at the L2/memory interface, mean per
    dispatch) into ATOMICS_FILE, stamped with the kernel source hash."""
    import csv
    acc = {}
    for r in csv.DictReader(open(eaw_csv)):
        if FUSED_KERNEL in r["Kernel_Name"]:
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    mean = {k: sum(v) / len(v) for k, v in acc.items()}
    out = {"kernel": FUSED_KERNEL, "particles": n_particles,
           "dispatches": len(next(iter(acc.values()))) if acc else 0,
           "global_atomic_requests": mean.get("TCC_ATOMIC_sum"),
           "global_atomic_requests_at_memory_side": mean.get("TCC_EA0_ATOMIC_sum"),
           "write_requests": mean.get("TCC_EA0_WRREQ_sum"), "write_requests_64B": mean.get("TCC_EA0_WRREQ_64B_sum"),
           "kernel_source_hash": kernel_source_hash(), "command": ATOMICS_COMMAND}
    with open(ATOMICS_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def measured_atomics(n_particles):
    """Counter summary of the fused kernel's global atomics, or None if the
    kernel sources changed since it was taken."""
    try:
        with open(ATOMICS_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("particles") != n_particles:
        return None
    return t


PMC_COMMAND = ("cd /tmp && rocprofv3 --pmc {c} -f csv -d <out>/pmc_{c} -o {c} -- python3 <repo>/bench.py "
               "--steps 1 --warmup 1 --substeps-per-step 10 --no-autotune --no-step-n --no-cpu-baseline --no-batched "
               "--no-bgdo --no-models --no-mcis --no-ipf --no-det --no-configs --no-atomics")


def write_traffic(fetch_csv: str, write_csv: str, n_particles: int = 2_000_000) -> dict:
    """Summarise two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE, in
    KiB per dispatch) of PMC_COMMAND into TRAFFIC_FILE: the 256 MiB
    calibration copy (largest copy-kernel dispatch) and the mean over the
    fused-kernel dispatches, stamped with the hash of the kernel sources."""
    import csv

    def read(path, counter):
        copy, fused = 0.0, []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"])
                if r["Kernel_Name"] == "__amd_rocclr_copyBuffer":
                    copy = max(copy, v)
                elif FUSED_KERNEL in r["Kernel_Name"]:
                    fused.append(v)
        if not fused or copy <= 0:
            raise SystemExit(f"{path}: no {counter} rows for the copy and the fused kernel")
        return copy, sum(fused) / len(fused), len(fused)

    cf, ff, nf = read(fetch_csv, "FETCH_SIZE")
    cw, fw, nw = read(write_csv, "WRITE_SIZE")
    t = {"kernel": FUSED_KERNEL + " (fused G2P + return map + stress + P2G)",
         "workload": "large_scene, 2,000,000 particles, 128^3", "particles": n_particles,
         "kernel_source_hash": kernel_source_hash(), "fused_fetch_kib": ff, "fused_write_kib": fw,
         "dispatches": min(nf, nw), "copy_bytes": 256 * 1024 * 1024, "copy_fetch_kib": cf, "copy_write_kib": cw,
         "command_fetch": PMC_COMMAND.format(c="FETCH_SIZE"), "command_write": PMC_COMMAND.format(c="WRITE_SIZE")}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
        fh.write("\n")
    return t


def bgdo_timing(sc, frames=25, substeps_per_frame=20):
    """One BGDO iteration (Alg. 1) on the workload: a gradient-free run of
    frames x substeps_per_frame substeps storing key frames {0, t, n}, one
    substep from each and the log E update.  Wall time, device-synchronised."""
    import numpy as np
    import torch

    from paper_2602_01723_amd import bgdo as BG
    from paper_2602_01723_amd import binding as B
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, p.clone(), 2)  # warm-up (allocations, first sort)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    BG.bgdo(ctx, p, frames, substeps_per_frame)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    upd = p.log_E.cpu().numpy().astype(np.float64) - sc.log_E
    return {"workload": f"same scene, {frames} frames x {substeps_per_frame} substeps, key frames "
                        f"{BG.default_key_frames(frames)}, one iteration",
            "seconds": dt, "substeps": frames * substeps_per_frame,
            "mean_log_E_update": float(upd.mean()),
            "paper_context": "39 s BGDO forward per scene on an RTX A6000 (different scenes, not comparable)"}


def deterministic_timing(sc, substeps=20, reps=3):
    """Cost of MPM_FLAG_DETERMINISTIC on the workload: resident substeps
    (mpm_advance) with and without the flag, wall time per substep
    (device-synchronised, best of reps), and whether two deterministic runs
    from the same state agree bit for bit."""
    import numpy as np
    import torch

    from paper_2602_01723_amd import binding as B
    out = {}
    finals = []
    for det in (False, True):
        best = float("inf")
        for r in range(reps):
            ctx = B.init_from_scene(sc, deterministic=det)
            p = B.Particles.from_scene(sc)
            B.mpm_load(ctx, p)
            B.mpm_advance(ctx, 1)  # primes the grid
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.mpm_advance(ctx, substeps)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
            if det and r < 2:
                B.mpm_store(ctx, p)
                torch.cuda.synchronize()
                finals.append(p.x.cpu().numpy().view(np.uint32).copy())
            del ctx, p
            torch.cuda.empty_cache()
        out["deterministic" if det else "default"] = {"ms_per_substep": best / substeps * 1e3}
    out["slowdown"] = out["deterministic"]["ms_per_substep"] / out["default"]["ms_per_substep"]
    out["repeat_bitwise_equal"] = bool(len(finals) == 2 and np.array_equal(finals[0], finals[1]))
    out["workload"] = f"same scene, mpm_advance({substeps}) after one primed substep, best of {reps}"
    return out


def deterministic_batched_timing(n_batch=64, steps=100, K=20, reps=2):
    """Cost of MPM_FLAG_DETERMINISTIC on the batched forward + loss + adjoint
    (the 64-candidate batch, fixed launch tuning, eager on one stream): wall
    time per evaluation and the mean time per launch of each timed kernel
    class, with and without the flag."""
    import torch

    from paper_2602_01723_amd import batch as BT
    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes
    sc = scenes.make_scene("candidate_batch", n_batch=n_batch, n_substeps=steps)
    tl = BT.per_particle(sc.extras["target_log_E"], sc.batch_offsets)
    tn = BT.per_particle(sc.extras["target_nu"], sc.batch_offsets)
    xt = BT.target_positions(sc, steps, tl, tn)
    out = {"workload": f"{n_batch} candidates, {sc.n} particles, {steps} substeps (checkpoints every {K}) + "
                       f"position loss + backward, eager, mean of {reps}"}
    for det in (False, True):
        ev = BT.Evaluation(sc, steps, K, xt, tuning=BATCH_TUNING, deterministic=det)
        ev.run_eager()
        torch.cuda.synchronize()
        B.mpm_profile(ev.ctx, True)
        B.mpm_profile_read(ev.ctx)
        t0 = time.perf_counter()
        for _ in range(reps):
            ev.run_eager()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        prof = B.mpm_profile_read(ev.ctx)
        out["deterministic" if det else "default"] = {
            "ms_per_evaluation": wall * 1e3,
            "us_per_launch": {k: round(v[0] / max(v[1], 1) * 1e3, 1) for k, v in prof.items() if v[1]}}
        del ev
        torch.cuda.empty_cache()
    out["slowdown"] = out["deterministic"]["ms_per_evaluation"] / out["default"]["ms_per_evaluation"]
    return out


MODEL_VARIANTS = (("fixed_corotated", 0, 0), ("hencky", 1, 0), ("neo_hookean", 2, 0), ("stvk", 3, 0),
                  ("fluid_elastic", 4, 0), ("volume", 5, 0), ("hencky+von_mises", 1, 1),
                  ("hencky+drucker_prager", 1, 2), ("fixed_corotated+fluid", 0, 3), ("hencky+sigma", 1, 4))


def per_model_timing(sc, steps=3, substeps=10):
    """Fused-kernel time (HIP events) of the same workload with every
    particle given one material, for each elastic model and return map."""
    import torch

    from paper_2602_01723_amd import binding as B
    out = {}
    for name, el, pl in MODEL_VARIANTS:
        mat = dict(elastic=el, plastic=pl, yield_stress=1e3, friction_deg=30.0)
        ctx = B.mpm_init(sc.grid_res, sc.dt, [mat] * len(sc.materials), sc.n, None, sc.gravity, sc.bound)
        p = B.Particles.from_scene(sc)
        B.mpm_step_n(ctx, p, substeps)
        torch.cuda.synchronize()
        B.mpm_profile(ctx, True)
        B.mpm_profile_read(ctx)
        for _ in range(steps):
            B.mpm_step_n(ctx, p, substeps)
        torch.cuda.synchronize()
        ms, n = B.mpm_profile_read(ctx)["fused_substep"]
        d = B.mpm_get_diagnostics(ctx)
        out[name] = {"fused_us": round(ms / max(n, 1) * 1e3, 1),
                     "particle_substeps_per_s_fused": sc.n / (ms / max(n, 1) / 1e3),
                     "nonfinite": d["nonfinite"], "out_of_grid": d["out_of_grid"]}
        del ctx, p
    return out


def mcis_timing(reps=3):
    """MCIS interior fill (Sec. 4.1) at the scale of the 2M workload: 12
    ellipsoid instances, 1M surface points, 8M inside candidates, 1M drawn.
    Wall time of mpm_mcis_select (it synchronises), best of `reps` after a
    warm-up; the oracle on a bounded sample of one instance beside it."""
    import numpy as np
    import torch

    from oracle import mpm_oracle as O
    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes
    rng = np.random.default_rng(11)
    ns = np.exp(rng.uniform(math.log(2e4), math.log(2e5), 12))
    ns = np.floor(ns * (1_000_000 / ns.sum())).astype(np.int64)
    ns[0] += 1_000_000 - ns.sum()
    d = scenes.mcis_inputs(seed=12, n_shell=tuple(int(v) for v in ns), cand_per_shell=8.0, fill_frac=0.125,
                           r_range=(0.05, 0.12))
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a.T)).cuda()
    surf, cand, u = dev(d["surface"]), dev(d["candidates"]), torch.as_tensor(d["u"]).cuda()
    args = (surf, d["surface_offsets"], cand, d["candidate_offsets"], u, d["n_select"])
    B.mpm_mcis_select(*args)
    best = math.inf
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.mpm_mcis_select(*args)
        best = min(best, time.perf_counter() - t0)
    M = int(d["candidate_offsets"][-1])
    # oracle: the first 4000 surface points and 20000 candidates of instance 0
    so, co = d["surface_offsets"], d["candidate_offsets"]
    s_n, c_n = min(4000, int(so[1])), min(20000, int(co[1]))
    t0 = time.perf_counter()
    O.mcis_select_instance(d["candidates"][:c_n], d["surface"][:s_n], d["u"][:c_n], c_n // 8)
    t_cpu = time.perf_counter() - t0
    return {"workload": "12 ellipsoid instances, 1,000,000 surface points, 8,000,000 inside candidates, "
                        "1,000,000 drawn (sigma 0.02, eps 1e-6)",
            "seconds": best, "candidates_per_s": M / best,
            "oracle": {"candidates_per_s": c_n / t_cpu, "cores": torch.get_num_threads(),
                       "sample": f"{c_n} candidates against {s_n} surface points (brute force, {t_cpu:.1f} s)"},
            "paper_context": "IPF with MCIS 22 s per scene on an RTX A6000 (with DBSCAN and hulls; not comparable)"}


def ipf_timing(reps=3):
    """Candidate generation of the interior fill (Sec. 4.1) and the whole
    fill on the GPU at the scale of the 2M workload: 12 ellipsoid instances
    with 1M hull points (their Qhull meshes), 16 raw candidates per point
    (16M), kept by the six-ray occupancy, then MCIS selects 1/8 of the kept
    ones.  Wall times (both calls synchronise), best of `reps` after a
    warm-up; the oracle on a bounded sample beside it."""
    import numpy as np
    import torch

    from oracle import mpm_oracle as O
    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes
    rng = np.random.default_rng(11)
    ns = np.exp(rng.uniform(math.log(2e4), math.log(2e5), 12))
    ns = np.floor(ns * (1_000_000 / ns.sum())).astype(np.int64)
    ns[0] += 1_000_000 - ns.sum()
    t0 = time.perf_counter()
    d = scenes.ipf_inputs(seed=13, n_shell=tuple(int(v) for v in ns), raw_per_point=16.0, r_range=(0.05, 0.12))
    t_setup = time.perf_counter() - t0
    planes = lambda a, dt: torch.as_tensor(np.ascontiguousarray(np.asarray(a, dt).reshape(-1, 3).T)).cuda()
    hv, ht, u = planes(d["hull_vertices"], np.float32), planes(d["hull_triangles"], np.int32), planes(d["u"], np.float64)
    surf = planes(d["surface"], np.float32)
    args = (hv, d["hull_vertex_offsets"], ht, d["hull_triangle_offsets"], u, d["raw_offsets"])
    cand, offs, _ = B.mpm_ipf_candidates(*args)
    M = int(offs[-1])
    u_sel = torch.rand(M, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    u_sel = 1.0 - u_sel
    n_sel = [int(v) // 8 for v in np.diff(offs)]
    B.mpm_mcis_select(surf, d["surface_offsets"], cand, offs, u_sel, n_sel)
    best_ipf = best_fill = math.inf
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cand, offs, _ = B.mpm_ipf_candidates(*args)
        t1 = time.perf_counter()
        B.mpm_mcis_select(surf, d["surface_offsets"], cand, offs, u_sel, n_sel)
        t2 = time.perf_counter()
        best_ipf, best_fill = min(best_ipf, t1 - t0), min(best_fill, t2 - t0)
    R = int(d["raw_offsets"][-1])
    T = int(d["hull_triangle_offsets"][-1])
    # oracle: 200 raw candidates of instance 0 against its whole hull
    v0, v1 = d["hull_vertex_offsets"][:2]
    t0_, t1_ = d["hull_triangle_offsets"][:2]
    lo, hi = O.ipf_box(d["hull_vertices"][v0:v1])
    q = O.ipf_points(d["u"][:200], lo, hi)
    tri = d["hull_vertices"][v0:v1][d["hull_triangles"][t0_:t1_]]
    t0 = time.perf_counter()
    O.ipf_ray_votes(q, tri)
    t_cpu = time.perf_counter() - t0
    return {"workload": f"12 ellipsoid instances, 1,000,000 hull points ({T} Qhull triangles), {R} raw "
                        f"candidates, {M} kept (occupancy > 0.6), {sum(n_sel)} drawn by MCIS",
            "ipf_seconds": best_ipf, "raw_candidates_per_s": R / best_ipf,
            "fill_seconds": best_fill, "kept": M,
            "host_setup_seconds": round(t_setup, 2),
            "oracle": {"raw_candidates_per_s": 200 / t_cpu, "cores": torch.get_num_threads(),
                       "sample": f"200 raw candidates against instance 0's {t1_ - t0_} triangles "
                                 f"(brute force, {t_cpu:.1f} s)"}}


def summarize_adjoint_counters(csv_paths, n_particles=None) -> dict:
    """Per-dispatch means of every counter in rocprofv3 --pmc runs of
    `bench.py --adjoint-counters`, per adjoint kernel, and per particle
    (the 64-candidate batch: 2,374,644 particles); FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch) are also scaled by the same counter's reading for the
    run's 256 MiB copy."""
    import csv
    n = n_particles or 2_374_644
    sums, cnts, copy = {}, {}, {}
    for path in csv_paths:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                k, c, v = r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])
                if k == "__amd_rocclr_copyBuffer":
                    copy[c] = max(copy.get(c, 0.0), v)
                    continue
                key = "k_adj_g2p" if "k_adj_g2p" in k else ("k_adj_p2g" if "k_adj_p2g" in k else None)
                if key is None:
                    continue
                sums.setdefault(key, {}).setdefault(c, 0.0)
                sums[key][c] += v
                cnts.setdefault(key, {}).setdefault(c, 0)
                cnts[key][c] += 1
    out = {"particles": n}
    for key in sums:
        d = {}
        for c in sums[key]:
            mean = sums[key][c] / cnts[key][c]
            d[c] = mean
            if c.startswith("SQ_INSTS") or c in ("SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_WAIT_INST_ANY"):
                d[c + "_per_particle"] = mean * 64.0 / n
            if c in ("FETCH_SIZE", "WRITE_SIZE") and copy.get(c):
                scale = 256 * 1024 * 1024 / (copy[c] * 1024.0)
                d[c + "_bytes_scaled"] = mean * 1024.0 * scale
                d[c + "_bytes_per_particle"] = mean * 1024.0 * scale / n
        d["dispatches"] = max(cnts[key].values())
        out[key] = d
    out["copy_calibration_kib"] = copy
    return out


def summarize_batched_trace(trace_csv: str) -> str:
    """One batched evaluation from a rocprofv3 kernel trace of --batched-only:
    the dispatches between the last two full-size position-loss kernels (the
    backward of one graph replay and the forward of the next), per kernel."""
    import collections
    import csv
    with open(trace_csv) as fh:
        rows = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
    big = [i for i, r in enumerate(rows)
           if "position_loss" in r["Kernel_Name"] and int(r["Grid_Size_X"]) >= 2_000_000]
    if len(big) < 2:
        raise SystemExit(f"{trace_csv}: fewer than two full-size position-loss dispatches")
    win = rows[big[-2]:big[-1]]
    acc = collections.defaultdict(lambda: [0, 0])
    for r in win:
        k = r["Kernel_Name"][:55]
        acc[k][0] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        acc[k][1] += 1
    tot = sum(v[0] for v in acc.values())
    wall = int(win[-1]["End_Timestamp"]) - int(win[0]["Start_Timestamp"])
    out = [f"window wall {wall / 1e6:.1f} ms, kernel sum {tot / 1e6:.1f} ms, dispatches {len(win)}"]
    for k, v in sorted(acc.items(), key=lambda kv: -kv[1][0])[:14]:
        out.append(f"{k:55s} {v[1]:6d} {v[0] / 1e6:9.2f} ms {v[0] / max(v[1], 1) / 1e3:9.1f} us "
                   f"{100 * v[0] / tot:5.1f}%")
    return "\n".join(out)


def summarize_counters(csv_paths, kernel=FUSED_KERNEL, n_particles=2_000_000) -> dict:
    """Per-dispatch means of rocprofv3 --pmc counters for `kernel`, with a few
    derived figures (wave-level instructions per particle, LDS bank-conflict
    cycles per LDS instruction cycle, share of wave time issuing VALU)."""
    import collections
    import csv
    acc = collections.defaultdict(list)
    for path in csv_paths:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if kernel in r["Kernel_Name"]:
                    acc[r["Counter_Name"]].append(float(r["Counter_Value"]))
    mean = {k: sum(v) / len(v) for k, v in acc.items()}
    out = {"kernel": kernel, "dispatches": max((len(v) for v in acc.values()), default=0), "mean": mean}
    per = lambda c: mean[c] * 64.0 / n_particles if c in mean else None
    out["valu_instructions_per_particle"] = per("SQ_INSTS_VALU")
    out["lds_instructions_per_particle"] = per("SQ_INSTS_LDS")
    if "SQ_LDS_BANK_CONFLICT" in mean and "SQ_ACTIVE_INST_LDS" in mean:
        out["lds_bank_conflict_per_active_lds_cycle"] = mean["SQ_LDS_BANK_CONFLICT"] / mean["SQ_ACTIVE_INST_LDS"]
    if "SQ_ACTIVE_INST_VALU" in mean and "SQ_WAVE_CYCLES" in mean:
        out["wave_time_issuing_valu"] = mean["SQ_ACTIVE_INST_VALU"] / mean["SQ_WAVE_CYCLES"]
    if "SQ_WAIT_INST_LDS" in mean and "SQ_WAVE_CYCLES" in mean:
        out["wave_time_waiting_lds"] = mean["SQ_WAIT_INST_LDS"] / mean["SQ_WAVE_CYCLES"]
    return out


def atomic_probe():
    """Rates of the atomic operations the fused kernel is built on, measured
    on this device in this run (libmpm_probes.so): LDS 64-bit adds with
    lane-consecutive words and in the P2G scatter's node pattern (and the
    32-bit integer and FP32 alternatives), and global FP32 adds to
    lane-distinct floats and to the 4 channels of a node."""
    from paper_2602_01723_amd import probes as P
    out = {}
    for word in ("u64", "u32", "f32"):
        for name, pat in ((f"lds_add_{word}_consecutive", 0), (f"lds_add_{word}_p2g_pattern", 1)):
            best = max(P.lds_add(pat, word)["lane_ops_per_s"] for _ in range(3))
            out[name] = best
    for name, pat in (("global_add_f32_distinct", 0), ("global_add_f32_node_channels", 1)):
        best = max(P.global_add_f32(pat)["lane_ops_per_s"] for _ in range(3))
        out[name] = best
    return {k: round(v / 1e12, 4) for k, v in out.items()} | {"unit": "T lane-ops/s"}


def copy_probe(reps=20):
    """A plain 256 MiB device copy: the calibration point of the HBM counters,
    and (timed over reps copies of the same size) the bandwidth a plain copy
    attains on this device, in GB/s of bytes read + written."""
    import torch
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    del a, b
    t = sorted(times)[len(times) // 2]
    return 2 * 256 * 1024 * 1024 / t / 1e9


def batched_setup(n_batch=64, steps=100, K=20, tuning=None):
    """The candidate batch, its targets and one Evaluation of all candidates
    in one context, autotuned (the autotuner's trial calls: forward, one
    checkpoint interval long, on the context's internal copies) unless a
    tuning is given."""
    from paper_2602_01723_amd import batch as BT
    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes
    sc = scenes.make_scene("candidate_batch", n_batch=n_batch, n_substeps=steps)
    tl = BT.per_particle(sc.extras["target_log_E"], sc.batch_offsets)
    tn = BT.per_particle(sc.extras["target_nu"], sc.batch_offsets)
    xt = BT.target_positions(sc, steps, tl, tn)
    ev = BT.Evaluation(sc, steps, K, xt, tuning=tuning)
    if tuning is None:
        tun = B.mpm_autotune(ev.ctx, ev.p, K)
        tuning = {k: tun[k] for k in ("chunk", "sort_every", "workgroups", "tile_cap")}
    log(f"  batched launch tuning: {tuning}")
    return sc, xt, ev, tuning


# launch tuning of the batched evaluation for counter runs (the autotuner's
# choice for it: 1536-particle items, 512 workgroups, a re-sort every 32
# substeps), so the profiled run carries no autotuning trials
BATCH_TUNING = {"chunk": 1536, "sort_every": 32, "workgroups": 512, "tile_cap": 1331}


def adjoint_counter_run(n_batch=64, steps=100, K=20, reps=2):
    """The batched forward + adjoint for counter runs of the adjoint kernels:
    a 256 MiB copy (the counters' calibration), the candidates with
    BATCH_TUNING, then `reps` evaluations issued eagerly on the evaluation's
    stream with a device synchronisation before and after each (no graph,
    no waits between streams)."""
    import torch
    copy_probe(reps=2)
    sc, _, ev, tuning = batched_setup(n_batch, steps, K, tuning=dict(BATCH_TUNING))
    times = []
    for _ in range(reps):
        ev.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev._record(ev.stream)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    log(f"  eager evaluation: {min(times) * 1e3:.1f} ms for {n_batch} candidates")
    return {"particles": sc.n, "substeps": steps, "eager_ms": min(times) * 1e3, "tuning": tuning}


def batched_vs_plain(n_batch=64, steps=100, K=20, reps=3):
    """Forward + adjoint of n_batch candidates (own 48^3 grid each): one
    hipGraph for the whole batch against per-candidate eager solves."""
    import numpy as np
    import torch

    from paper_2602_01723_amd import batch as BT
    sc, xt, ev, tuning = batched_setup(n_batch, steps, K)
    # the plain per-candidate solves use the batch's launch tuning
    ev.run_eager()
    torch.cuda.synchronize()
    ev.capture()
    ev.run_graph()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ev.run_graph()
        torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / reps
    gl_b, _ = ev.gradients()
    log(f"  batched: {t_batched * 1e3:.1f} ms per evaluation of {n_batch} candidates")
    # the adjoint kernels' durations: one eager evaluation with HIP events
    # around each launch (a graph replay cannot record them)
    from paper_2602_01723_amd import binding as B
    B.mpm_profile(ev.ctx, True)
    B.mpm_profile_read(ev.ctx)
    ev.run_eager()
    torch.cuda.synchronize()
    prof = B.mpm_profile_read(ev.ctx)
    B.mpm_profile(ev.ctx, False)
    adj = {}
    for cls, nbytes in (("adjoint_g2p", ADJ_G2P_BYTES), ("adjoint_p2g", ADJ_P2G_BYTES)):
        ms, cnt = prof[cls]
        if cnt:
            avg = ms / cnt * 1e-3
            adj[cls] = dict(avg_launch_us=round(avg * 1e6, 1), launches=cnt, bytes_per_particle=nbytes,
                            achieved_gbs=round(nbytes * sc.n / avg / 1e9, 1),
                            frac=round(nbytes * sc.n / avg / 1e9 / HBM_PEAK_GBS, 4))
    fwd_bwd_gbs = FWD_BWD_BYTES * sc.n * steps / t_batched / 1e9
    plain = BT.plain_evaluations(sc, steps, K, xt, tuning=tuning)
    plain[0].run_eager()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pe in plain:
        pe.run_eager()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log(f"  plain: {t_plain * 1e3:.1f} ms for {n_batch} sequential solves")
    diffs = []
    for b, pe in enumerate(plain):
        lo, hi = sc.batch_offsets[b], sc.batch_offsets[b + 1]
        g1, _ = pe.gradients()
        sb, sp = float(gl_b[lo:hi].sum()), float(g1.sum())
        diffs.append(abs(sb - sp) / max(abs(sp), 1e-30))
    return {
        "workload": f"{n_batch} candidates, one fixed-corotated ellipsoid each on its own {sc.grid_res}^3 grid, "
                    f"{int(np.diff(sc.batch_offsets).min())}-{int(np.diff(sc.batch_offsets).max())} particles, "
                    f"{steps} substeps forward + adjoint, checkpoint every {K}",
        "particles": sc.n, "substeps": steps, "tuning": {"autotuned": True, **tuning},
        "batched_grads_per_s": n_batch / t_batched, "plain_grads_per_s": n_batch / t_plain,
        "speedup": t_plain / t_batched, "batched_ms": t_batched * 1e3, "plain_ms": t_plain * 1e3,
        "fwd_bwd_particle_substeps_per_s": sc.n * steps / t_batched,
        "roofline_fwd_bwd": {"bound": "hbm", "bytes_per_particle_substep": FWD_BWD_BYTES,
                             "achieved": round(fwd_bwd_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(fwd_bwd_gbs / HBM_PEAK_GBS, 4), "kernels": adj},
        "max_rel_diff_candidate_grad_logE": max(diffs), "median_rel_diff_candidate_grad_logE": float(np.median(diffs)),
    }


def config_timings():
    """The other workloads, each on a context of its own, autotuned like the
    headline (mpm_autotune on trial calls of 20 substeps; the tuning kept is
    reported): the plain cube at its stated count (20,480 particles, 32^3;
    100 substeps through mpm_step_n), the Gaussian-scene cloud (300,000
    particles, 64^3; 1,000 substeps on the resident scene) and the
    differentiation workload (200,000 particles, 64^3; 200 substeps taped
    every 20, the position-loss cotangent and the backward: one gradient)."""
    import numpy as np
    import torch

    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes
    out = {}

    def tune(ctx, sc):
        t = B.mpm_autotune(ctx, B.Particles.from_scene(sc), 20)
        return {k: t[k] for k in ("chunk", "workgroups", "sort_every")}

    sc = scenes.make_scene("cube_uniform")
    ctx = B.init_from_scene(sc)
    tuning = tune(ctx, sc)
    p = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, p, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.mpm_step_n(ctx, p, 100)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out["cube_20480"] = dict(particles=sc.n, substeps=100, seconds=round(t, 5), particle_substeps_per_s=sc.n * 100 / t,
                             path="mpm_step_n(100)", tuning=tuning)
    del ctx, p
    sc = scenes.make_scene("gaussian_cloud")
    ctx = B.init_from_scene(sc)
    tuning = tune(ctx, sc)
    p = B.Particles.from_scene(sc)
    B.mpm_load(ctx, p)
    B.mpm_advance(ctx, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.mpm_advance(ctx, 1000)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out["gaussian_cloud_300k"] = dict(particles=sc.n, substeps=1000, seconds=round(t, 4),
                                      particle_substeps_per_s=sc.n * 1000 / t, path="mpm_load + mpm_advance(1000)",
                                      tuning=tuning)
    del ctx, p
    sc = scenes.make_scene("colliding_pair", E=(2e5, 5e4), nu=(0.25, 0.35))
    steps, K, N = sc.n_substeps, sc.checkpoint_every, sc.n
    ctx = B.init_from_scene(sc)
    tuning = tune(ctx, sc)
    tgt = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, tgt, steps)
    x_target = tgt.x.clone()
    logE = np.full(N, math.log(1e5), np.float32)
    nu = np.full(N, 0.3, np.float32)
    p = B.Particles.from_arrays(sc.x, sc.v, sc.C, sc.F, sc.mass, sc.vol0, logE, nu, sc.mat_id)
    init = p.clone()
    tape = torch.empty(B.mpm_tape_size(ctx, steps, K) // 4 + 64, device="cuda")
    w = torch.full((N,), 1.0 / (3 * N), device="cuda")
    g_x = torch.empty(3, N, device="cuda")
    gl = torch.empty(N, device="cuda")
    gn = torch.empty(N, device="cuda")

    def grad():
        for k in ("x", "v", "C", "F"):
            getattr(p, k).copy_(getattr(init, k))
        B.mpm_step_n(ctx, p, steps, tape=tape, checkpoint_every=K)
        B.mpm_position_loss_grad(ctx, p.x, x_target, w, g_x)
        B.mpm_backward(ctx, p, tape, steps, g_x=g_x, g_log_E=gl, g_nu=gn)

    grad()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        grad()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    out["colliding_pair_200k"] = dict(particles=N, substeps=steps, checkpoint_every=K, seconds_per_gradient=round(t, 4),
                                      grads_per_s=1.0 / t, fwd_bwd_particle_substeps_per_s=N * steps / t,
                                      path="mpm_step_n with tape + mpm_position_loss_grad + mpm_backward",
                                      tuning=tuning)
    del ctx, p, init, tape, tgt
    torch.cuda.empty_cache()
    out["large_domain_512"] = large_domain_timing()
    return out


def large_domain_timing(substeps=20):
    """A large, mostly empty domain: 2,000,000 particles in a cube of side
    0.125 (about 9 per occupied cell) on a 512^3 grid (134 M nodes, 2.1 GB
    per grid buffer), resident substeps with the block-sparse grid (the
    default at this size) and with dense clearing forced."""
    import torch

    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes
    sc = scenes.make_scene("cube_uniform", n=2_000_000, grid_res=512, side=0.125, centre=(0.5, 0.5, 0.5),
                           dt=2e-5)
    res = {"particles": sc.n, "grid_res": 512, "substeps": substeps,
           "path": "mpm_load + mpm_advance(1) + timed mpm_advance(substeps)"}
    for grid in ("auto", "dense"):
        ctx = B.init_from_scene(sc, grid=grid)
        p = B.Particles.from_scene(sc)
        B.mpm_load(ctx, p)
        B.mpm_advance(ctx, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.mpm_advance(ctx, substeps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        res["sparse_grid" if grid == "auto" else "dense_grid"] = dict(
            ms_per_substep=t / substeps * 1e3, particle_substeps_per_s=sc.n * substeps / t)
        del ctx, p
        torch.cuda.empty_cache()
    res["speedup"] = res["dense_grid"]["ms_per_substep"] / res["sparse_grid"]["ms_per_substep"]
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, n_sub=2):
    """The FP64 oracle on `n_sub` substeps of the full workload, on the host
    with all threads; plus one substep of a 1/16-size copy of the workload on
    a single thread (reported alongside, same unit)."""
    import torch

    from oracle import mpm_oracle as O
    from paper_2602_01723_amd import scenes

    def timed(scene, n, threads):
        saved = torch.get_num_threads()
        torch.set_num_threads(threads)
        try:
            params = O.Params.from_scene(scene)
            state = O.state_from_scene(scene)
            t0 = time.perf_counter()
            for _ in range(n):
                state = O.substep(state, params)
            return time.perf_counter() - t0
        finally:
            torch.set_num_threads(saved)

    cores = torch.get_num_threads()
    dt = timed(sc, n_sub, cores)
    small = scenes.make_scene("large_scene", n_total=max(sc.n // 16, 1000))
    dt1 = timed(small, 1, 1)
    return dict(value=sc.n * n_sub / dt, unit="particle-substeps/s", cores=cores, kind="oracle", cpu=cpu_model(),
                host_cpus=os.cpu_count(),
                sample=f"{n_sub} substeps of the full {sc.n}-particle workload from its initial state "
                       f"({dt:.1f} s, float64 PyTorch CPU)",
                one_core={"value": small.n / dt1, "cores": 1,
                          "sample": f"1 substep of the {small.n}-particle copy of the workload ({dt1:.1f} s)"})


def item_geometry(n_total=2_000_000, item=768):
    """Grid work of one fused launch implied by the work-item decomposition of
    the workload at its initial positions (host only): the library's cell
    keys (4^3-cell blocks, Morton order inside), items of at most `item`
    particles per block, and per item the G2P tile (base-cell box + 2 nodes
    per axis) and the nodes the P2G tile flushes (the union of the item's
    particles' 27-node stencils: the nodes its tile holds mass for)."""
    import numpy as np

    from paper_2602_01723_amd import scenes
    sc = scenes.make_scene("large_scene", n_total=n_total)
    n = sc.grid_res
    nb = (n + 3) // 4
    c = np.clip(np.floor(sc.x.astype(np.float64) * n - 0.5), 0, n - 1).astype(np.int64)
    blk = ((c[:, 0] >> 2) * nb + (c[:, 1] >> 2)) * nb + (c[:, 2] >> 2)

    def spread2(v):
        return (v & 1) | ((v & 2) << 2)

    key = blk * 64 + (spread2(c[:, 0] & 3) << 2 | spread2(c[:, 1] & 3) << 1 | spread2(c[:, 2] & 3))
    order = np.argsort(key, kind="stable")
    cs, bs = c[order], blk[order]
    starts = np.flatnonzero(np.r_[True, bs[1:] != bs[:-1]])
    ends = np.r_[starts[1:], len(bs)]
    item_id = np.empty(len(bs), np.int64)
    n_items = 0
    for s0, e0 in zip(starts, ends):
        item_id[s0:e0] = n_items + np.arange(e0 - s0) // item
        n_items += (e0 - s0 + item - 1) // item
    lo = np.full((n_items, 3), 1 << 30)
    hi = np.full((n_items, 3), -1)
    for a in range(3):
        np.minimum.at(lo[:, a], item_id, cs[:, a])
        np.maximum.at(hi[:, a], item_id, cs[:, a])
    g2p_nodes = int(np.prod(hi - lo + 3, 1).sum())
    n3 = n ** 3
    ic = np.unique(item_id * n3 + (cs[:, 0] * n + cs[:, 1]) * n + cs[:, 2])
    it, cl = ic // n3, ic % n3
    cx, cy, cz = cl // (n * n), (cl // n) % n, cl % n
    nodes = np.unique(np.concatenate([it * n3 + ((cx + i) * n + (cy + j)) * n + (cz + k)
                                      for i in range(3) for j in range(3) for k in range(3)]))
    active = int(len(np.unique(nodes % n3)))
    return {"workload": f"large_scene, {sc.n} particles, {n}^3, initial positions", "items": int(n_items),
            "particles_per_item": sc.n / n_items, "nodes_with_mass": active, "g2p_tile_nodes": g2p_nodes,
            "flushed_nodes": int(len(nodes)), "flush_lane_atomics": 4 * int(len(nodes)),
            "g2p_loads_per_node_with_mass": g2p_nodes / active, "flushes_per_node_with_mass": len(nodes) / active}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--substeps-per-step", type=int, default=20)
    ap.add_argument("--sort-every", type=int, default=0)
    ap.add_argument("--item", type=int, default=0, help="particles per work item (0 = library default)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch tuning instead of running mpm_autotune before warm-up "
                         "(--item / --sort-every also skip the autotuner)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched vs plain fwd+bwd comparison")
    ap.add_argument("--n-total", type=int, default=2_000_000)
    ap.add_argument("--no-bgdo", action="store_true", help="skip the BGDO iteration timing")
    ap.add_argument("--no-models", action="store_true", help="skip the per-model fused-kernel timing")
    ap.add_argument("--no-mcis", action="store_true", help="skip the MCIS interior-fill timing")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the timings of the other workloads (cube, Gaussian cloud, differentiation)")
    ap.add_argument("--no-atomics", action="store_true", help="skip the atomic-throughput probes")
    ap.add_argument("--no-step-n", action="store_true",
                    help="skip timing the same frames through mpm_step_n (caller-order I/O at every call)")
    ap.add_argument("--mcis-only", action="store_true", help="time only the MCIS interior fill and exit")
    ap.add_argument("--no-ipf", action="store_true", help="skip the candidate-generation timing")
    ap.add_argument("--no-det", action="store_true", help="skip the deterministic-mode timing")
    ap.add_argument("--det-only", action="store_true",
                    help="time only the deterministic mode (the 2M scene and the batched forward + adjoint) and exit")
    ap.add_argument("--ipf-only", action="store_true", help="time only the candidate generation and exit")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched vs plain forward + adjoint and exit")
    ap.add_argument("--adjoint-counters", action="store_true",
                    help="run the batched forward + adjoint eagerly (no graph, no plain leg) and exit: the run "
                         "that counter passes over the adjoint kernels profile")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_CSV",
                    help="per-dispatch counter means of the fused kernel from rocprofv3 --pmc runs, and exit")
    ap.add_argument("--summarize-adjoint-counters", nargs="+", metavar="PMC_CSV",
                    help="per-dispatch counter means of the adjoint kernels from rocprofv3 --pmc runs of "
                         "--adjoint-counters, and exit (no GPU use)")
    ap.add_argument("--summarize-batched-trace", metavar="TRACE_CSV",
                    help="per-kernel time of one batched evaluation in a rocprofv3 trace, and exit (no GPU use)")
    ap.add_argument("--write-valu", metavar="P1_CSV",
                    help="summarise the p1 instruction-mix counter run into the VALU file and exit (no GPU use)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs into the traffic file and exit (no GPU use)")
    ap.add_argument("--write-atomics", metavar="EAW_CSV",
                    help="summarise the memory-side request pass into the atomics file and exit (no GPU use)")
    ap.add_argument("--item-geometry", action="store_true",
                    help="count the fused launch's G2P tile loads and flushed nodes from the workload's item "
                         "geometry and exit (no GPU use)")
    args = ap.parse_args()
    if args.write_atomics:
        print(json.dumps(write_atomics(args.write_atomics, n_particles=args.n_total)))
        return
    if args.item_geometry:
        print(json.dumps(item_geometry(args.n_total, args.item or 768)))
        return
    if args.summarize_counters:
        print(json.dumps(summarize_counters(args.summarize_counters, n_particles=args.n_total), indent=1))
        return
    if args.summarize_adjoint_counters:
        print(json.dumps(summarize_adjoint_counters(args.summarize_adjoint_counters), indent=1))
        return
    if args.summarize_batched_trace:
        print(summarize_batched_trace(args.summarize_batched_trace))
        return
    if args.write_valu:
        print(json.dumps(write_valu(args.write_valu, n_particles=args.n_total)))
        return
    if args.write_traffic:
        print(json.dumps(write_traffic(*args.write_traffic, n_particles=args.n_total)))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the workload would shard by scene or by grid slab)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.mcis_only:
        print(json.dumps({"mcis": mcis_timing()}), flush=True)
        return
    if args.ipf_only:
        print(json.dumps({"ipf": ipf_timing()}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched_fwd_bwd": batched_vs_plain()}), flush=True)
        return
    if args.adjoint_counters:
        print(json.dumps({"adjoint_counter_run": adjoint_counter_run()}), flush=True)
        return
    if args.det_only:
        det = deterministic_timing(scenes.make_scene("large_scene", n_total=args.n_total))
        det["batched_fwd_bwd"] = deterministic_batched_timing()
        print(json.dumps({"deterministic": det}), flush=True)
        return
    copy_gbs = copy_probe()
    log(f"  plain 256 MiB copy: {copy_gbs:.0f} GB/s (read + write)")
    probes = None
    if not args.no_atomics:
        probes = atomic_probe()
        log(f"  atomic probes: {probes}")
    log("generating workload ...")
    t = time.perf_counter()
    sc = scenes.make_scene("large_scene", n_total=args.n_total)
    log(f"  {sc.n} particles, {sc.grid_res}^3 grid, generated in {time.perf_counter() - t:.1f} s")

    torch.cuda.synchronize()
    free0, total_mem = torch.cuda.mem_get_info()
    ctx = B.init_from_scene(sc, sort_every=args.sort_every)
    if args.item:
        B.mpm_set_tuning(ctx, chunk=args.item)
    p = B.Particles.from_scene(sc)
    S = args.substeps_per_step
    autotuned = not (args.no_autotune or args.item or args.sort_every)
    if autotuned:  # untimed, before warm-up: trial calls of S substeps on internal copies
        t = time.perf_counter()
        tun = B.mpm_autotune(ctx, p, S)
        log(f"  autotuned in {time.perf_counter() - t:.1f} s: {tun}")
    tuning = B.mpm_get_tuning(ctx)
    # one step = one render frame: S substeps of the scene held in the
    # context (mpm_load, untimed, before warm-up), then the frame's positions
    # and Gaussian covariances F Sigma0 F^T in the caller's order
    cov0 = torch.tensor(np.ascontiguousarray(sc.cov0.T)).cuda()
    x_out = torch.empty(3, sc.n, device="cuda")
    cov_out = torch.empty(6, sc.n, device="cuda")

    def frame():
        B.mpm_advance(ctx, S)
        B.mpm_export_frame(ctx, x_out, cov0, cov_out)

    B.mpm_load(ctx, p)
    for w in range(args.warmup):
        frame()
        torch.cuda.synchronize()
        log(f"  warmup step {w + 1}/{args.warmup} done")

    B.mpm_profile(ctx, True)
    B.mpm_profile_read(ctx)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        frame()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.mpm_profile_read(ctx)
    B.mpm_profile(ctx, False)
    elapsed = t1 - t0
    log(f"  timed {args.steps} steps x {S} substeps in {elapsed:.3f} s")

    diag = B.mpm_get_diagnostics(ctx)
    free1, _ = torch.cuda.mem_get_info()  # context, particles and grids of the workload
    m, _, _ = B.grid_state(ctx)
    active = int((m > 0).sum().item())
    torch.cuda.synchronize()
    step_n = None
    if not args.no_step_n:
        # the same frames through mpm_step_n: the caller's x, v, C, F and
        # parameters in and x, v, C, F out at every call
        B.mpm_step_n(ctx, p, S)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for k in range(args.steps):
            B.mpm_step_n(ctx, p, S)
        torch.cuda.synchronize()
        te = time.perf_counter() - ts
        step_n = dict(value=sc.n * S * args.steps / te, ms_per_step=te / args.steps * 1e3,
                      what="mpm_step_n per step: caller-order arrays in and out at every call, no frame export")
        log(f"  mpm_step_n path: {step_n['value']:.3e} particle-substeps/s")

    value = sc.n * S * args.steps / elapsed
    fused_ms, fused_n = prof["fused_substep"]
    fused_avg_s = fused_ms / max(fused_n, 1) / 1e3
    bytes_launch = BYTES_PER_PARTICLE * sc.n + BYTES_PER_ACTIVE_NODE * active
    achieved = bytes_launch / fused_avg_s / 1e9 if fused_n else None
    traffic = measured_traffic(sc.n)
    roofline = dict(bound="hbm", kernel="k_substep<fused>", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=(achieved / HBM_PEAK_GBS) if achieved else None, traffic=traffic,
                    bytes_per_launch=bytes_launch, avg_launch_us=fused_avg_s * 1e6, launches=fused_n,
                    active_nodes=active, copy_attained=copy_gbs,
                    frac_of_copy=(achieved / copy_gbs) if achieved else None)
    # what does bound the kernel: VALU issue (counter-measured instructions
    # per particle over the live launch time, against the issue peak)
    ipp = measured_valu(sc.n)
    if ipp and fused_n:
        issued = ipp * sc.n / fused_avg_s
        roofline["valu_issue"] = dict(instructions_per_particle=ipp, achieved=issued / 1e12,
                                      peak=VALU_PEAK_LANE_INSTR / 1e12, unit="T lane-instructions/s",
                                      frac=issued / VALU_PEAK_LANE_INSTR)
    # atomic throughput of the fused kernel: its LDS adds (108 per particle)
    # over the launch, against the probes' rates on this device
    if probes and fused_n:
        lds_rate = LDS_ADDS_PER_PARTICLE * sc.n / fused_avg_s / 1e12
        roofline["atomics"] = dict(
            lds_add_u64_per_launch=LDS_ADDS_PER_PARTICLE * sc.n, lds_achieved=round(lds_rate, 4),
            lds_peak_p2g_pattern=probes["lds_add_u64_p2g_pattern"],
            lds_peak_consecutive=probes["lds_add_u64_consecutive"],
            lds_frac_of_p2g_pattern=round(lds_rate / probes["lds_add_u64_p2g_pattern"], 4),
            global_add_f32_peak_node_channels=probes["global_add_f32_node_channels"],
            global_add_f32_peak_distinct=probes["global_add_f32_distinct"], unit="T lane-ops/s",
            note="LDS adds averaged over the whole launch; the P2G scatter is about a third of it")
        ga = measured_atomics(sc.n)
        if ga and ga.get("global_atomic_requests"):
            # the tile flushes' float atomics, counted at the L2 (TCC_ATOMIC) and at
            # the memory side (TCC_EA0_ATOMIC): every one is performed there
            roofline["atomics"].update(
                global_atomic_requests_per_launch=round(ga["global_atomic_requests"]),
                global_atomic_requests_achieved=round(ga["global_atomic_requests"] / fused_avg_s / 1e9, 2),
                global_atomic_requests_unit="G requests/s",
                global_atomics_at_memory_side=round(ga["global_atomic_requests_at_memory_side"] /
                                                    ga["global_atomic_requests"], 4))
    breakdown = {k: dict(ms=round(v[0], 3), launches=v[1]) for k, v in prof.items() if v[1]}
    log("  kernel time by class:", json.dumps(breakdown))
    log("  diagnostics:", diag)

    del ctx, p
    torch.cuda.empty_cache()
    bgdo = None
    if not args.no_bgdo:
        log("one BGDO iteration ...")
        bgdo = bgdo_timing(sc)
        log(f"  {bgdo['seconds']:.3f} s for {bgdo['substeps']} substeps + 3 key frames")
        torch.cuda.empty_cache()
    models = None
    if not args.no_models:
        log("fused kernel per constitutive model ...")
        models = per_model_timing(sc)
        log("  " + ", ".join(f"{k} {v['fused_us']} us" for k, v in models.items()))
        torch.cuda.empty_cache()
    mcis = None
    if not args.no_mcis:
        log("MCIS interior fill ...")
        mcis = mcis_timing()
        log(f"  {mcis['seconds'] * 1e3:.1f} ms for 8M candidates")
        torch.cuda.empty_cache()
    det = None
    if not args.no_det:
        log("deterministic mode ...")
        det = deterministic_timing(sc)
        log(f"  {det['deterministic']['ms_per_substep']:.3f} vs {det['default']['ms_per_substep']:.3f} ms per "
            f"substep, repeat bitwise equal: {det['repeat_bitwise_equal']}")
        torch.cuda.empty_cache()
    ipf = None
    if not args.no_ipf:
        log("candidate generation + interior fill ...")
        ipf = ipf_timing()
        log(f"  {ipf['ipf_seconds'] * 1e3:.1f} ms for {ipf['raw_candidates_per_s'] * ipf['ipf_seconds']:.0f} raw "
            f"candidates, fill {ipf['fill_seconds'] * 1e3:.1f} ms")
        torch.cuda.empty_cache()
    batched = None
    if not args.no_batched:
        log("batched vs plain forward + adjoint ...")
        batched = batched_vs_plain()
        log(f"  {batched['batched_grads_per_s']:.2f} vs {batched['plain_grads_per_s']:.2f} candidate gradients/s")

    configs = None
    if not args.no_configs:
        log("other workloads ...")
        configs = config_timings()
        log("  " + json.dumps(configs))
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline(scenes.make_scene("large_scene", n_total=args.n_total))
        log(f"  oracle: {cpu['value']:.3e} particle-substeps/s on {cpu['cores']} threads, "
            f"{cpu['one_core']['value']:.3e} on 1")

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
            "particles": sc.n, "grid_res": sc.grid_res, "substeps_per_step": S,
            "tuning": {"autotuned": autotuned, **{k: tuning[k] for k in ("chunk", "sort_every", "workgroups",
                                                                         "tile_cap")}},
            "step": "mpm_advance(S) + mpm_export_frame (x and covariances in the caller's order) on the "
                    "scene held in the context; mpm_load untimed, before warm-up",
            "kernel_time_by_class_ms": breakdown,
            "diagnostics": {k: diag[k] for k in ("nonfinite", "out_of_grid", "tile_overflow", "tile_escapes")},
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_n_caller_order": step_n,
        "batched_fwd_bwd": batched,
        "other_workloads": configs,
        "bgdo": bgdo,
        "per_model_fused": models,
        "mcis": mcis,
        "ipf": ipf,
        "deterministic": det,
        "device_memory_gb": round((free0 - free1) / 1e9, 3),
        "paper_context": {
            "figure": "about 1 minute and 7 GB per scene for the whole pipeline (IPF 22 s, BGDO forward "
                      "39 s, backward under 1 s), 1x NVIDIA RTX A6000 48 GB (Table 1)",
            "comparable": False,
            "why": "the paper's scenes, particle counts, substeps and precision are not given; the "
                   "workloads here are synthetic stand-ins"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
