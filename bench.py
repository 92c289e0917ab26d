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


KERNEL_SOURCES = ("paper_2602_01723_amd/csrc/mpm_kernels.hpp", "paper_2602_01723_amd/csrc/mpm_math.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_substep_large_scene_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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
                "--no-step-n --no-cpu-baseline --no-batched --no-bgdo --no-models --no-mcis")


def write_valu(p1_csv, n_particles=2_000_000):
    """Summarise the p1 instruction-mix pass (SQ_INSTS_VALU) of the fused
    kernel into VALU_FILE, stamped with the kernel source hash."""
    c = summarize_counters([p1_csv], n_particles=n_particles)
    out = {"kernel": "k_substep<1>", "particles": n_particles, "dispatches": c["dispatches"],
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


PMC_COMMAND = ("cd /tmp && rocprofv3 --pmc {c} -f csv -d <out>/pmc_{c} -o {c} -- python3 <repo>/bench.py "
               "--steps 1 --warmup 1 --substeps-per-step 10 --no-autotune --no-step-n --no-cpu-baseline --no-batched "
               "--no-bgdo --no-models --no-mcis")


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
                elif "k_substep<1>" in r["Kernel_Name"]:
                    fused.append(v)
        if not fused or copy <= 0:
            raise SystemExit(f"{path}: no {counter} rows for the copy and the fused kernel")
        return copy, sum(fused) / len(fused), len(fused)

    cf, ff, nf = read(fetch_csv, "FETCH_SIZE")
    cw, fw, nw = read(write_csv, "WRITE_SIZE")
    t = {"kernel": "k_substep<1> (fused G2P + return map + stress + P2G)",
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


def summarize_counters(csv_paths, kernel="k_substep<1>", n_particles=2_000_000) -> dict:
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


def batched_setup(n_batch=64, steps=100, K=20):
    """The candidate batch, its targets and one Evaluation of all candidates
    in one context, autotuned (the autotuner's trial calls: forward, one
    checkpoint interval long, on the context's internal copies)."""
    from paper_2602_01723_amd import batch as BT
    from paper_2602_01723_amd import binding as B
    from paper_2602_01723_amd import scenes
    sc = scenes.make_scene("candidate_batch", n_batch=n_batch, n_substeps=steps)
    tl = BT.per_particle(sc.extras["target_log_E"], sc.batch_offsets)
    tn = BT.per_particle(sc.extras["target_nu"], sc.batch_offsets)
    xt = BT.target_positions(sc, steps, tl, tn)
    ev = BT.Evaluation(sc, steps, K, xt)
    tun = B.mpm_autotune(ev.ctx, ev.p, K)
    tuning = {k: tun[k] for k in ("chunk", "sort_every", "workgroups", "tile_cap")}
    log(f"  batched launch tuning: {tuning}")
    return sc, xt, ev, tuning


def batched_graph_only(n_batch=64, steps=100, K=20, reps=3):
    """The batched forward + adjoint graph alone (for counter runs of the
    adjoint kernels): capture, then `reps` replays."""
    import torch
    sc, _, ev, tuning = batched_setup(n_batch, steps, K)
    ev.capture()
    ev.run_graph()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ev.run_graph()
        torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    log(f"  batched: {t * 1e3:.1f} ms per evaluation of {n_batch} candidates")
    return {"particles": sc.n, "substeps": steps, "batched_ms": t * 1e3, "tuning": tuning}


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
        "max_rel_diff_candidate_grad_logE": max(diffs), "median_rel_diff_candidate_grad_logE": float(np.median(diffs)),
    }


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
    return dict(value=sc.n * n_sub / dt, unit="particle-substeps/s", cores=cores, kind="oracle",
                sample=f"{n_sub} substeps of the full {sc.n}-particle workload from its initial state "
                       f"({dt:.1f} s, float64 PyTorch CPU)",
                one_core={"value": small.n / dt1, "cores": 1,
                          "sample": f"1 substep of the {small.n}-particle copy of the workload ({dt1:.1f} s)"})


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
    ap.add_argument("--no-step-n", action="store_true",
                    help="skip timing the same frames through mpm_step_n (caller-order I/O at every call)")
    ap.add_argument("--mcis-only", action="store_true", help="time only the MCIS interior fill and exit")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched vs plain forward + adjoint and exit")
    ap.add_argument("--adjoint-counters", action="store_true",
                    help="replay only the batched forward + adjoint graph (no plain leg) and exit: the run "
                         "that counter passes over the adjoint kernels profile")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PMC_CSV",
                    help="per-dispatch counter means of the fused kernel from rocprofv3 --pmc runs, and exit")
    ap.add_argument("--summarize-batched-trace", metavar="TRACE_CSV",
                    help="per-kernel time of one batched evaluation in a rocprofv3 trace, and exit (no GPU use)")
    ap.add_argument("--write-valu", metavar="P1_CSV",
                    help="summarise the p1 instruction-mix counter run into the VALU file and exit (no GPU use)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs into the traffic file and exit (no GPU use)")
    args = ap.parse_args()
    if args.summarize_counters:
        print(json.dumps(summarize_counters(args.summarize_counters, n_particles=args.n_total), indent=1))
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
    if args.batched_only:
        print(json.dumps({"batched_fwd_bwd": batched_vs_plain()}), flush=True)
        return
    if args.adjoint_counters:
        print(json.dumps({"batched_graph": batched_graph_only()}), flush=True)
        return
    copy_gbs = copy_probe()
    log(f"  plain 256 MiB copy: {copy_gbs:.0f} GB/s (read + write)")
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
    batched = None
    if not args.no_batched:
        log("batched vs plain forward + adjoint ...")
        batched = batched_vs_plain()
        log(f"  {batched['batched_grads_per_s']:.2f} vs {batched['plain_grads_per_s']:.2f} candidate gradients/s")

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
        "bgdo": bgdo,
        "per_model_fused": models,
        "mcis": mcis,
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
