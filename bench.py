#!/usr/bin/env python3
"""Benchmark of the MeshBlock hydro update on one MI355X.

Workload: a 128^3 periodic domain as 64 MeshBlocks of 32^3 cells with the
Saha H/He table EOS and dual energy (cold Mach-1e7 Gaussian stream), FP64.
One step = one pass of the whole hot path: the CFL reduction (per-block
minimum, global minimum, level assignment) and one RK2 step of every block
(two stage launches with PLM, table EOS inversion, HLLC, divergence, dual
energy update), inputs resident in HBM.

Prints one JSON line.  `value` is the cell-updates/s of the learned form:
one launch per RK phase for all levels; before the second stage a pass finds
the table cell of every cell's state by a search started from the learned
network's prediction (the network runs on the matrix cores; it is trained
first on the GPU by the library's own kernels, training time reported, not
timed), and that cell seeds the stage's face and compression queries of the
cell; the first stage takes the cells the previous step's second stage (or
the CFL reduction) recorded, and after a step the reduction reduces the CFL
minima that step's second stage left.  Beside it: the same with the network inside the stage kernel, seeding
the next stage from the output states (learned_inkernel), the temporal form
(searches start from the input state's cell), the chained form (the pass
bisects), the plain form (bisection for every query, one launch per level)
and the learned form with the HLLE solver; all but the last give
bit-identical states.  Each form runs --warmup steps, then --repeats timed
runs of exactly --steps steps each (the state evolving on); its rate is that
of the median run.  The roofline
entry is for the stage kernel (HIP events on the library's stream); the CPU
baseline is the FP64 oracle on the host, on a bounded number of steps of the
same workload, and its final state doubles as the accuracy check of the GPU
run.

The "lat" object times whole LAT windows (CFL reduction, level assignment,
2^Lmax sub-cycles) on the full-size polytrope (ideal gas, fixed potential) and
on the production-shaped mesh (4096 mixed 16^3/32^3 blocks, table EOS, point
mass): the batched forms (one launch per RK phase for all active levels,
window captured in a hipGraph) beside the plain form (one launch per level).
It reports cell-updates/s from the library's update counters and the
sync-equivalent rate (cells x 2^Lmax per window over the time), which shows
the work LAT saves.  The "gravity" object times the self-gravity multigrid on
the 256^3 Jeans wave (V-cycles and the solve-every-step coupled update), the
"remap" object the restart remap of the 128^3 stream onto a 256^3 grid.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 vector instruction per SIMD
# every 4 cycles (16 lanes; FP64 FMA at this rate is the 78.6 TFLOP/s vector peak)
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def counters_from_profiles(workload, family="stage"):
    """Counter summary of the stage kernel (HBM bytes, SQ counters per launch)
    or of the multigrid kernels (HBM bytes per V-cycle) if it was taken on the
    current kernel source; else {}."""
    name = f"stage_traffic_{workload}.json" if family == "stage" else f"multigrid_traffic_{workload}.json"
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return {}
    from paper_2609_37859_amd.profile_summary import kernel_source_hash
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_source_hash(family):
        return {}
    return d


FORMS = {
    "learned": "batched launches; before the second stage a pass finds the table cell of every cell's state by "
               "a search started from the learned network's prediction; it seeds the cell's face and "
               "compression queries (the first stage takes the cells the last second stage recorded)",
    "learned_inkernel": "batched launches; each stage finds the table cells of its output states by searches "
                        "started from the learned network's prediction inside the stage kernel; they seed the "
                        "next stage's face and compression queries",
    "temporal": "batched launches; each stage finds the table cells of its output states by searches started "
                "from its input states' cells; they seed the next stage's queries",
    "chained": "batched launches; before the second stage the table cell of every cell's state is bisected; it "
               "seeds the cell's face and compression queries (the first stage takes the cells the last second "
               "stage recorded)",
    "plain": "one launch per level; bisection for every table query",
    "learned_hlle": "the learned form with the HLLE Riemann solver of the paper's production runs",
}


def train_seed(T, W, table, steps=2000, nsamples=1 << 20, nquery=1 << 24):
    """Train the learned seed on the GPU with the library's kernels: 2^20
    samples, labels from the library's table inversion.  Then evaluate it on
    2^24 fresh queries of the same distribution: |dlogT| percentiles of the
    prediction, the histogram of secant steps of the seeded searches (-1: the
    seed did not lead to the bracketing cell within the step limit and
    bisection decided), and the time per query of the batched inversion with
    and without the seed (same cells, checked).  Returns (params, seconds,
    final loss, evaluation dict)."""
    import torch
    cfg = W.Config(eos_kind=1, e_floor=table.e_floor)
    mesh = W.uniform_mesh(1, 1, 1, 8, 1.0)
    ctx = T.Context(cfg, mesh, W.uniform_state(mesh, W.Config()), table=table)
    x = torch.from_numpy(W.seed_training_samples(table, nsamples, 1)).cuda()
    lT, _, _ = ctx.eos_invert(x[:, 0].contiguous(), x[:, 1].contiguous(), mode=0)
    ctx.mlp_init(W.mlp_init_params(2), W.seed_ranges(table))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = ctx.mlp_train(x, lT, steps=steps, batch=4096, lr=1e-3, seed=1)
    secs = time.perf_counter() - t0
    xq = torch.from_numpy(W.seed_training_samples(table, nquery, 3)).cuda()
    qr, qe = xq[:, 0].contiguous(), xq[:, 1].contiguous()
    lq, j0, _ = ctx.eos_invert(qr, qe, mode=0)
    err = (ctx.mlp_forward(xq) - lq).abs().cpu().numpy()
    q = {f"p{p}": float(np.percentile(err, p)) for p in (50, 90, 99, 99.99)}
    q["max"] = float(err.max())
    ctx.mlp_enable_seed(True)
    ns = {}
    for mode in (0, 1):
        ctx.eos_invert(qr, qe, mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            out = ctx.eos_invert(qr, qe, mode=mode)
        torch.cuda.synchronize()
        ns[mode] = 1e9 * (time.perf_counter() - t0) / (5 * nquery)
    l1, j1, it1 = out
    if not (torch.equal(j0, j1) and torch.equal(lq, l1)):
        raise SystemExit("seeded inversion differs from the table-only one")
    hist = np.bincount(it1.cpu().numpy().astype(np.int64) + 1)
    q["queries"] = nquery
    q["secant_steps_histogram"] = {str(k - 1): int(v) for k, v in enumerate(hist) if v}
    q["bisection_fallback_rate"] = float(hist[0]) / nquery
    q["ns_per_query_table_only"] = ns[0]
    q["ns_per_query_seeded"] = ns[1]
    params = ctx.mlp_params()
    ctx.close()
    return params, secs, float(loss[-1]), q


def run_form(T, W, cfg, mesh, U, table, steps, warmup, inv_mode, batched, seed_params=None, tile=-1, riemann=0,
             repeats=3):
    """Time `steps` steps `repeats` times in a row (the state evolves on) and
    return the median elapsed time: a single host or clock hiccup inside one
    timed run does not decide the rate."""
    import torch
    ctx = T.Context(dataclasses.replace(cfg, riemann=riemann), mesh, U, table=table, inv_mode=inv_mode)
    if seed_params is not None:
        ctx.mlp_init(seed_params, W.seed_ranges(table))
        ctx.mlp_enable_seed(True)
    if tile >= 0:
        ctx.set_tile(tile)
    else:
        ctx.autotune(reps=2)
    for _ in range(warmup):
        _, dt0, lev, L = ctx.reduce_dt()
        ctx.run_window(dt0 * 2 ** L, batched=batched)
    ctx.sync()
    ctx.set_timing(True)
    els = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, dt0, lev, L = ctx.reduce_dt()
            ctx.run_window(dt0 * 2 ** L, batched=batched)
        ctx.sync()
        torch.cuda.synchronize()
        els.append(time.perf_counter() - t0)
    el = sorted(els)[len(els) // 2]
    stage_ms, launches = ctx.stage_time()
    st = ctx.stats()
    tile = ctx.get_tile()
    ctx.close()
    return el, stage_ms, launches, st, tile


def run_lat(T, W, cfg, mesh, U, windows, warmup, inv_mode=0, batched=True, graph=False, table=None, phi=None,
            seed_params=None):
    """LAT windows (reduce_dt, level assignment, one window of 2^Lmax sub-cycles)
    timed end to end; returns rates from the library's own update counters."""
    import torch
    ctx = T.Context(cfg, mesh, U, phi=phi, table=table, inv_mode=inv_mode)
    if seed_params is not None:
        ctx.mlp_init(seed_params, W.seed_ranges(table))
        ctx.mlp_enable_seed(True)
    ctx.autotune(reps=3)
    for _ in range(warmup):
        _, dt0, lev, L = ctx.reduce_dt()
        ctx.run_window(dt0 * 2 ** L, batched=batched, graph=graph)
    ctx.sync()
    st0 = ctx.stats()
    sync_equiv = 0
    hist = np.zeros(8, dtype=np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(windows):
        _, dt0, lev, L = ctx.reduce_dt()
        ctx.run_window(dt0 * 2 ** L, batched=batched, graph=graph)
        sync_equiv += mesh.ncells * 2 ** L
        hist[:len(np.bincount(lev))] += np.bincount(lev)
    ctx.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st1 = ctx.stats()
    tile = T.tile_shapes()[ctx.get_tile()]
    ctx.close()
    cu = st1["cell_updates"] - st0["cell_updates"]
    bu = st1["block_updates"] - st0["block_updates"]
    return {"value": cu / el, "sync_equivalent": sync_equiv / el, "ms_per_window": 1e3 * el / windows,
            "windows": windows, "block_updates": int(bu), "block_updates_sync": int(sync_equiv // mesh.ncells *
                                                                                      mesh.nblocks),
            "levels": [int(v) for v in np.trim_zeros(hist, "b")], "tile": tile}


def lat_section(T, W, table, seed_params, windows, warmup):
    """LAT-batched forms beside the plain per-level form on the two LAT workloads."""
    out = {}
    cfg, mesh, U, phi, info = W.polytrope_c3()
    cfg = dataclasses.replace(cfg, merge_frac=0.01)  # performance runs merge sparse top bins
    out["polytrope"] = {
        "workload": "256^3 as 512 MeshBlocks of 32^3, n=1.5 polytrope (1 Msun, 1 Rsun) in a 1e-10 atmosphere, fixed "
                    "potential, ideal gas, N_LAT=3, merge_frac 0.01, outflow",
        "batched_graph": run_lat(T, W, cfg, mesh, U, windows, warmup, batched=True, graph=True, phi=phi),
        "plain": run_lat(T, W, cfg, mesh, U, windows, warmup, batched=False, graph=False, phi=phi)}
    cfg, mesh, U = W.debris_stream_c5(table)
    cfg = dataclasses.replace(cfg, merge_frac=0.01)
    out["production"] = {
        "workload": "4096 MeshBlocks (1688 x 32^3 + 2408 x 16^3, 65.2M cells), Saha table EOS, dual energy, "
                    "1e3 Msun point mass with excision in a moving frame, debris stream, N_LAT=3, merge_frac 0.01",
        "learned": run_lat(T, W, cfg, mesh, U, windows, warmup, inv_mode=4, batched=True, graph=True, table=table,
                           seed_params=seed_params),
        "temporal": run_lat(T, W, cfg, mesh, U, windows, warmup, inv_mode=3, batched=True, graph=True,
                            table=table),
        "learned_dense_ghosts": run_lat(T, W, dataclasses.replace(cfg, ghost_dense=1), mesh, U, windows, warmup,
                                        inv_mode=4, batched=True, graph=True, table=table, seed_params=seed_params),
        "plain": run_lat(T, W, cfg, mesh, U, windows, warmup, inv_mode=0, batched=False, graph=False,
                         table=table)}
    return out


def mg_bytes_per_cycle(levels):
    """Algorithmic HBM bytes of one multigrid cycle: per cell of every level but
    the coarsest, four sweeps (read phi and the source, write phi: 24 B each),
    the restriction of the solution and of the defect computed on the fly
    (16 B read, 3 B written per fine cell), the coarse source and correction
    passes (3 + 3 B per fine cell) and the prolongation (16 B read-modify-write,
    1 B of coarse reads); on the finest level the extra sweep and the defect
    norm (24 + 16 B)."""
    n = [a * b * c for a, b, c in levels]
    return 138 * sum(n[:-1]) + 40 * n[0]


def gravity_section(T, W, cycles, steps):
    """Self-gravity multigrid on the linear Jeans wave at 256^3 (the paper's
    Jeans-test grid): time per V-cycle (fixed cycles, warm start) and the
    coupled update (a solve to an RMS defect of 1e-10 at every step)."""
    import torch
    cfg, mesh, U, phi0, fpg = W.jeans_wave(nx=256, nt=256, n=32)
    ctx = T.Context(cfg, mesh, U, phi=phi0)
    c0, d0 = ctx.gravity_solve(fpg, 4, warm=False)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, d = ctx.gravity_solve(fpg, cycles, tol=0.0, warm=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    levels = [(mesh.nx, mesh.ny, mesh.nz)]  # every axis halves while all are at least 4
    while min(levels[-1]) >= 4:
        levels.append(tuple(v // 2 for v in levels[-1]))
    ms = 1e3 * el / cycles
    nbytes = mg_bytes_per_cycle(levels)
    achieved = nbytes / (ms * 1e-3) / 1e9
    traffic = None
    prof = counters_from_profiles("jeans256", family="gravity")
    if prof.get("hbm_bytes_per_unit"):
        traffic = prof["hbm_bytes_per_unit"]
    if steps <= 0:
        ctx.close()
        return {"ms_per_vcycle": ms, "vcycles_timed": cycles}
    # the coupled update: solve (warm, RMS defect <= 1e-10), CFL, one RK2 step
    for _ in range(2):
        ctx.gravity_solve(fpg, 20, tol=1e-10, warm=True)
        _, dt, _, _ = ctx.reduce_dt()
        ctx.step_level(0, dt)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ncyc = 0
    for _ in range(steps):
        k, _ = ctx.gravity_solve(fpg, 20, tol=1e-10, warm=True)
        ncyc += k
        _, dt, _, _ = ctx.reduce_dt()
        ctx.step_level(0, dt)
    ctx.sync()
    torch.cuda.synchronize()
    el2 = time.perf_counter() - t0
    ctx.close()
    return {"workload": "256^3 periodic as 512 MeshBlocks of 32^3, linear Jeans wave (lambda/lambda_J = 0.8, "
                        "amplitude 1e-3), ideal gas gamma 5/3",
            "levels": levels, "ms_per_vcycle": ms, "vcycles_timed": cycles,
            "defect_contraction": float((d[-1] / d[0]) ** (1.0 / cycles)) if d[0] > 0 else None,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "mg_* (one V-cycle)",
                         "algorithmic_bytes_per_vcycle": nbytes},
            "coupled": {"value": mesh.ncells * steps / el2, "unit": "cell-updates/s", "steps": steps,
                        "ms_per_step": 1e3 * el2 / steps, "vcycles_per_solve": ncyc / steps,
                        "form": "per step: multigrid solve to an RMS defect of 1e-10 (warm start), CFL reduction, "
                                "one RK2 step with the solved potential"}}


def remap_section(T, W, table, reps):
    """Restart remap of the 128^3 table-EOS stream onto a grid twice as fine
    (256^3 as 512 x 32^3, origin shifted by a quarter source cell), timed over
    reps remaps; HBM roof on the algorithmic bytes (every target value written
    once, every source value read once)."""
    import torch
    cfg, mesh, U = W.stream_c2(table)
    dx = mesh.dx[0] / 2
    dst = W.uniform_mesh(8, 8, 8, 32, dx, x0=tuple(x + 0.25 * mesh.dx[0] for x in mesh.x0))
    a = T.Context(cfg, mesh, U, table=table)
    b = T.Context(cfg, dst, W.uniform_state(dst, cfg), table=table)
    b.remap_from(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.remap_from(a)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    a.close()
    b.close()
    nbytes = 8 * cfg.nv * (dst.ncells + mesh.ncells)
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"workload": "128^3 table-EOS stream (dual energy) remapped onto 256^3 (512 x 32^3, dx/2, origin shifted "
                        "by a quarter source cell): 8 sub-cell samples of the trilinear interpolant per target cell",
            "ms_per_remap": ms, "target_cells_per_s": dst.ncells / (ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes": nbytes}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed runs of --steps steps per form; each form reports the median run")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps for the CPU baseline / accuracy check")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="learned,temporal,chained,plain,learned_hlle,learned_inkernel",
                    help="comma list of forms to time: learned, temporal, chained, plain, learned_hlle, "
                         "learned_inkernel (learned is the headline when present)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="stage-kernel variant id to use instead of autotuning (profiling runs fix it)")
    ap.add_argument("--lat-windows", type=int, default=5,
                    help="timed LAT windows per form on the polytrope and production-shaped workloads (0: skip)")
    ap.add_argument("--gravity-cycles", type=int, default=10,
                    help="timed multigrid V-cycles on the 256^3 Jeans wave (0: skip the self-gravity section)")
    ap.add_argument("--gravity-steps", type=int, default=10,
                    help="timed coupled steps (solve + RK2 step) on the 256^3 Jeans wave (0: skip them)")
    ap.add_argument("--remap-reps", type=int, default=5, help="timed restart remaps (0: skip the remap section)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2609_37859_amd import tdh as T
    from paper_2609_37859_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    T.lib()

    table = W.saha_table()
    cfg, mesh, U = W.stream_c2(table)
    ncell = mesh.ncells
    nv = cfg.nv

    # accuracy check and CPU baseline on the same bounded sample
    acc = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from tests.parity import rel_err
        ctx = T.Context(cfg, mesh, U, table=table, inv_mode=2)
        dts = T.run_sync_steps(ctx, args.cpu_steps)
        g = ctx.get_state()
        ctx.close()
        t0 = time.perf_counter()
        o, _ = oracle.run_sync(cfg, mesh, U, args.cpu_steps, table=table, dts=dts)
        cpu_s = time.perf_counter() - t0
        acc = float(np.max(rel_err(nv, mesh, g, o)))
        cpu = {"value": ncell * args.cpu_steps / cpu_s, "unit": "cell-updates/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{args.cpu_steps} RK2 steps of the full 128^3 workload (GPU step sizes), {cpu_s:.1f} s"}

    forms = args.forms.split(",")
    params, train_s, train_loss, seed_err = train_seed(T, W, table)
    res = {}
    for name, mode, batched, riemann in (("learned", 4, True, 0), ("temporal", 3, True, 0), ("chained", 2, True, 0),
                                         ("plain", 0, False, 0), ("learned_hlle", 4, True, 1),
                                         ("learned_inkernel", 1, True, 0)):
        if name in forms:
            res[name] = run_form(T, W, cfg, mesh, U, table, args.steps, args.warmup, inv_mode=mode, batched=batched,
                                 seed_params=params if mode in (1, 4) else None, tile=args.tile, riemann=riemann,
                                 repeats=args.repeats)
    lat = lat_section(T, W, table, params, args.lat_windows, 1) if args.lat_windows > 0 else None
    grav = gravity_section(T, W, args.gravity_cycles, args.gravity_steps) if args.gravity_cycles > 0 else None
    remap = remap_section(T, W, table, args.remap_reps) if args.remap_reps > 0 else None
    head = "learned" if "learned" in res else next(iter(res))
    el, stage_ms, launches, st, tile = res[head]

    def rate(name):
        return ncell * args.steps / res[name][0] if name in res else None

    value = rate(head)
    plain = rate("plain")
    # algorithmic HBM bytes of the stage kernel: stage 1 reads Q^n and writes Q^(1),
    # stage 2 reads Q^n and Q^(1) and writes Q^(n+1): 5 nv doubles per cell and step
    bytes_per_step = 5 * nv * 8 * ncell
    # per launch (two launches per step on this single-level workload) over the
    # average launch duration of every timed run
    launch_ms = stage_ms / max(launches, 1)
    achieved = 0.5 * bytes_per_step / (launch_ms * 1e-3) / 1e9
    prof = counters_from_profiles("c2")
    traffic = prof.get("hbm_bytes_per_launch")
    valu = prof.get("sq", {}).get("SQ_INSTS_VALU")
    valu_issue = None
    if valu:
        issue = valu / (launch_ms * 1e-3)
        valu_issue = {"wave_insts_per_launch": valu, "achieved": issue, "peak": VALU_PEAK_WAVE_INSTS,
                      "unit": "wave64 VALU instructions/s", "frac": issue / VALU_PEAK_WAVE_INSTS}
    out = {
        "metric": "FP64 cell-updates/s (LAT-batched+MLP-EOS vs plain) at <=1e-11 rel err; % HBM roof",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "repeats": args.repeats,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2: 128^3 periodic as 64 MeshBlocks of 32^3, Saha H/He table EOS 256x256, dual "
                               "energy, cold Mach-1e7 Gaussian stream, CFL 0.3", "cells": ncell, "nv": nv,
                   "form": FORMS[head],
                   "tile": T.tile_shapes()[tile]},
        "forms": {k: {"value": rate(k), "ms_per_step": 1e3 * v[0] / args.steps, "form": FORMS[k],
                      "stage_kernel_ms": v[1] / max(v[2], 1), "tile": T.tile_shapes()[v[4]]} for k, v in res.items()},
        "speedup_vs_plain": (value / plain) if plain else None,
        "learned_seed": {"train_steps": 2000, "batch": 4096, "samples": 1 << 20, "train_seconds": train_s,
                         "final_loss": train_loss, "evaluation": seed_err},
        "max_rel_err_vs_oracle": acc,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "stage_tiled", "avg_launch_ms": launch_ms,
                     "algorithmic_bytes_per_cell_update": 5 * nv * 8,
                     "valu_issue": valu_issue},
        "cpu_baseline": cpu,
        "lat": lat,
        "gravity": grav,
        "remap": remap,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
