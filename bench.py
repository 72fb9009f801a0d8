#!/usr/bin/env python3
"""Benchmark of the MeshBlock hydro update on one MI355X.

Headline workload: the production-shaped run, 4096 MeshBlocks (1688 x 32^3 +
2408 x 16^3, 65.2 M cells, FP64) with the Saha H/He table EOS, dual energy, a
moving 1e3 Msun point mass with excision, and localized adaptive time stepping
over four levels (N_LAT = 3, sparse top bins merged below 1 % of the blocks).
One step = one LAT window, one pass of the whole hot path: the CFL reduction
(per-block steps, global minimum, level assignment with merge and neighbour
limit) and the window's 2^Lmax sub-cycles of RK2 stages (PLM, seeded table
inversion, HLLC, divergence, gravity, dual-energy update, excision), the
delayed flux corrections and the level bookkeeping, inputs resident in HBM.

Prints one JSON line.  `value` is the cell-updates/s of the learned form: all
active levels in one launch per RK phase, the window replayed from a captured
hipGraph, and before each stage but a window's first a pass that finds the
table cell of every active cell's state by a search started from the learned
network's prediction (the network is trained first on the GPU by the
library's own kernels; training time reported, not timed).  Beside it: the
plain form (one launch per level, bisection for every table query, no graph).
Both give the same bits.  Each form runs --warmup windows, then --repeats
timed runs of exactly --steps windows; its rate is that of the median run,
from the library's own update counters.  The roofline entry is the stage
kernel of the learned form: after the timed runs the same form runs --steps
windows once more without graph replay, every stage launch bracketed by HIP
events on the library's stream; 240 algorithmic bytes per cell-update over the
summed launch time.  The CPU baseline is the FP64 oracle on the host on the
512-block sub-domain of the same run (5.3 M cells) over two windows, with its
own CFL steps and levels (single-thread rate on the first window beside it);
the GPU headline form runs the same two windows from the same initial state,
and the two end states give max_rel_err_vs_oracle.

Secondary objects: "c2" times the 128^3 table-EOS stream (64 x 32^3, single
level) in six inversion forms with its own stage-kernel roofline, "lat" the
256^3 polytrope (ideal gas, fixed potential, LAT) batched beside per-level,
"learned_seed" the network's training and evaluation, "gravity" the
self-gravity multigrid on the 256^3 Jeans wave, "remap" the restart remap of
the 128^3 stream onto 256^3, "amr" the production-shaped run on two refinement
levels (134.2 M cells) with its stage kernel's roofline and the oracle on a
sub-domain.
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
FP64_VECTOR_PEAK_TFLOPS = 78.6
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
            seed_params=None, tile=-1):
    """LAT windows (reduce_dt, level assignment, one window of 2^Lmax sub-cycles)
    timed end to end; returns rates from the library's own update counters.
    tile < 0: the autotuner picks the stage variant (its id is returned)."""
    import torch
    ctx = T.Context(cfg, mesh, U, phi=phi, table=table, inv_mode=inv_mode)
    if seed_params is not None:
        ctx.mlp_init(seed_params, W.seed_ranges(table))
        ctx.mlp_enable_seed(True)
    if tile >= 0:
        ctx.set_tile(tile)
    else:
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
    tile_id = ctx.get_tile()
    tile = T.tile_shapes()[tile_id]
    ctx.close()
    cu = st1["cell_updates"] - st0["cell_updates"]
    bu = st1["block_updates"] - st0["block_updates"]
    return {"value": cu / el, "sync_equivalent": sync_equiv / el, "ms_per_window": 1e3 * el / windows,
            "windows": windows, "block_updates": int(bu), "block_updates_sync": int(sync_equiv // mesh.ncells *
                                                                                      mesh.nblocks),
            "levels": [int(v) for v in np.trim_zeros(hist, "b")], "tile": tile, "tile_id": tile_id}


def lat_section(T, W, windows, warmup):
    """The polytrope (ideal gas, fixed potential, LAT): batched launches replayed
    from a graph beside one launch per level."""
    cfg, mesh, U, phi, info = W.polytrope_c3()
    cfg = dataclasses.replace(cfg, merge_frac=0.01)  # performance runs merge sparse top bins
    batched = run_lat(T, W, cfg, mesh, U, windows, warmup, batched=True, graph=True, phi=phi)
    return {
        "workload": "256^3 as 512 MeshBlocks of 32^3, n=1.5 polytrope (1 Msun, 1 Rsun) in a 1e-10 atmosphere, fixed "
                    "potential, ideal gas, N_LAT=3, merge_frac 0.01, outflow",
        "note": "both forms use the stage variant the autotuner picked for the batched form",
        "batched_graph": batched,
        "plain": run_lat(T, W, cfg, mesh, U, windows, warmup, batched=False, graph=False, phi=phi,
                         tile=batched["tile_id"])}


C5_WORKLOAD = ("production-shaped: 4096 MeshBlocks (1688 x 32^3 + 2408 x 16^3, 65.2M cells), Saha H/He table EOS "
               "256x256, dual energy, 1e3 Msun point mass with excision in a moving frame, debris stream, LAT "
               "N_LAT=3, merge_frac 0.01, CFL 0.3, outflow")

C5_FORMS = {
    "learned": "LAT-batched (all active levels in one launch per RK phase, window replayed from a hipGraph); "
               "before each stage but a window's first, a pass finds every active cell's table cell by a search "
               "started from the learned network's prediction (the window's first stage takes the cells the CFL "
               "reduction found); the cell seeds the cell's face and compression queries",
    "plain": "one launch per level per RK phase, no graph; bisection for every table query",
}


def _timed_windows(ctx, windows, graph, batched=True):
    """`windows` LAT windows (CFL reduction, level assignment, window), timed
    end to end; returns (seconds, cell updates, block updates, sync-equivalent
    cell updates, level histogram)."""
    import torch
    st0 = ctx.stats()
    sync_equiv = 0
    hist = np.zeros(8, dtype=np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(windows):
        _, dt0, lev, L = ctx.reduce_dt()
        ctx.run_window(dt0 * 2 ** L, batched=batched, graph=graph)
        sync_equiv += ctx.mesh.ncells * 2 ** L
        h = np.bincount(lev)
        hist[:len(h)] += h
    ctx.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st1 = ctx.stats()
    return (el, st1["cell_updates"] - st0["cell_updates"], st1["block_updates"] - st0["block_updates"], sync_equiv,
            hist)


def _timing_pass(make_ctx, windows, warmup, batched=True):
    """Stage-kernel launch timing over the windows of a form's first timed run:
    a fresh context (make_ctx) repeats the same warm-up windows, then runs
    `windows` windows without graph replay with HIP events recorded on the
    library's stream around every stage launch (in a run of one section and
    one form these are the process's last stage dispatches, the ones the
    profile summaries average with --last)."""
    ctx = make_ctx()
    for _ in range(warmup):
        _, dt0, lev, L = ctx.reduce_dt()
        ctx.run_window(dt0 * 2 ** L, batched=batched, graph=False)
    ctx.sync()
    ctx.set_timing(True)
    el, cu, _, _, _ = _timed_windows(ctx, windows, graph=False, batched=batched)
    stage_ms, launches = ctx.stage_time()
    ctx.close()
    return {"windows": windows, "cell_updates": int(cu), "stage_kernel_ms": stage_ms,
            "stage_launches": int(launches), "ms_per_window": 1e3 * el / windows,
            "windows_timed": f"the first timed run's windows ({warmup} warm-up windows, then {windows}), "
                             "on a fresh context"}


def c5_section(T, W, table, params, forms, windows, warmup, repeats, tile):
    """The headline: the production-shaped LAT workload in the learned and the
    plain form.  Returns {form: result}; the learned form adds the stage
    kernel's launch timing (_timing_pass) over the windows of its first timed
    run."""
    cfg, mesh, U = W.debris_stream_c5(table)
    cfg = dataclasses.replace(cfg, merge_frac=0.01)
    out = {}
    for name, mode, batched, graph in (("learned", 4, True, True), ("plain", 0, False, False)):
        if name not in forms:
            continue

        def make_ctx(mode=mode):
            c = T.Context(cfg, mesh, U, table=table, inv_mode=mode)
            if mode == 4:
                c.mlp_init(params, W.seed_ranges(table))
                c.mlp_enable_seed(True)
            return c

        ctx = make_ctx()
        t_tune = time.perf_counter()
        if tile >= 0:
            ctx.set_tile(tile)
        else:
            ctx.autotune(reps=3)
        ctx.sync()
        t_tune = time.perf_counter() - t_tune
        for _ in range(warmup):
            _, dt0, lev, L = ctx.reduce_dt()
            ctx.run_window(dt0 * 2 ** L, batched=batched, graph=graph)
        ctx.sync()
        st_before = ctx.stats()
        runs = sorted((_timed_windows(ctx, windows, graph, batched) for _ in range(repeats)), key=lambda r: r[0])
        st_after = ctx.stats()
        el, cu, bu, se, hist = runs[len(runs) // 2]
        r = {"value": cu / el, "ms_per_window": 1e3 * el / windows, "windows": windows, "repeats": repeats,
             "sync_equivalent": se / el, "block_updates": int(bu),
             "block_updates_sync": int(se // mesh.ncells * mesh.nblocks),
             "levels": [int(v) for v in np.trim_zeros(hist, "b")], "tile": T.tile_shapes()[ctx.get_tile()],
             "form": C5_FORMS[name],
             # outside the timed windows: the autotuner, and the graph captures of the warm-up (a window
             # whose Lmax has no graph yet is captured inside a timed window: counted here)
             "autotune_s": t_tune if tile < 0 else None,
             "graph_captures_warmup": int(st_before["graph_captures"]),
             "capture_ms_warmup": st_before["capture_ms"],
             "graph_captures_in_timed_runs": int(st_after["graph_captures"] - st_before["graph_captures"]),
             "capture_ms_in_timed_runs": st_after["capture_ms"] - st_before["capture_ms"]}
        used_tile = ctx.get_tile()
        ctx.close()
        if name == "learned":
            def make_tuned():
                c = make_ctx()
                c.set_tile(used_tile)
                return c
            r["timing_pass"] = _timing_pass(make_tuned, windows, warmup, batched)
        out[name] = r
    return out


AMR_WORKLOAD = ("production-shaped run on two refinement levels: the 301 flagged regions refined into eight "
                "level-1 blocks each, 1688 level-0 + 2408 level-1 MeshBlocks of 32^3 (134.2M cells), Saha H/He "
                "table EOS 256x256, dual energy, 1e3 Msun point mass with excision in a moving frame, debris "
                "stream, LAT N_LAT=3, merge_frac 0.01, CFL 0.3, outflow")


def amr_section(T, W, table, params, windows, warmup, oracle_windows):
    """The two-level (coarse-fine) LAT run in the learned form (its own stage
    kernel kind), with the stage kernel's launch timing (_timing_pass) over the
    windows of the timed run, and on the region sub-domain AMR_SUBDOMAIN the
    oracle (timed on the host's threads) against the same form."""
    import oracle
    from tests.parity import rel_err
    cfg, mesh, U = W.debris_stream_amr(table)
    cfg = dataclasses.replace(cfg, merge_frac=0.01)

    def make_ctx():
        c = T.Context(cfg, mesh, U, table=table, inv_mode=4)
        c.mlp_init(params, W.seed_ranges(table))
        c.mlp_enable_seed(True)
        return c

    ctx = make_ctx()
    for _ in range(warmup):
        _, dt0, lev, L = ctx.reduce_dt()
        ctx.run_window(dt0 * 2 ** L, batched=True, graph=True)
    ctx.sync()
    el, cu, bu, se, hist = _timed_windows(ctx, windows, graph=True)
    ctx.close()
    tp = _timing_pass(make_ctx, windows, warmup)
    cu2, stage_ms, launches = tp["cell_updates"], tp["stage_kernel_ms"], tp["stage_launches"]
    del U
    bpc = 5 * 6 * 8
    launch_ms = stage_ms / max(launches, 1)
    alg = bpc * cu2 / max(launches, 1)
    achieved = alg / (launch_ms * 1e-3) / 1e9
    out = {"workload": AMR_WORKLOAD, "cells": int(mesh.ncells), "blocks": int(mesh.nblocks),
           "value": cu / el, "unit": "cell-updates/s", "ms_per_window": 1e3 * el / windows, "windows": windows,
           "sync_equivalent": se / el, "block_updates": int(bu), "levels": [int(v) for v in np.trim_zeros(hist, "b")],
           "form": "learned (mode 4, network, batched, graph); stage kernel kind of its own with cross-level ghosts",
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "stage_tiled (two-level kind)",
                        "avg_launch_ms": launch_ms, "launches": int(launches),
                        "algorithmic_bytes_per_launch": alg, "algorithmic_bytes_per_cell_update": bpc}}
    if oracle_windows > 0:
        cfg_s, mesh_s, U_s = W.debris_stream_amr(table, box=W.AMR_SUBDOMAIN)
        cfg_s = dataclasses.replace(cfg_s, merge_frac=0.01)
        t0 = time.perf_counter()
        o, info, obu, ocu = oracle.run_lat(cfg_s, mesh_s, U_s, oracle_windows, table=table)
        cpu_s = time.perf_counter() - t0
        ctx = T.Context(cfg_s, mesh_s, U_s, table=table, inv_mode=4)
        ctx.mlp_init(params, W.seed_ranges(table))
        ctx.mlp_enable_seed(True)
        lev_equal = True
        for w in range(oracle_windows):
            _, dt0, lev, L = ctx.reduce_dt()
            lev_equal &= bool(np.array_equal(lev, info[w][0])) and L == info[w][1]
            ctx.run_window(dt0 * 2 ** L, batched=True, graph=True)
        g = ctx.get_state()
        ctx.close()
        strict = rel_err(cfg_s.nv, mesh_s, g, o)
        spread = []
        for kw in ({"fused": True}, {"fused": False, "long_math": True}):
            with oracle.interp_rounding(**kw):
                spread.append(rel_err(cfg_s.nv, mesh_s, oracle.run_lat(cfg_s, mesh_s, U_s, oracle_windows,
                                                                       table=table)[0], o))
        spread = np.max(spread, axis=0)
        out["cpu_baseline"] = {"value": ocu / cpu_s, "unit": "cell-updates/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "host_cpu": host_cpu_model(),
                               "sample": f"{oracle_windows} LAT windows of the sub-domain {W.AMR_SUBDOMAIN} "
                                         f"({mesh_s.ncells} cells, {mesh_s.nblocks} blocks, "
                                         f"{int(mesh_s.rlev.sum())} refined; {ocu} cell-updates), own CFL steps "
                                         f"and levels, {cpu_s:.1f} s"}
        out["accuracy"] = {"max_rel_err_vs_oracle_strict": float(np.max(strict)),
                           "per_variable_strict": [float(v) for v in strict],
                           "oracle_spread_strict": [float(v) for v in spread],
                           "bar": "strict <= max(1e-11, 4 x the oracle's own spread) (the point-mass bar)",
                           "levels_bit_exact": lev_equal,
                           "case": f"sub-domain {W.AMR_SUBDOMAIN}, {oracle_windows} windows, learned form"}
    return out


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def c5_oracle_section(T, W, table, params, windows=2, single_thread=True, tile=-1):
    """The 512-block sub-domain of the production-shaped run: the oracle over
    `windows` windows with its own CFL steps and levels (timed on the host's
    threads; the first window again on one thread), and the GPU headline form
    over the same windows from the same initial state.  Returns (cpu_baseline,
    accuracy dict)."""
    import oracle
    from tests.parity import rel_err
    cfg, mesh, U = W.debris_stream_c5(table, box=W.C5_SUBDOMAIN_512)
    cfg = dataclasses.replace(cfg, merge_frac=0.01)
    t0 = time.perf_counter()
    o, info, bu, cu = oracle.run_lat(cfg, mesh, U, windows, table=table)
    cpu_s = time.perf_counter() - t0
    cpu = {"value": cu / cpu_s, "unit": "cell-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{windows} LAT windows of the 512-block sub-domain of the production-shaped run "
                     f"({mesh.ncells} cells: 112 x 32^3 + 400 x 16^3; {cu} cell-updates, {bu} block updates), "
                     f"own CFL steps and levels, {cpu_s:.1f} s",
           "host_cpu": host_cpu_model()}
    if single_thread:
        with oracle.threads(1):
            t1 = time.perf_counter()
            _, _, _, cu1 = oracle.run_lat(cfg, mesh, U, 1, table=table)
            s1 = time.perf_counter() - t1
        cpu["single_thread"] = {"value": cu1 / s1, "cores": 1, "sample": f"the first window ({cu1} cell-updates), "
                                                                         f"{s1:.1f} s"}
    ctx = T.Context(cfg, mesh, U, table=table, inv_mode=4)
    ctx.mlp_init(params, W.seed_ranges(table))
    ctx.mlp_enable_seed(True)
    if tile >= 0:
        ctx.set_tile(tile)
    else:
        ctx.autotune(reps=2)
    lev_equal = True
    dt_rel = 0.0
    for w in range(windows):
        _, dt0, lev, L = ctx.reduce_dt()
        lev_o, L_o, dt0_o, _ = info[w]
        lev_equal &= bool(np.array_equal(lev, lev_o)) and L == L_o
        dt_rel = max(dt_rel, abs(dt0 / dt0_o - 1))
        ctx.run_window(dt0 * 2 ** L, batched=True, graph=True)
    g = ctx.get_state()
    ctx.close()
    stencil = rel_err(cfg.nv, mesh, g, o, stencil=True)
    strict = rel_err(cfg.nv, mesh, g, o, stencil=False)
    spread = []
    for kw in ({"fused": True}, {"fused": False, "long_math": True}):
        with oracle.interp_rounding(**kw):
            spread.append(rel_err(cfg.nv, mesh, oracle.run_lat(cfg, mesh, U, windows, table=table)[0], o))
    spread = np.max(spread, axis=0)
    acc = {"max_rel_err_vs_oracle": float(np.max(stencil)), "max_rel_err_vs_oracle_strict": float(np.max(strict)),
           "per_variable_stencil": [float(v) for v in stencil], "per_variable_strict": [float(v) for v in strict],
           "oracle_spread_strict": [float(v) for v in spread],
           "metric": "per-cell relative error against the largest scale of the cell's 7-point stencil (the "
                     "point-mass bar, <= 1e-11); strict: against the cell's own scale, beside the oracle's own "
                     "spread under equally valid roundings",
           "levels_bit_exact": lev_equal, "max_dt0_rel_diff": dt_rel,
           "case": f"512-block sub-domain, {windows} windows, learned form (mode 4, network, batched, graph)"}
    return cpu, acc


def _query_eval(ctx, lr, le, reps=5):
    """Seeded (network start) against table-only inversion of device queries:
    |dlogT| percentiles of the network's prediction, secant-step histogram,
    bisection fallback rate, time per query of each (same cells, checked)."""
    import torch
    n = lr.numel()
    l0, j0, _ = ctx.eos_invert(lr, le, mode=0)
    err = (ctx.mlp_forward(torch.stack([lr, le], 1)) - l0).abs().cpu().numpy()
    q = {f"p{p}": float(np.percentile(err, p)) for p in (50, 90, 99, 99.99)}
    q["max"] = float(err.max())
    ns = {}
    for mode in (0, 1):
        ctx.eos_invert(lr, le, mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = ctx.eos_invert(lr, le, mode=mode)
        torch.cuda.synchronize()
        ns[mode] = 1e9 * (time.perf_counter() - t0) / (reps * n)
    l1, j1, it1 = out
    if not (torch.equal(j0, j1) and torch.equal(l0, l1)):
        raise SystemExit("seeded inversion differs from the table-only one")
    hist = np.bincount(it1.cpu().numpy().astype(np.int64) + 1)
    q.update({"queries": n, "secant_steps_histogram": {str(k - 1): int(v) for k, v in enumerate(hist) if v},
              "bisection_fallback_rate": float(hist[0]) / n, "ns_per_query_table_only": ns[0],
              "ns_per_query_seeded": ns[1], "seeded_over_table_only": ns[1] / ns[0]})
    return q


def seed_eval_section(T, W, table, params, windows=2):
    """Where the learned seed is evaluated beyond its training distribution:
    (1) every cell state of the polytrope run with the Saha table (the n = 1.5
    star of the LAT workload with the table EOS, initial internal energy from
    the Saha temperature at the polytrope's pressure), taken after each of
    `windows` LAT windows, as inversion queries; (2) a table of the paper's
    size (640 x 640 nodes over the same ranges), with a network trained on it
    by the same recipe, on 2^24 queries of its training distribution."""
    import torch
    cfg, mesh, U, phi, _ = W.polytrope_c3_saha(table)
    ctx = T.Context(cfg, mesh, U, phi=phi, table=table, inv_mode=4)
    ctx.mlp_init(params, W.seed_ranges(table))
    ctx.mlp_enable_seed(True)
    lrs, les = [], []
    for _ in range(windows):
        _, dt0, lev, L = ctx.reduce_dt()
        ctx.run_window(dt0 * 2 ** L, batched=True, graph=True)
        g = torch.from_numpy(ctx.get_state()).cuda()
        off = mesh.offsets(cfg.nv)
        for b in range(mesh.nblocks):
            n3 = int(mesh.blk[b, 0]) ** 3
            blk = g[off[b]:off[b + 1]].view(cfg.nv, n3)
            rho = blk[0]
            ke = 0.5 * (blk[1] ** 2 + blk[2] ** 2 + blk[3] ** 2) / rho
            u = torch.clamp(blk[4] - ke, min=rho * table.e_floor)
            lrs.append(torch.log10(rho))
            les.append(torch.log10(u / rho))
    poly = _query_eval(ctx, torch.cat(lrs).contiguous(), torch.cat(les).contiguous())
    poly["case"] = (f"every cell state (log rho, log e) of the 256^3 polytrope run with the Saha table after each of "
                    f"{windows} LAT windows (learned form)")
    ctx.close()
    big = W.saha_table(nrho=640, nT=640)
    p2, secs, loss, q2 = train_seed(T, W, big)
    q2.update({"case": "640 x 640 Saha table (the paper's table size), network trained on it (2000 Adam steps, "
                       "batch 4096, 2^20 samples), 2^24 queries of the training distribution",
               "train_seconds": secs, "final_loss": loss})
    return {"polytrope_saha": poly, "table_640": q2}


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


def c2_section(T, W, table, params, forms, steps, warmup, repeats, tile, cpu_steps):
    """The 128^3 table-EOS stream in six inversion forms (single level, one
    step = CFL reduction + RK2 step), with the stage kernel's roofline, and its
    accuracy check against the oracle (each side with its own CFL steps)."""
    cfg, mesh, U = W.stream_c2(table)
    ncell, nv = mesh.ncells, cfg.nv
    res = {}
    for name, mode, batched, riemann in (("learned", 4, True, 0), ("temporal", 3, True, 0), ("chained", 2, True, 0),
                                         ("plain", 0, False, 0), ("learned_hlle", 4, True, 1),
                                         ("learned_inkernel", 1, True, 0)):
        if name in forms:
            res[name] = run_form(T, W, cfg, mesh, U, table, steps, warmup, inv_mode=mode, batched=batched,
                                 seed_params=params if mode in (1, 4) else None, tile=tile, riemann=riemann,
                                 repeats=repeats)
    if not res:
        return None
    head = "learned" if "learned" in res else next(iter(res))
    el, stage_ms, launches, st, _ = res[head]

    def rate(name):
        return ncell * steps / res[name][0] if name in res else None

    # stage 1 reads Q^n and writes Q^(1), stage 2 reads Q^n and Q^(1) and writes
    # Q^(n+1): 5 nv doubles per cell and step, two launches per step
    launch_ms = stage_ms / max(launches, 1)
    achieved = 0.5 * 5 * nv * 8 * ncell / (launch_ms * 1e-3) / 1e9
    prof = counters_from_profiles("c2")
    out = {"workload": "128^3 periodic as 64 MeshBlocks of 32^3, Saha H/He table EOS 256x256, dual energy, cold "
                       "Mach-1e7 Gaussian stream, CFL 0.3, single level", "cells": ncell,
           "forms": {k: {"value": rate(k), "ms_per_step": 1e3 * v[0] / steps, "form": FORMS[k],
                         "stage_kernel_ms": v[1] / max(v[2], 1), "tile": T.tile_shapes()[v[4]]}
                     for k, v in res.items()},
           "speedup_vs_plain": rate(head) / rate("plain") if "plain" in res else None,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": prof.get("hbm_bytes_per_launch"),
                        "kernel": "stage_tiled", "avg_launch_ms": launch_ms,
                        "algorithmic_bytes_per_launch": 0.5 * 5 * nv * 8 * ncell}}
    if cpu_steps > 0:
        import oracle
        from tests.parity import rel_err
        ctx = T.Context(cfg, mesh, U, table=table, inv_mode=4)
        ctx.mlp_init(params, W.seed_ranges(table))
        ctx.mlp_enable_seed(True)
        T.run_sync_steps(ctx, cpu_steps)
        g = ctx.get_state()
        ctx.close()
        t0 = time.perf_counter()
        o, _ = oracle.run_sync(cfg, mesh, U, cpu_steps, table=table)
        cpu_s = time.perf_counter() - t0
        out["max_rel_err_vs_oracle"] = float(np.max(rel_err(nv, mesh, g, o, stencil=False)))
        out["oracle"] = {"value": ncell * cpu_steps / cpu_s, "cores": oracle.num_threads(),
                         "sample": f"{cpu_steps} RK2 steps of the full 128^3 workload (own CFL steps), {cpu_s:.1f} s"}
    return out


SECTIONS = "c5,c5_oracle,c2,lat,seed_eval,gravity,remap,amr"


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed LAT windows per run of the headline forms "
                                                          "(timed steps per run of the c2 forms)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of --steps windows per form; each form reports the median run")
    ap.add_argument("--sections", default=SECTIONS, help=f"comma list out of {SECTIONS}")
    ap.add_argument("--forms", default="learned,plain,temporal,chained,learned_hlle,learned_inkernel",
                    help="forms to time (headline: learned, plain; c2 also: temporal, chained, learned_hlle, "
                         "learned_inkernel)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="stage-kernel variant id to use instead of autotuning (profiling runs fix it)")
    ap.add_argument("--oracle-windows", type=int, default=2, help="windows of the oracle on the 512-block sub-domain")
    ap.add_argument("--no-single-thread", action="store_true", help="skip the single-thread oracle window")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps of the c2 accuracy check (0: skip)")
    ap.add_argument("--lat-windows", type=int, default=10, help="timed windows per form on the polytrope")
    ap.add_argument("--gravity-cycles", type=int, default=10, help="timed multigrid V-cycles on the 256^3 Jeans wave")
    ap.add_argument("--gravity-steps", type=int, default=10, help="timed coupled steps on the 256^3 Jeans wave")
    ap.add_argument("--remap-reps", type=int, default=5, help="timed restart remaps")
    ap.add_argument("--amr-windows", type=int, default=3, help="timed windows of the two-level run")
    ap.add_argument("--amr-oracle-windows", type=int, default=1,
                    help="windows of the oracle on the two-level sub-domain (0: skip)")
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
    sections = set(args.sections.split(","))
    forms = args.forms.split(",")

    def note(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    table = W.saha_table()
    params, train_s, train_loss, seed_err = train_seed(T, W, table)
    note(f"network trained in {train_s:.2f} s")
    c5 = c5_section(T, W, table, params, forms, args.steps, args.warmup, args.repeats, args.tile) \
        if "c5" in sections else {}
    note("headline forms timed")
    cpu, acc = (c5_oracle_section(T, W, table, params, args.oracle_windows, not args.no_single_thread, args.tile)
                if "c5_oracle" in sections else (None, None))
    note("oracle sub-domain done")
    c2 = c2_section(T, W, table, params, forms, args.steps, args.warmup, args.repeats, args.tile, args.cpu_steps) \
        if "c2" in sections else None
    lat = lat_section(T, W, args.lat_windows, 1) if "lat" in sections and args.lat_windows > 0 else None
    seed_eval = seed_eval_section(T, W, table, params) if "seed_eval" in sections else None
    grav = gravity_section(T, W, args.gravity_cycles, args.gravity_steps) \
        if "gravity" in sections and args.gravity_cycles > 0 else None
    remap = remap_section(T, W, table, args.remap_reps) if "remap" in sections and args.remap_reps > 0 else None
    amr = amr_section(T, W, table, params, args.amr_windows, 1, args.amr_oracle_windows) \
        if "amr" in sections and args.amr_windows > 0 else None
    note("two-level run done")

    head = c5.get("learned")
    plain = c5.get("plain")
    roof = None
    if head and "timing_pass" in head:
        tp = head["timing_pass"]
        bpc = 5 * 6 * 8  # stage 1 reads Q^n, writes Q^(1); stage 2 reads both, writes Q^(n+1): 5 nv doubles
        launch_ms = tp["stage_kernel_ms"] / max(tp["stage_launches"], 1)
        alg_per_launch = bpc * tp["cell_updates"] / max(tp["stage_launches"], 1)
        achieved = alg_per_launch / (launch_ms * 1e-3) / 1e9
        prof = counters_from_profiles("c5")
        sq = prof.get("sq", {})
        valu = sq.get("SQ_INSTS_VALU")
        # instruction and FLOP rates over the profiled launches' own mean duration
        # (the counters' launches, not this run's timing pass)
        pms = prof.get("avg_launch_ms")
        f64 = None
        if pms and "SQ_INSTS_VALU_FMA_F64" in sq:
            flop = 64 * (sq["SQ_INSTS_VALU_ADD_F64"] + sq["SQ_INSTS_VALU_MUL_F64"] + sq["SQ_INSTS_VALU_TRANS_F64"]
                         + 2 * sq["SQ_INSTS_VALU_FMA_F64"])
            tf = flop / (pms * 1e-3) / 1e12
            f64 = {"flop_per_launch": flop, "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "profiled_launch_ms": pms}
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": prof.get("hbm_bytes_per_launch"),
                "kernel": "stage_tiled", "avg_launch_ms": launch_ms, "launches": tp["stage_launches"],
                "algorithmic_bytes_per_launch": alg_per_launch, "algorithmic_bytes_per_cell_update": bpc,
                "valu_issue": ({"wave_insts_per_launch": valu, "achieved": valu / (pms * 1e-3),
                                "peak": VALU_PEAK_WAVE_INSTS, "unit": "wave64 VALU instructions/s",
                                "frac": valu / (pms * 1e-3) / VALU_PEAK_WAVE_INSTS,
                                "profiled_launch_ms": pms} if valu and pms else None),
                "fp64": f64}
    value = head["value"] if head else None
    out = {
        "metric": "FP64 cell-updates/s (LAT-batched+MLP-EOS vs plain) at <=1e-11 rel err; % HBM roof",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "repeats": args.repeats,
        "ms_per_step": head["ms_per_window"] if head else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": C5_WORKLOAD, "step": "one LAT window (CFL reduction, level assignment, 2^Lmax "
                                                     "sub-cycles)", "cells": 65175552, "blocks": 4096, "nv": 6,
                   "form": C5_FORMS["learned"], "tile": head["tile"] if head else None},
        "forms": c5,
        "speedup_vs_plain": (value / plain["value"]) if head and plain else None,
        "max_rel_err_vs_oracle": acc["max_rel_err_vs_oracle"] if acc else None,
        "accuracy": acc,
        "roofline": roof,
        "cpu_baseline": cpu,
        "learned_seed": {"train_steps": 2000, "batch": 4096, "samples": 1 << 20, "train_seconds": train_s,
                         "final_loss": train_loss, "evaluation": seed_err, "beyond_training": seed_eval},
        "c2": c2,
        "lat": lat,
        "gravity": grav,
        "remap": remap,
        "amr": amr,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
