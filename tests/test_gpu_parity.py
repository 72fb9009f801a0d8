"""GPU path (libtdh through its C ABI) against the CPU oracle.

Both sides get the same seeded synthetic inputs from the input module; the
oracle never sees GPU output: it takes its own CFL steps and LAT levels (or
steps and levels the test fixes for both).  Bar: max relative error <= 1e-11
per variable and cell against the cell's own scale (tests/parity.py; on the
point-mass workloads the stencil-scale form and the oracle's own rounding
spread, point_mass_bar), bit-exact for integer results (levels, schedule,
table cells) and between launch forms of the GPU path itself.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_2609_37859_amd import workloads as W
from tests.parity import TOL, point_mass_bar, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_37859_amd import tdh as T
    T.lib()
    return T


def _run_gpu_sync(T, cfg, mesh, U, nsteps, table=None, phi=None, dts=None, seed_params=None, **kw):
    ctx = T.Context(cfg, mesh, U, phi=phi, table=table, **kw)
    if seed_params is not None:
        ctx.mlp_init(seed_params, W.seed_ranges(table))
        ctx.mlp_enable_seed(True)
    used = T.run_sync_steps(ctx, nsteps, dts)
    out = ctx.get_state()
    ctx.close()
    return out, used


@pytest.fixture(scope="module")
def seed_params(tdh, saha):
    """The learned seed trained on the GPU by the library's kernels (C4 recipe,
    600 Adam steps)."""
    import torch
    cfg = W.Config(eos_kind=1, e_floor=saha.e_floor)
    mesh = W.uniform_mesh(1, 1, 1, 8, 1.0)
    ctx = tdh.Context(cfg, mesh, W.uniform_state(mesh, W.Config()), table=saha)
    x = torch.from_numpy(W.seed_training_samples(saha, 1 << 20, 1)).cuda()
    lT, _, _ = ctx.eos_invert(x[:, 0].contiguous(), x[:, 1].contiguous(), mode=0)
    ctx.mlp_init(W.mlp_init_params(2), W.seed_ranges(saha))
    ctx.mlp_train(x, lT, steps=600, batch=4096, lr=1e-3, seed=1)
    p = ctx.mlp_params()
    ctx.close()
    return p


def _gpu_lat_windows(T, cfg, mesh, U, windows, table=None, phi=None, graph=True, seed_params=None, **kw):
    """`windows` LAT windows with the library's own CFL steps and levels;
    returns (state, per-window (dt_block, dt0, levels, Lmax), stats)."""
    ctx = T.Context(cfg, mesh, U, phi=phi, table=table, **kw)
    if seed_params is not None:
        ctx.mlp_init(seed_params, W.seed_ranges(table))
        ctx.mlp_enable_seed(True)
    info = []
    for _ in range(windows):
        dtb, dt0, lev, L = ctx.reduce_dt()
        info.append((dtb, dt0, lev, L))
        ctx.run_window(dt0 * 2 ** L, batched=True, graph=graph)
    out, st = ctx.get_state(), ctx.stats()
    ctx.close()
    return out, info, st


def _oracle_alts(orc, fn):
    """fn() run under the oracle's two alternative roundings (the point-mass bar)."""
    out = []
    for kw in ({"fused": True}, {"fused": False, "long_math": True}):
        with orc.interp_rounding(**kw):
            out.append(fn())
    return out


def _check_windows(g_info, o_info):
    """Per window: the library's dt_b within 1e-13 of the oracle's, and its
    levels equal to the oracle's own assignment bit for bit."""
    for (dtb, dt0, lev, L), (lev_o, L_o, dt0_o, dtb_o) in zip(g_info, o_info):
        assert np.max(np.abs(dtb / dtb_o - 1)) < 1e-13
        assert abs(dt0 / dt0_o - 1) < 1e-13
        assert L == L_o and np.array_equal(lev, lev_o), np.nonzero(lev != lev_o)


def test_c1_entropy_wave_20_steps(tdh, orc):
    """One periodic 32^3 block, ideal gas, each side choosing its own CFL steps."""
    cfg, mesh, U = W.entropy_wave_c1()
    g, dg = _run_gpu_sync(tdh, cfg, mesh, U, 20)
    o, do = orc.run_sync(cfg, mesh, U, 20)
    assert np.max(np.abs(dg / do - 1)) < 1e-13
    err = rel_err(5, mesh, g, o)
    print("C1 rel err per variable", err)
    assert np.all(err <= TOL)


def test_uniform_state_bit_exact(tdh, orc):
    for dual in (0, 1):
        cfg = W.Config(dual=dual)
        mesh = W.uniform_mesh(2, 2, 1, 16, (0.1, 0.2, 0.15))
        U = W.uniform_state(mesh, cfg)
        g, _ = _run_gpu_sync(tdh, cfg, mesh, U, 5, dts=[1e-3] * 5)
        assert np.array_equal(g, U)


def test_periodic_conservation_gpu(tdh, orc):
    cfg = W.Config(dual=1)
    mesh = W.uniform_mesh(2, 2, 2, 16, 1.0 / 32)
    U = W.random_smooth_state(mesh, cfg, seed=3, amp=0.3)
    g, dts = _run_gpu_sync(tdh, cfg, mesh, U, 10)
    o, dto = orc.run_sync(cfg, mesh, U, 10)
    assert np.max(np.abs(dts / dto - 1)) < 1e-13
    G0, G1 = W.to_global(mesh, 6, U), W.to_global(mesh, 6, g)
    for v in (0, 4):
        assert abs(math.fsum(G1[v].ravel()) - math.fsum(G0[v].ravel())) <= 1e-14 * math.fsum(G0[v].ravel())
    err = rel_err(6, mesh, g, o)
    assert np.all(err <= TOL), err


@pytest.fixture(scope="module")
def c2_oracle(orc, saha):
    cfg, mesh, U = W.stream_c2(saha)
    o, do = orc.run_sync(cfg, mesh, U, 20, table=saha)
    return cfg, mesh, U, o, do


@pytest.mark.parametrize("inv_mode", [0, 1, 2, 3, 4])
def test_c2_table_dual_energy_20_steps(tdh, c2_oracle, saha, seed_params, inv_mode):
    """C2 at full size: 128^3 as 64 blocks of 32^3, Saha table, dual energy,
    Mach 1e7 stream, 20 steps with each side's own CFL steps, in every
    inversion form: bisection (0), the network inside the stage kernel (1),
    a bisection pass (2), carried cells (3), a network-started pass (4, the
    benchmark's learned form); 1 and 4 with the network trained on the GPU."""
    cfg, mesh, U, o, do = c2_oracle
    net = seed_params if inv_mode in (1, 4) else None
    g, dg = _run_gpu_sync(tdh, cfg, mesh, U, 20, table=saha, inv_mode=inv_mode, seed_params=net)
    assert np.max(np.abs(dg / do - 1)) < 1e-13
    err = rel_err(6, mesh, g, o)
    print("C2 mode", inv_mode, "rel err per variable", err)
    assert np.all(err <= TOL)


def test_inversion_modes_agree_bitwise_and_with_oracle(tdh, orc, saha):
    import torch
    cfg = W.Config(eos_kind=1, e_floor=saha.e_floor)
    ctx = tdh.Context(cfg, W.uniform_mesh(1, 1, 1, 8, 1.0), W.uniform_state(W.uniform_mesh(1, 1, 1, 8, 1.0), W.Config()),
                      table=saha)
    rng = np.random.default_rng(5)
    n = 1 << 16
    lr = rng.uniform(-12.2, 2.2, n)
    le = rng.uniform(saha.le.min() - 0.2, saha.le.max() + 0.2, n)
    lT0, j0, it0 = ctx.eos_invert(torch.from_numpy(lr), torch.from_numpy(le), mode=0)
    lT2, j2, it2 = ctx.eos_invert(torch.from_numpy(lr), torch.from_numpy(le), mode=2)
    torch.cuda.synchronize()
    assert torch.equal(j0, j2) and torch.equal(lT0, lT2)
    jo, wo, lTo = orc.table_invert(saha, lr, le)
    jg = j0.cpu().numpy()
    lTg = lT0.cpu().numpy()
    same = jg == jo
    assert same.mean() > 0.999
    assert np.max(np.abs(lTg - lTo)) < 1e-12
    ctx.close()


def _centre_cells(ctx, cfg, mesh, g, table):
    """Exact table cell of every cell's state, from the library's bisection."""
    import torch
    off = mesh.offsets(6)
    lr, le = [], []
    for b in range(mesh.nblocks):
        q = g[off[b]:off[b + 1]].reshape(6, -1)
        K = 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
        Uc = q[4] - K
        Ueos = np.where((Uc > 0) & (Uc > cfg.eta1 * q[4]), Uc, q[5])
        Ue = np.maximum(Ueos, q[0] * table.e_floor)
        lr.append(np.log10(q[0]))
        le.append(np.log10(Ue / q[0]))
    _, j, _ = ctx.eos_invert(torch.from_numpy(np.concatenate(lr)), torch.from_numpy(np.concatenate(le)), mode=0)
    return j.cpu().numpy()


def test_temporal_seeds_track_the_state(tdh, saha):
    """inv_mode 3: after a state upload no seed is held (-1); after steps the
    held seeds are the table cells of the current state (up to the odd cell at
    a bracket edge, where host and device logarithms may round apart), and
    the state equals the bisection run's bit for bit."""
    cfg, mesh, U = W.stream_c2(saha, nb=2)
    ctx = tdh.Context(cfg, mesh, U, table=saha, inv_mode=3)
    assert np.all(ctx.seed_cells() == -1)
    tdh.run_sync_steps(ctx, 3, dts=[3e-4] * 3)
    g = ctx.get_state()
    seeds = ctx.seed_cells()
    exact = _centre_cells(ctx, cfg, mesh, g, saha)
    assert np.mean(seeds == exact) > 0.999, np.mean(seeds == exact)
    ctx.set_state(U)
    assert np.all(ctx.seed_cells() == -1)
    ctx.close()
    ref = tdh.Context(cfg, mesh, U, table=saha, inv_mode=0)
    tdh.run_sync_steps(ref, 3, dts=[3e-4] * 3)
    assert np.array_equal(ref.get_state(), g)
    ref.close()


def test_table_eos_evaluation_matches_oracle(tdh, orc, saha):
    """P and c_s from (rho, U) over the whole table range and beyond its edges
    (clamped), against the oracle's evaluation with the C library's log10 and
    pow: the library's own base-10 logarithm and the table interpolation agree
    to a few units in the last place (bound 1e-13 relative)."""
    import torch
    cfg = W.Config(eos_kind=1, e_floor=saha.e_floor)
    mesh = W.uniform_mesh(1, 1, 1, 8, 1.0)
    ctx = tdh.Context(cfg, mesh, W.uniform_state(mesh, W.Config()), table=saha)
    rng = np.random.default_rng(21)
    n = 1 << 18
    lr = rng.uniform(-12.3, 2.3, n)
    x = W.seed_training_samples(saha, n, 22)
    le = x[:, 1] + rng.uniform(-0.3, 0.3, n)  # table range and a little beyond
    rho = 10.0 ** lr
    U = rho * 10.0 ** le
    Pg, cg = ctx.eos_eval(torch.from_numpy(rho), torch.from_numpy(U))
    torch.cuda.synchronize()
    Po, co = orc.eos_eval(cfg, rho, U, table=saha)
    ctx.close()
    eP = np.max(np.abs(Pg.cpu().numpy() / Po - 1))
    ec = np.max(np.abs(cg.cpu().numpy() / co - 1))
    print("EOS eval max rel err P", eP, "c_s", ec)
    assert eP < 1e-13 and ec < 1e-13


def test_levels_bit_exact_and_dt_parity(tdh, orc):
    """C3-shaped polytrope (reduced to 4^3 blocks of 16^3): per-block CFL steps
    agree to 1e-13, and the library's level assignment from its own dt_b
    equals the oracle's assignment from the oracle's dt_b bit for bit (no
    block's ratio dt_b / dt0 lies within 1e-12 of a power of two, where the two
    roundings could decide apart)."""
    cfg, mesh, U, phi, info = W.polytrope_c3(nb=4, n=16)
    ctx = tdh.Context(cfg, mesh, U, phi=phi)
    dtb, dt0, lev, L = ctx.reduce_dt()
    ctx.close()
    dto = orc.cfl(cfg, mesh, U, phi=phi)
    assert np.max(np.abs(dtb / dto - 1)) < 1e-13
    lev_o, L_o, dt0_o = orc.lat_assign(cfg, mesh, dto)
    r = dto / dt0_o                                 # >= 1; the levels change where r crosses 2, 4, 8 ...
    near = np.abs(r / 2.0 ** np.round(np.log2(r)) - 1) < 1e-12
    assert not np.any(near & (r > 1.5))
    assert L == L_o and abs(dt0 / dt0_o - 1) < 1e-13
    assert np.array_equal(lev, lev_o)
    assert L >= 1


def _lat_run_gpu(T, cfg, mesh, U, phi, levels, dt0, windows, batched=True, graph=False, step_api=False, tile=None):
    ctx = T.Context(cfg, mesh, U, phi=phi)
    if tile is not None:
        ctx.set_tile(tile)
    Lmax = int(np.max(levels))
    for w in range(windows):
        ctx.set_levels(levels)
        dtc = dt0 * 2 ** Lmax
        if step_api:
            for k in range(2 ** Lmax):
                lmin = 0 if k == 0 else Lmax - ((k & -k).bit_length() - 1)
                ctx.step_level(lmin, dtc / 2 ** lmin)
        else:
            ctx.run_window(dtc, batched=batched, graph=graph)
    out = ctx.get_state()
    st = ctx.stats()
    ctx.close()
    return out, st


def test_lat_window_parity_polytrope(tdh, orc):
    """LAT windows on the reduced polytrope: GPU equals the oracle to 1e-11
    with the oracle's level assignment; all launch forms agree bit for bit."""
    cfg, mesh, U, phi, info = W.polytrope_c3(nb=4, n=16)
    dto = orc.cfl(cfg, mesh, U, phi=phi)
    lev, L, dt0 = orc.lat_assign(cfg, mesh, dto)
    assert L >= 1
    o = U
    t = 0.0
    for w in range(2):
        o, nupd = orc.lat_window(cfg, mesh, o, lev, dt0, phi=phi, t0=t)
        t += dt0 * 2 ** L
    g, st = _lat_run_gpu(tdh, cfg, mesh, U, phi, lev, dt0, 2)
    err = rel_err(5, mesh, g, o)
    print("LAT rel err", err, st)
    assert np.all(err <= TOL)
    assert st["block_updates"] == 2 * nupd
    g2, _ = _lat_run_gpu(tdh, cfg, mesh, U, phi, lev, dt0, 2, batched=False)
    g3, _ = _lat_run_gpu(tdh, cfg, mesh, U, phi, lev, dt0, 2, graph=True)
    g4, _ = _lat_run_gpu(tdh, cfg, mesh, U, phi, lev, dt0, 2, step_api=True)
    assert np.array_equal(g, g2) and np.array_equal(g, g3) and np.array_equal(g, g4)


@pytest.mark.parametrize("ghost_dense,riemann", [(1, 0), (0, 1), (1, 1)])
def test_lat_dense_ghosts_and_hlle_polytrope(tdh, orc, ghost_dense, riemann):
    """LAT windows on the reduced polytrope with the RK2 dense-output ghosts
    and/or the HLLE solver: GPU equals the oracle to 1e-11; launch forms and
    the fused and split stage forms agree bit for bit."""
    base, mesh, U, phi, info = W.polytrope_c3(nb=4, n=16)
    cfg = dataclasses.replace(base, ghost_dense=ghost_dense, riemann=riemann)
    dto = orc.cfl(cfg, mesh, U, phi=phi)
    lev, L, dt0 = orc.lat_assign(cfg, mesh, dto)
    assert L >= 1
    o, t = U, 0.0
    for w in range(2):
        o, nupd = orc.lat_window(cfg, mesh, o, lev, dt0, phi=phi, t0=t)
        t += dt0 * 2 ** L
    g, st = _lat_run_gpu(tdh, cfg, mesh, U, phi, lev, dt0, 2)
    err = rel_err(5, mesh, g, o)
    print("LAT dense/HLLE rel err", err)
    assert np.all(err <= TOL)
    if ghost_dense:  # the dense output changes the result where neighbours are mid-step
        lin, _ = orc.lat_window(dataclasses.replace(cfg, ghost_dense=0), mesh, U, lev, dt0, phi=phi)
        one, _ = orc.lat_window(cfg, mesh, U, lev, dt0, phi=phi)
        assert not np.array_equal(lin, one)
    g2, _ = _lat_run_gpu(tdh, cfg, mesh, U, phi, lev, dt0, 2, batched=False)
    g3, _ = _lat_run_gpu(tdh, cfg, mesh, U, phi, lev, dt0, 2, graph=True)
    split = [i for i, d in enumerate(tdh.tile_shapes()) if d[0] == 0][0]
    g4, _ = _lat_run_gpu(tdh, cfg, mesh, U, phi, lev, dt0, 2, tile=split)
    assert np.array_equal(g, g2) and np.array_equal(g, g3) and np.array_equal(g, g4)


@pytest.mark.parametrize("kind", ["c1", "c2"])
def test_hlle_sync_parity(tdh, orc, saha, kind):
    """The HLLE solver on C1 (ideal gas) and on the C2 table + dual-energy
    stream (20 steps, carried seed cells): GPU equals the oracle to 1e-11."""
    if kind == "c1":
        base, mesh, U = W.entropy_wave_c1()
        table, nv, kw = None, 5, {}
    else:
        base, mesh, U = W.stream_c2(saha)
        table, nv, kw = saha, 6, {"inv_mode": 3}
    cfg = dataclasses.replace(base, riemann=1)
    g, dg = _run_gpu_sync(tdh, cfg, mesh, U, 20, table=table, **kw)
    o, do = orc.run_sync(cfg, mesh, U, 20, table=table)
    assert np.max(np.abs(dg / do - 1)) < 1e-13
    err = rel_err(nv, mesh, g, o)
    print(kind, "HLLE rel err", err)
    assert np.all(err <= TOL)


def test_lat_reflux_conservation_gpu(tdh, orc):
    cfg = W.Config(dual=1)
    mesh = W.uniform_mesh(4, 2, 2, 8, 1.0 / 32)
    U = W.random_smooth_state(mesh, cfg, seed=8, amp=0.3)
    bx = mesh.blk[:, 1] // 8
    lev = np.array([{0: 2, 1: 1, 2: 0, 3: 1}[int(x)] for x in bx], dtype=np.int32)
    g, st = _lat_run_gpu(tdh, cfg, mesh, U, None, lev, 1e-3, 1)
    o, n = orc.lat_window(cfg, mesh, U, lev, 1e-3)
    assert np.all(rel_err(6, mesh, g, o) <= TOL)
    G0, G1 = W.to_global(mesh, 6, U), W.to_global(mesh, 6, g)
    for v in range(5):
        assert abs(math.fsum(G1[v].ravel()) - math.fsum(G0[v].ravel())) <= 1e-14 * math.fsum(G0[0].ravel())


def test_high_mach_wave_gpu(tdh, orc):
    """Dual-energy entropy wave at Mach ~7.7e7 (blocks of 16^3): GPU = oracle."""
    cfg, mesh, U = W.high_mach_wave(ncell=64, nt=16, dual=1)
    g, dts = _run_gpu_sync(tdh, cfg, mesh, U, 30)
    o, dto = orc.run_sync(cfg, mesh, U, 30)
    assert np.max(np.abs(dts / dto - 1)) < 1e-13
    err = rel_err(6, mesh, g, o)
    print("high-Mach wave rel err", err)
    assert np.all(err <= TOL)


def test_mixed_block_sizes_point_mass_excision(tdh, orc, saha):
    """Mixed 16^3 / 32^3 blocks (some 32^3 regions split into eight 16^3), Saha
    table, dual energy, moving softened point mass with excision, outflow.

    The stream's axis and the zero of its velocity sit off the grid's face
    planes.  On a face plane of mirror symmetry the exact mass flux is zero, and
    where such a face separates an excised from an active cell the one-way sink
    rule (keep the face's fluxes only if its mass flux enters the sink) is then
    decided by rounding: an equally faithful 10^x in the EOS flips it and moves
    the neighbouring cells by 1e-5 in one step, in the oracle itself."""
    split = np.zeros((2, 2, 3), dtype=bool)
    split[0, 1, 1] = split[1, 0, 2] = True
    dx = 2e10
    mesh = W.mixed_mesh((3, 2, 2), 32, split, dx, x0=(0.0, 0.0, 0.0), bc=(1, 1, 1))
    cfg = W.Config(eos_kind=1, dual=1, grav_kind=2, rho_floor=1e-12, p_floor=0.0, e_floor=saha.e_floor,
                   gm_bh=1.327e29, r_exc=4 * dx, r_soft=0.1 * dx, bh_x0=(50 * dx, 30 * dx, 33 * dx),
                   v_frame=(1e7, 0.0, 0.0))
    L = np.array([mesh.nx, mesh.ny, mesh.nz]) * dx

    def fn(x, y, z):
        r2 = (y - 0.5 * L[1] - 0.3 * dx) ** 2 + (z - 0.5 * L[2] + 0.2 * dx) ** 2
        rho = 1e-11 + 1e-4 * np.exp(-r2 / (2 * (6 * dx) ** 2))
        _, e = W.saha_pe(rho, 8e3)
        Uint = rho * e
        vx = 3e6 * np.sin(2 * np.pi * (x - 0.37 * dx) / L[0])
        return [rho, rho * vx, 0 * x, 0 * x, Uint + 0.5 * rho * vx * vx, Uint]
    U = W.pack_state(mesh, 6, fn)
    dts = [orc.cfl(cfg, mesh, U, table=saha).min()] * 6
    g, _ = _run_gpu_sync(tdh, cfg, mesh, U, 6, table=saha, dts=dts)
    o, _ = orc.run_sync(cfg, mesh, U, 6, table=saha, dts=dts)
    alts = _oracle_alts(orc, lambda: orc.run_sync(cfg, mesh, U, 6, table=saha, dts=dts)[0])
    ok, rep = point_mass_bar(6, mesh, g, o, alts)
    print("mixed blocks, point mass:", rep)
    assert ok


def test_all_tiles_bitwise_equal(tdh, orc, saha):
    """Every stage tile shape gives the same state bit for bit (C2 stream on
    a 2^3-block mesh, 4 steps), and the autotuner picks one of them."""
    cfg, mesh, U = W.stream_c2(saha, nb=2)
    shapes = tdh.tile_shapes()
    outs = []
    for t in range(len(shapes)):
        ctx = tdh.Context(cfg, mesh, U, table=saha, inv_mode=2)
        ctx.set_tile(t)
        tdh.run_sync_steps(ctx, 4, dts=[3e-4] * 4)
        outs.append(ctx.get_state())
        ctx.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    ctx = tdh.Context(cfg, mesh, U, table=saha)
    best, ms = ctx.autotune(reps=1)
    assert 0 <= best < len(shapes) and ms[best] > 0
    ctx.close()


def test_bench_workload_parity_sampled(tdh, orc, saha):
    """The benchmark's workload (C2, 128^3, seeded form, tile from the
    autotuner) after 3 GPU steps equals 3 oracle steps."""
    cfg, mesh, U = W.stream_c2(saha)
    ctx = tdh.Context(cfg, mesh, U, table=saha, inv_mode=2)
    ctx.autotune(reps=1)
    dts = tdh.run_sync_steps(ctx, 3)
    g = ctx.get_state()
    ctx.close()
    o, dto = orc.run_sync(cfg, mesh, U, 3, table=saha)
    assert np.max(np.abs(dts / dto - 1)) < 1e-13
    assert np.all(rel_err(6, mesh, g, o) <= TOL)


def test_c3_full_size_eight_windows(tdh, orc):
    """C3 at its full size (256^3 as 512 x 32^3, fixed polytrope potential,
    N_LAT = 3) over 8 coarse steps, each side with its own CFL steps and level
    assignment: every window's levels equal bit for bit, dt_b within 1e-13, the
    block-update count equal, and the end state within 1e-11 (batched launches
    replayed from a captured graph)."""
    import time
    cfg, mesh, U, phi, info = W.polytrope_c3()
    g, g_info, st = _gpu_lat_windows(tdh, cfg, mesh, U, 8, phi=phi)
    t0 = time.perf_counter()
    o, o_info, bu, cu = orc.run_lat(cfg, mesh, U, 8, phi=phi)
    _check_windows(g_info, o_info)
    assert st["block_updates"] == bu and st["cell_updates"] == cu
    err = rel_err(5, mesh, g, o)
    print("C3 full size, 8 windows: rel err", err, "updates", bu, "levels", [np.bincount(i[0]) for i in o_info],
          "oracle s", round(time.perf_counter() - t0, 1), flush=True)
    assert np.all(err <= TOL)


def _c5_reduced(saha):
    return W.debris_stream_c5(saha, regions=(4, 3, 2), n_split=6, dxr=1.0)


def test_c5_shaped_subdomain_lat_window(tdh, orc, saha):
    """C5-shaped run on a reduced region grid: mixed 16^3/32^3 blocks, Saha
    table, dual energy, moving point mass with excision, LAT levels from each
    side's own CFL; two windows in modes 2 and 3 (bitwise equal), against the
    oracle's two windows."""
    cfg, mesh, U = _c5_reduced(saha)
    outs = []
    for mode in (2, 3):  # centre cells bisected before each stage / carried from the last stage
        g, g_info, _ = _gpu_lat_windows(tdh, cfg, mesh, U, 2, table=saha, inv_mode=mode, graph=False)
        outs.append((g, g_info))
    assert np.array_equal(outs[0][0], outs[1][0])
    o, o_info, _, _ = orc.run_lat(cfg, mesh, U, 2, table=saha)
    _check_windows(outs[0][1], o_info)
    alts = _oracle_alts(orc, lambda: orc.run_lat(cfg, mesh, U, 2, table=saha)[0])
    ok, rep = point_mass_bar(6, mesh, outs[0][0], o, alts)
    print("C5-shaped reduced, 2 windows:", rep, "levels", [np.bincount(i[0]) for i in o_info])
    assert ok


def test_c5_shaped_dense_ghosts_window(tdh, orc, saha):
    """The C5-shaped sub-domain with the RK2 dense-output ghosts (the
    compiled table-EOS, point-mass, dense-ghost kind): one LAT window against
    the oracle, and a visible difference from the linear ghosts."""
    cfg, mesh, U = _c5_reduced(saha)
    cfg = dataclasses.replace(cfg, ghost_dense=1)
    g, g_info, _ = _gpu_lat_windows(tdh, cfg, mesh, U, 1, table=saha, inv_mode=2, graph=False)
    assert g_info[0][3] > 0
    o, o_info, _, _ = orc.run_lat(cfg, mesh, U, 1, table=saha)
    _check_windows(g_info, o_info)
    alts = _oracle_alts(orc, lambda: orc.run_lat(cfg, mesh, U, 1, table=saha)[0])
    ok, rep = point_mass_bar(6, mesh, g, o, alts)
    lin, _, _, _ = orc.run_lat(dataclasses.replace(cfg, ghost_dense=0), mesh, U, 1, table=saha)
    print("C5-shaped dense-ghost window:", rep, "max |dense - linear|", np.max(np.abs(o - lin)))
    assert ok
    assert not np.array_equal(o, lin)


def test_c5_subdomain_512_learned_form_two_windows(tdh, orc, saha, seed_params):
    """The benchmark's headline form on the 512-block sub-domain of the
    production-shaped run (112 x 32^3 + 400 x 16^3, Saha table, dual energy,
    moving point mass, N_LAT = 3, merge_frac 0.01): network-started seed
    passes (mode 4, network trained on the GPU), batched launches replayed from
    a graph, two windows with the library's own CFL steps and levels, against
    the oracle's two windows from its own."""
    cfg, mesh, U = W.debris_stream_c5(saha, box=W.C5_SUBDOMAIN_512)
    cfg = dataclasses.replace(cfg, merge_frac=0.01)
    g, g_info, st = _gpu_lat_windows(tdh, cfg, mesh, U, 2, table=saha, inv_mode=4, seed_params=seed_params)
    o, o_info, bu, cu = orc.run_lat(cfg, mesh, U, 2, table=saha)
    _check_windows(g_info, o_info)
    assert st["block_updates"] == bu
    alts = _oracle_alts(orc, lambda: orc.run_lat(cfg, mesh, U, 2, table=saha)[0])
    ok, rep = point_mass_bar(6, mesh, g, o, alts)
    print("C5 512-block sub-domain, learned form, 2 windows:", rep, "levels", [np.bincount(i[0]) for i in o_info],
          flush=True)
    assert ok


@pytest.mark.parametrize("case", ["c2_mode2", "c2_mode4_hlle", "c5_sync_point_mass", "c5_lat_point_mass",
                                  "polytrope_lat", "polytrope_lat_split_tile"])
def test_cfl_from_the_second_stage_equals_the_reduction(tdh, orc, saha, case):
    """After a single-level window of the fused form the CFL reduction takes
    the minima its second stages left; they equal, bit for bit, what the
    reduction computes from the state itself (the same state uploaded again,
    which drops them), levels included, and in modes 2 and 4 the recorded
    table cells equal the reduction's.  LAT windows (whose refluxes change
    completed blocks), the moving point mass, the ideal gas and the split
    form leave none, and the reduction runs: the same equalities hold."""
    table = None
    phi = None
    if case.startswith("c2"):
        cfg, mesh, U = W.stream_c2(saha, nb=2)
        table = saha
        mode = 2 if case == "c2_mode2" else 4
        if case.endswith("hlle"):
            cfg = dataclasses.replace(cfg, riemann=1)
        kw = dict(table=table, inv_mode=mode)
    elif case.startswith("c5"):  # mixed blocks, moving point mass with excision; one level or LAT
        cfg, mesh, U = W.debris_stream_c5(saha, regions=(4, 3, 2), n_split=6, dxr=1.0)
        if case == "c5_sync_point_mass":
            cfg = dataclasses.replace(cfg, n_lat=0)
        table = saha
        kw = dict(table=table, inv_mode=2)
    else:
        cfg, mesh, U, phi, _ = W.polytrope_c3(nb=4, n=16)
        kw = dict(phi=phi)
    ctx = tdh.Context(cfg, mesh, U, **kw)
    if case == "polytrope_lat_split_tile":
        ctx.set_tile(len([t for t in tdh.tile_shapes() if t[0] > 0]))  # the first split form
    for w in range(3):
        dtb, dt0, lev, L = ctx.reduce_dt()
        if w == 0:  # the initial state at t = 0
            dto = orc.cfl(cfg, mesh, U, table=table, phi=phi, t=0.0)
            assert np.all(np.abs(dtb / dto - 1) < 1e-13)
        ctx.run_window(dt0 * 2 ** L, batched=True)
        cells_after = ctx.seed_cells() if table is not None else None
        f_dtb, f_dt0, f_lev, f_L = ctx.reduce_dt()
        cells_fused = ctx.seed_cells() if table is not None else None
        g = ctx.get_state()
        ctx.set_state(g)
        k_dtb, k_dt0, k_lev, k_L = ctx.reduce_dt()
        assert np.array_equal(f_dtb, k_dtb) and f_dt0 == k_dt0 and np.array_equal(f_lev, k_lev) and f_L == k_L
        if table is not None:
            assert np.array_equal(cells_fused, ctx.seed_cells())
            if L == 0 and cfg.grav_kind != 2:  # the window's second stages recorded them
                assert np.array_equal(cells_after, cells_fused)
    print(case, "levels", np.bincount(k_lev), "dt0", k_dt0)
    ctx.close()


def test_cfl_after_a_window_on_caller_levels(tdh, orc, saha):
    """Levels installed by the caller on a run configured without LAT: the
    window refluxes completed blocks, so the reduction reads the state again
    and equals, bit for bit, the reduction of the same state uploaded anew."""
    cfg, mesh, U = W.stream_c2(saha, nb=2)
    ctx = tdh.Context(cfg, mesh, U, table=saha, inv_mode=2)
    dtb, dt0, lev, L = ctx.reduce_dt()
    assert L == 0
    levels = np.zeros(mesh.nblocks, dtype=np.int8)
    levels[::2] = 1
    ctx.set_levels(levels)
    ctx.run_window(dt0, batched=True)
    f = ctx.reduce_dt()
    ctx.set_state(ctx.get_state())
    k = ctx.reduce_dt()
    assert np.array_equal(f[0], k[0]) and f[1] == k[1]
    ctx.close()


def test_c5_full_size_lat_window(tdh, orc, saha):
    """The production-shaped workload at full size (4096 blocks, 65.2 M cells,
    Saha table, dual energy, moving point mass with excision, N_LAT = 3,
    merge_frac 0.01) in the benchmark's launch configuration (batched launches
    replayed from a captured graph): the library's dt_b and levels equal the
    oracle's own, and one window meets the point-mass bar."""
    import time
    cfg, mesh, U = W.debris_stream_c5(saha)
    cfg = dataclasses.replace(cfg, merge_frac=0.01)
    g, g_info, _ = _gpu_lat_windows(tdh, cfg, mesh, U, 1, table=saha, inv_mode=2)
    t0 = time.perf_counter()
    o, o_info, _, _ = orc.run_lat(cfg, mesh, U, 1, table=saha)
    secs = time.perf_counter() - t0
    _check_windows(g_info, o_info)
    alts = _oracle_alts(orc, lambda: orc.run_lat(cfg, mesh, U, 1, table=saha)[0])
    ok, rep = point_mass_bar(6, mesh, g, o, alts)
    print("C5 full-size window: levels", np.bincount(o_info[0][0]), "oracle seconds", round(secs, 1), rep, flush=True)
    assert ok
