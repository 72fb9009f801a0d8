"""Learned EOS seed network on the GPU (MFMA bf16 kernels) against the oracle.

Exactness: with dyadic inputs and weights (few significant bits) every fp32
sum is exact, so the bf16 rounding decisions coincide and the GPU forward
and gradient equal the oracle's exactly.  On random data the GPU accumulates
in fp32 in another order; the comparison then allows the rare bf16 rounding
flip that causes (each moves a value by one bf16 step, 2^-8 relative).
"""
import numpy as np
import pytest

from paper_2609_37859_amd import workloads as W

pytestmark = pytest.mark.gpu

RANGES = (-12.0, 2.0, 10.0, 16.0, 3.0, 8.0)  # log rho, log e, log T ranges


@pytest.fixture(scope="module")
def gctx(saha):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_37859_amd import tdh as T
    cfg = W.Config(eos_kind=1, e_floor=saha.e_floor)
    mesh = W.uniform_mesh(1, 1, 1, 8, 1.0)
    ctx = T.Context(cfg, mesh, W.uniform_state(mesh, W.Config()), table=saha)
    yield ctx
    ctx.close()


def raw_from_norm(xn, lo, hi):
    return lo + (xn + 1.0) * 0.5 * (hi - lo)


def test_forward_and_gradient_exact_on_dyadic_data(gctx, orc):
    import torch
    rng = np.random.default_rng(11)
    n = 128
    p = np.zeros(orc.N_PARAMS)
    p[0:128] = rng.integers(-8, 9, 128) / 8.0
    p[128:192] = rng.integers(-8, 9, 64) / 16.0
    p[192:4288] = rng.integers(-4, 5, 4096) / 64.0
    p[4288:4352] = rng.integers(-4, 5, 64) / 16.0
    p[4352:4416] = rng.integers(-4, 5, 64) / 32.0
    p[4416] = 0.125
    xn = rng.integers(-8, 9, (n, 2)) / 8.0
    tn = rng.integers(-8, 9, n) / 8.0
    lr_lo, lr_hi, le_lo, le_hi, lt_lo, lt_hi = RANGES
    raw = np.stack([raw_from_norm(xn[:, 0], lr_lo, lr_hi), raw_from_norm(xn[:, 1], le_lo, le_hi)], 1)
    # the library normalises raw inputs in FP64 then rounds to fp32; recover exactly what it sees
    xs = np.stack([(2 * (raw[:, 0] - lr_lo) / (lr_hi - lr_lo) - 1).astype(np.float32),
                   (2 * (raw[:, 1] - le_lo) / (le_hi - le_lo) - 1).astype(np.float32)], 1).astype(np.float64)
    assert np.array_equal(xs, xn)
    lT = raw_from_norm(tn, lt_lo, lt_hi)
    gctx.mlp_init(p.astype(np.float32), RANGES)
    yo = orc.mlp_forward(p, xn, round_bf16=True)
    yg = gctx.mlp_forward(torch.from_numpy(raw).cuda()).cpu().numpy()
    yg_n = 2 * (yg - lt_lo) / (lt_hi - lt_lo) - 1
    assert np.max(np.abs(yg_n - yo)) < 1e-6
    loss_g, grad_g = gctx.mlp_loss_grad(torch.from_numpy(raw).cuda(), torch.from_numpy(lT).cuda())
    loss_o, grad_o = orc.mlp_loss_grad(p, xn, tn, round_bf16=True)
    assert abs(loss_g - loss_o) <= 1e-6 * max(1.0, abs(loss_o))
    assert np.max(np.abs(grad_g - grad_o)) <= 1e-5 * max(1.0, np.abs(grad_o).max())


def test_gradient_matches_oracle_on_random_data(gctx, orc):
    """Random weights and inputs: the GPU accumulates in fp32 in the matrix
    cores' order, the oracle exactly, so a hidden activation whose fp32 sum
    lies within fp32 rounding of a bf16 rounding boundary can round one bf16
    step apart (a flip, ~2^-16 of the roundings).  Element by element: every
    sample's output and every gradient component agree to fp32 accumulation
    accuracy except a bounded number touched by flips, and those stay within
    the effect of a few flips."""
    import torch
    rng = np.random.default_rng(12)
    n = 4096
    p = (rng.normal(0, 0.3, orc.N_PARAMS)).astype(np.float32).astype(np.float64)
    xn = rng.uniform(-1, 1, (n, 2))
    lr_lo, lr_hi, le_lo, le_hi, lt_lo, lt_hi = RANGES
    raw = np.stack([raw_from_norm(xn[:, 0], lr_lo, lr_hi), raw_from_norm(xn[:, 1], le_lo, le_hi)], 1)
    xs = np.stack([(2 * (raw[:, 0] - lr_lo) / (lr_hi - lr_lo) - 1).astype(np.float32),
                   (2 * (raw[:, 1] - le_lo) / (le_hi - le_lo) - 1).astype(np.float32)], 1).astype(np.float64)
    tn = rng.uniform(-1, 1, n)
    lT = raw_from_norm(tn, lt_lo, lt_hi)
    tn_seen = (2 * (lT - lt_lo) / (lt_hi - lt_lo) - 1).astype(np.float32).astype(np.float64)
    gctx.mlp_init(p.astype(np.float32), RANGES)
    yo = orc.mlp_forward(p, xs, round_bf16=True)
    yg = gctx.mlp_forward(torch.from_numpy(raw).cuda()).cpu().numpy()
    yg_n = 2 * (yg - lt_lo) / (lt_hi - lt_lo) - 1
    dy = np.abs(yg_n - yo)
    ys = np.abs(yo).max()
    off_y = dy > 1e-5 * ys                 # outputs a flip reached
    print("forward: samples beyond fp32 accuracy", int(off_y.sum()), "of", n, "max", dy.max() / ys)
    assert off_y.sum() <= n // 100
    assert dy.max() <= 2e-2 * ys           # a few bf16 steps of one hidden unit
    loss_g, grad_g = gctx.mlp_loss_grad(torch.from_numpy(raw).cuda(), torch.from_numpy(lT).cuda())
    loss_o, grad_o = orc.mlp_loss_grad(p, xs, tn_seen, round_bf16=True)
    assert abs(loss_g / loss_o - 1) < 1e-4
    gs = np.abs(grad_o).max()
    dg = np.abs(grad_g - grad_o)
    off_g = dg > 1e-5 * gs
    print("gradient: components beyond fp32 accuracy", int(off_g.sum()), "of", grad_o.size, "max", dg.max() / gs)
    assert off_g.sum() <= grad_o.size // 100
    assert dg.max() <= 1e-3 * gs


def test_adam_step_matches_oracle(gctx, orc):
    """One and ten Adam steps from the same test-drawn gradients: the GPU's
    fp32 master weights equal the oracle's fp64 Adam element by element within
    fp32 rounding of each step (two units in the last place of the weight plus
    2^-18 of the step size, per step)."""
    rng = np.random.default_rng(14)
    p0 = rng.normal(0, 0.3, orc.N_PARAMS).astype(np.float32)
    gctx.mlp_init(p0, RANGES)
    w = p0.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    lr = 1e-3
    for k in range(1, 11):
        g = rng.normal(0, 1, orc.N_PARAMS).astype(np.float32)
        g[::37] *= np.float32(1e-5)                   # small components, where eps matters
        gctx.mlp_adam_step(g, lr)
        orc.mlp_adam(w, m, v, g.astype(np.float64), k, lr)
        if k in (1, 10):
            pg = gctx.mlp_params().astype(np.float64)
            tol = k * (2.0 ** -22 * np.abs(w) + 2.0 ** -18 * lr)
            d = np.abs(pg - w)
            print("Adam step", k, "max |gpu - oracle| / tol", (d / tol).max())
            assert np.all(d <= tol)
            assert np.all(np.abs(pg - p0) > 0)      # every weight moved


def _train_seed(ctx, saha, steps=2000, n=1 << 20, seed=1):
    """C4 recipe: 2^20 table samples, log rho ~ U[-12, 2], log e uniform between
    the row's values at 1e3 K and 1e8 K; labels from the table inversion."""
    import torch
    x = W.seed_training_samples(saha, n, seed)
    xt = torch.from_numpy(x).cuda()
    lT, _, _ = ctx.eos_invert(xt[:, 0].contiguous(), xt[:, 1].contiguous(), mode=0)
    p0 = W.mlp_init_params(seed=2)
    ctx.mlp_init(p0, W.seed_ranges(saha))
    loss = ctx.mlp_train(xt, lT, steps=steps, batch=4096, lr=1e-3, seed=seed)
    return loss


def test_training_on_gpu_reduces_loss_and_seeds_the_inversion(gctx, saha):
    import torch
    loss = _train_seed(gctx, saha, steps=600)
    assert np.all(np.isfinite(loss))
    assert loss[-20:].mean() < 0.05 * loss[:5].mean()
    gctx.mlp_enable_seed(True)
    xq = torch.from_numpy(W.seed_training_samples(saha, 1 << 16, 3)).cuda()
    lT0, j0, it0 = gctx.eos_invert(xq[:, 0].contiguous(), xq[:, 1].contiguous(), mode=0)
    lT1, j1, it1 = gctx.eos_invert(xq[:, 0].contiguous(), xq[:, 1].contiguous(), mode=1)
    torch.cuda.synchronize()
    assert torch.equal(j0, j1) and torch.equal(lT0, lT1)  # the seed never changes the answer
    pred = gctx.mlp_forward(xq).cpu().numpy()
    err = np.abs(pred - lT0.cpu().numpy())
    assert np.percentile(err, 50) < 5 * saha.dlT  # within a few table cells
    gctx.mlp_enable_seed(False)


def test_what_the_trained_network_gains_over_bisection(gctx, saha):
    """What the network gains: on queries of its training distribution with no
    history, its prediction starts the table search next to the answer, so the
    search reads far fewer table columns than the plain bisection does, and
    the answer is the same.  Column reads beyond the two end nodes both forms
    read: bisection one per halving (log2 of the node intervals, 8 on 256
    nodes) plus the right neighbour when the last halving left it unread;
    seeded, two per secant try (the cell's two nodes), and where the seed
    misses after newton_max_iter steps the same bisection on top."""
    import torch
    _train_seed(gctx, saha)  # the C4 recipe: 2000 steps
    gctx.mlp_enable_seed(True)
    xq = torch.from_numpy(W.seed_training_samples(saha, 1 << 16, 5)).cuda()
    lT0, j0, it0 = gctx.eos_invert(xq[:, 0].contiguous(), xq[:, 1].contiguous(), mode=0)
    lT1, j1, it1 = gctx.eos_invert(xq[:, 0].contiguous(), xq[:, 1].contiguous(), mode=1)
    torch.cuda.synchronize()
    gctx.mlp_enable_seed(False)
    assert torch.equal(j0, j1) and torch.equal(lT0, lT1)
    it0, it1 = it0.cpu().numpy(), it1.cpu().numpy()
    assert np.all(it0 == -1)                                 # mode 0: bisection every time
    halvings = int(np.ceil(np.log2(saha.nT - 1)))
    bisect_reads = halvings + 0.5                            # the right neighbour about half the time
    maxit = 4                                                # the context's newton_max_iter
    seeded = np.where(it1 >= 0, 2.0 * (it1 + 1), 2.0 * (maxit + 1) + bisect_reads)
    fallback = float(np.mean(it1 < 0))
    hist = np.bincount(it1[it1 >= 0], minlength=maxit + 1)
    print(f"column reads per query: bisection {bisect_reads:.1f}, network-seeded {seeded.mean():.2f}; "
          f"secant steps {hist.tolist()}, fallback rate {fallback:.2e}")
    assert fallback < 1e-3
    assert seeded.mean() < 0.5 * bisect_reads


def test_corrupted_network_changes_nothing(gctx, saha):
    """A broken seed (garbage weights) makes every query fall back; the
    inversion results are unchanged bit for bit."""
    import torch
    p = np.full(4417, 37.0, dtype=np.float32)
    gctx.mlp_init(p, W.seed_ranges(saha))
    gctx.mlp_enable_seed(True)
    xq = torch.from_numpy(W.seed_training_samples(saha, 1 << 14, 4)).cuda()
    lT0, j0, _ = gctx.eos_invert(xq[:, 0].contiguous(), xq[:, 1].contiguous(), mode=0)
    lT1, j1, it1 = gctx.eos_invert(xq[:, 0].contiguous(), xq[:, 1].contiguous(), mode=1)
    torch.cuda.synchronize()
    assert torch.equal(j0, j1) and torch.equal(lT0, lT1)
    gctx.mlp_enable_seed(False)


def test_hydro_with_learned_seed_equals_bisection_bitwise(gctx, saha):
    """C2 stream on a 2^3-block mesh: inv_mode 1 (network seed), 2 (bisected
    centre cells), 3 (centre cells carried between stages), 4 (a pass of
    network-started searches before each stage) and 0 (bisection) give the same
    state bit for bit."""
    from paper_2609_37859_amd import tdh as T
    import torch
    _train_seed(gctx, saha, steps=300)
    params = gctx.mlp_params()
    cfg, mesh, U = W.stream_c2(saha, nb=2)
    outs = []
    for mode in (0, 1, 2, 3, 4):
        ctx = T.Context(cfg, mesh, U, table=saha, inv_mode=mode)
        if mode in (1, 4):
            ctx.mlp_init(params, W.seed_ranges(saha))
            ctx.mlp_enable_seed(True)
        T.run_sync_steps(ctx, 3, dts=[3e-4] * 3)
        outs.append(ctx.get_state())
        ctx.close()
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_cfl_pass_records_the_first_stage_seeds(gctx, saha):
    """Modes 2 and 4: the CFL reduction records the table cell of every cell of
    the current state (the cells its bisection for the sound speed finds), so
    the window's first stage needs no seed pass;
    steps driven by the CFL step equal the bisection run bit for bit, also
    after a state upload between the reduction and the step (the recorded
    cells are then dropped)."""
    from paper_2609_37859_amd import tdh as T
    _train_seed(gctx, saha, steps=300)
    params = gctx.mlp_params()
    cfg, mesh, U = W.stream_c2(saha, nb=2)
    from tests.test_gpu_parity import _centre_cells
    outs, dts, cells = [], [], {}
    for mode in (0, 2, 4):
        ctx = T.Context(cfg, mesh, U, table=saha, inv_mode=mode)
        if mode == 4:
            ctx.mlp_init(params, W.seed_ranges(saha))
            ctx.mlp_enable_seed(True)
        assert np.all(ctx.seed_cells() == -1)
        ctx.reduce_dt()
        if mode:
            cells[mode] = ctx.seed_cells()
        else:
            assert np.all(ctx.seed_cells() == -1)  # mode 0 records nothing
        used = list(T.run_sync_steps(ctx, 3))
        g = ctx.get_state()
        ctx.reduce_dt()
        ctx.set_state(U)          # recorded cells of g dropped with the upload
        used += list(T.run_sync_steps(ctx, 1, dts=[3e-4]))
        outs.append((g, ctx.get_state()))
        dts.append(used)
        ctx.close()
    assert np.array_equal(cells[2], cells[4])
    exact = _centre_cells(gctx, cfg, mesh, U, saha)
    assert np.mean(cells[2] == exact) > 0.999, np.mean(cells[2] == exact)
    for o, d in zip(outs[1:], dts[1:]):
        assert d == dts[0]
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
