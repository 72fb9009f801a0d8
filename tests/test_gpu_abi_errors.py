"""Error behaviour of the C ABI (include/tdh.h): calls out of range or out of
schedule return their documented status, with a message, and leave the
context usable; nothing is launched for them."""
import numpy as np
import pytest

from paper_2609_37859_amd import workloads as W

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def tdh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_37859_amd import tdh as T
    T.lib()
    return T


def _lat_context(T):
    cfg = W.Config(n_lat=1)
    mesh = W.uniform_mesh(2, 1, 1, 8, 1.0 / 16)
    U = W.uniform_state(mesh, cfg)
    return T.Context(cfg, mesh, U), mesh, U


def test_stepping_out_of_range_or_schedule(tdh):
    ctx, mesh, U = _lat_context(tdh)
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        ctx.step_level(0, 0.0)
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        ctx.run_window(-1.0)
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        ctx.run_window(float("nan"))
    ctx.set_levels(np.array([0, 1], dtype=np.int8))
    with pytest.raises(tdh.TdhError, match=r"\(-4\)"):
        ctx.step_level(1, 1e-3)          # sub-cycle 0 advances level 0
    ctx.step_level(0, 1e-3)              # sub-cycle 0 of a two-sub-cycle window
    with pytest.raises(tdh.TdhError, match=r"\(-4\)"):
        ctx.reduce_dt()                  # inside a window
    with pytest.raises(tdh.TdhError, match=r"\(-4\)"):
        ctx.get_state()
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        ctx.step_level(1, 1e-3)          # dt * 2^level must equal the window's coarse step
    ctx.step_level(1, 0.5e-3)            # completes the window
    assert ctx.time == pytest.approx(1e-3, rel=0, abs=0)
    assert np.allclose(ctx.get_state(), U, rtol=1e-13, atol=0)   # a uniform state stays uniform
    ctx.close()


def test_levels_tiles_and_optional_parts(tdh):
    ctx, mesh, U = _lat_context(tdh)
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        ctx.set_levels(np.array([0, 31], dtype=np.int8))
    big = W.uniform_mesh(3, 1, 1, 8, 1.0 / 24, bc=(1, 1, 1))
    c3 = tdh.Context(W.Config(n_lat=2), big, W.uniform_state(big, W.Config(n_lat=2)))
    c3.set_levels(np.array([0, 1, 2], dtype=np.int8))       # neighbours one level apart
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        c3.set_levels(np.array([0, 2, 0], dtype=np.int8))   # a jump of two
    c3.close()
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        ctx.set_tile(len(tdh.tile_shapes()))
    with pytest.raises(tdh.TdhError, match=r"\(-4\)"):
        ctx.gravity_solve(1.0, 2)        # grav_kind 0: no stored potential
    with pytest.raises(tdh.TdhError, match=r"\(-4\)"):
        ctx.frame_acceleration(1e-6)     # no point mass
    with pytest.raises(tdh.TdhError, match=r"\(-4\)"):
        ctx.seed_cells()                 # no table EOS
    with pytest.raises(tdh.TdhError, match=r"\(-4\)"):
        ctx.mlp_enable_seed(True)        # before tdh_mlp_init
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        ctx.galilean_boost(np.array([np.inf, 0.0, 0.0]), 0.0)
    # the context is still usable after every refusal
    _, dt0, lev, L = ctx.reduce_dt()
    ctx.run_window(dt0 * 2 ** L)
    assert np.allclose(ctx.get_state(), U, rtol=1e-13, atol=0)
    ctx.close()


def test_remap_between_different_variable_sets(tdh):
    a_cfg, b_cfg = W.Config(dual=1), W.Config(dual=0)
    mesh = W.uniform_mesh(1, 1, 1, 8, 1.0 / 8)
    a = tdh.Context(a_cfg, mesh, W.uniform_state(mesh, a_cfg))
    b = tdh.Context(b_cfg, mesh, W.uniform_state(mesh, b_cfg))
    with pytest.raises(tdh.TdhError, match=r"\(-1\)"):
        b.remap_from(a)
    a.close()
    b.close()


def test_window_graphs_are_captured_once_per_lmax(tdh):
    """A window replayed from a graph is captured the first time its Lmax (and
    launch form) occurs and replayed afterwards; tdh_stats counts the captures
    and their host time."""
    big = W.uniform_mesh(3, 1, 1, 8, 1.0 / 24, bc=(1, 1, 1))
    cfg = W.Config(n_lat=2)
    ctx = tdh.Context(cfg, big, W.uniform_state(big, cfg))
    _, dt0, _, _ = ctx.reduce_dt()
    assert ctx.stats()["graph_captures"] == 0
    ctx.set_levels(np.array([0, 1, 2], dtype=np.int8))      # Lmax 2
    for _ in range(2):
        ctx.run_window(dt0, batched=True, graph=True)
    st = ctx.stats()
    assert st["graph_captures"] == 1 and st["capture_ms"] > 0.0 and st["windows"] == 2
    ctx.set_levels(np.array([0, 0, 0], dtype=np.int8))      # Lmax 0: a graph of its own
    for _ in range(2):
        ctx.run_window(dt0, batched=True, graph=True)
    ctx.set_levels(np.array([0, 1, 2], dtype=np.int8))      # Lmax 2 again: replayed
    ctx.run_window(dt0, batched=True, graph=True)
    ctx.run_window(dt0, batched=True, graph=False)          # no graph: nothing captured
    st = ctx.stats()
    assert st["graph_captures"] == 2 and st["windows"] == 6
    ctx.close()
