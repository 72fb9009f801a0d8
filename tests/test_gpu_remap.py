"""Restart remap, Galilean boost and frame acceleration on the GPU (through the
C ABI) against the oracle."""
import numpy as np
import pytest

from paper_2609_37859_amd import workloads as W
from tests.parity import TOL, rel_err
from tests.test_oracle_remap import _vortex_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_37859_amd import tdh as T
    T.lib()
    return T


def _remap_gpu(T, cfg, src, U, dst, t=0.0):
    a = T.Context(cfg, src, U)
    a.time = t
    b = T.Context(cfg, dst, W.uniform_state(dst, cfg))
    b.remap_from(a)
    out, tb = b.get_state(), b.time
    a.close()
    b.close()
    assert tb == t
    return out


@pytest.mark.parametrize("case", ["identity", "refine_shifted", "coarsen", "outside_excision", "band_both_sides"])
def test_remap_matches_the_oracle(tdh, orc, case):
    if case == "identity":
        cfg = W.Config(dual=1)
        src, dst = W.uniform_mesh(2, 2, 2, 16, 1.0 / 32), W.uniform_mesh(4, 4, 4, 8, 1.0 / 32)
        t = 0.0
    elif case == "refine_shifted":
        cfg = W.Config(dual=1)
        src = W.uniform_mesh(2, 2, 2, 16, 1.0 / 32, bc=(0, 1, 1))
        dst = W.mixed_mesh((2, 2, 2), 32, np.eye(2, dtype=bool)[None].repeat(2, 0), 0.6 / 32,
                           x0=(0.1 / 3, 0.05, 0.0), bc=(0, 1, 1))
        t = 0.0
    elif case == "coarsen":
        cfg = W.Config()
        src, dst = W.uniform_mesh(2, 2, 2, 16, 1.0 / 32), W.uniform_mesh(2, 2, 2, 8, 1.0 / 16)
        t = 0.0
    elif case == "band_both_sides":  # larger target on both x faces and the high y face, finer, table-free
        cfg = W.Config(dual=1, rho_floor=1e-6, p_floor=1e-8)
        src = W.uniform_mesh(2, 2, 2, 8, 1.0 / 16, bc=(1, 1, 0))
        dst = W.uniform_mesh(5, 3, 2, 8, 1.0 / 24, x0=(-0.3, 0.1, 0.0), bc=(1, 1, 0))
        t = 0.0
    else:
        cfg = W.Config(dual=1, grav_kind=2, gm_bh=1.0, r_soft=0.01, r_exc=0.1, bh_x0=(0.5, 0.5, 0.5),
                       v_frame=(0.2, 0.0, 0.0), rho_floor=1e-6, p_floor=1e-8)
        src, dst = W.uniform_mesh(2, 2, 2, 8, 1.0 / 16, bc=(1, 1, 1)), W.uniform_mesh(3, 2, 2, 8, 1.0 / 16, bc=(1, 1, 1))
        t = 0.5
    U = _vortex_state(src, cfg)
    g = _remap_gpu(tdh, cfg, src, U, dst, t)
    o = orc.remap(cfg, src, U, dst, t=t)
    err = rel_err(cfg.nv, dst, g, o)
    print(case, "remap rel err", err, "bitwise", np.array_equal(g, o))
    assert np.all(err <= TOL)
    if case in ("identity", "outside_excision"):
        assert np.array_equal(g, o)


def test_galilean_boost_matches_the_oracle(tdh, orc):
    cfg = W.Config(dual=1)
    mesh = W.uniform_mesh(2, 2, 1, 16, 1.0 / 32)
    U = _vortex_state(mesh, cfg)
    V = np.array([0.3, -1.2, 2.0])
    ctx = tdh.Context(cfg, mesh, U)
    ctx.galilean_boost(V, 1.0)
    g = ctx.get_state()
    ctx.close()
    o = orc.galilean_boost(cfg, mesh, U, V, 1.0)
    assert np.all(rel_err(6, mesh, g, o) <= TOL)
    assert not np.array_equal(g, U)


def test_frame_acceleration_matches_the_oracle(tdh, orc):
    """The C5-shaped reduced debris stream with its point mass: the
    density-weighted field over dense, non-excised cells."""
    table = W.saha_table()
    cfg, mesh, U = W.debris_stream_c5(table, regions=(4, 3, 2), n_split=6, dxr=1.0)
    ctx = tdh.Context(cfg, mesh, U, table=table)
    ctx.time = 1234.5
    A = ctx.frame_acceleration(1e-6)
    ctx.close()
    o = orc.frame_acceleration(cfg, mesh, U, 1e-6, t=1234.5)
    print("frame acceleration", A, o)
    assert np.all(np.abs(A - o) <= 1e-12 * np.max(np.abs(o)))
    assert np.max(np.abs(o)) > 0
