"""The allocation-free CFL reduction (tdh_reduce_dt_static) against
tdh_reduce_dt through the C ABI: bit-identical per-block steps, base step,
levels and finest level, on two calls in a row on one GPU, the second on a
smaller mesh (the shared device scratch keeps the first call's contents)."""
import dataclasses

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


def _same(a, b):
    return np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2]) and a[3] == b[3]


def test_static_reduction_equals_the_reduction(tdh, saha):
    # first call: the production-shaped sub-domain (mixed blocks, table EOS,
    # moving point mass, LAT), after a window so the state has moved on
    cfg, mesh, U = W.debris_stream_c5(saha, regions=(4, 3, 2), n_split=6, dxr=1.0)
    ctx = tdh.Context(cfg, mesh, U, table=saha, inv_mode=2)
    r = ctx.reduce_dt()
    ctx.run_window(r[1] * 2 ** r[3], batched=True)
    a = ctx.reduce_dt(static=True)
    b = ctx.reduce_dt()
    assert _same(a, b) and a[3] > 0
    ctx.close()
    # second call: a smaller mesh (fewer work items and blocks), single level,
    # after a window whose second stages left their CFL minima
    cfg2, mesh2, U2 = W.stream_c2(saha, nb=2)
    assert mesh2.ncells < mesh.ncells and mesh2.nblocks < mesh.nblocks
    ctx = tdh.Context(cfg2, mesh2, U2, table=saha, inv_mode=4)
    r = ctx.reduce_dt()
    ctx.run_window(r[1], batched=True)
    a = ctx.reduce_dt(static=True)
    b = ctx.reduce_dt()
    assert _same(a, b)
    # and the window it starts runs as after the other reduction
    ctx.run_window(a[1], batched=True)
    g_static = ctx.get_state()
    ctx.close()
    ref = tdh.Context(cfg2, mesh2, U2, table=saha, inv_mode=4)
    r = ref.reduce_dt()
    ref.run_window(r[1], batched=True)
    b = ref.reduce_dt()
    ref.run_window(b[1], batched=True)
    assert np.array_equal(ref.get_state(), g_static)
    ref.close()
