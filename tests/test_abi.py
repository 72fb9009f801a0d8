"""The C-ABI library loads and exports every function include/tdh.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os

import numpy as np
import pytest

from paper_2609_37859_amd import tdh as T


def test_header_declares_the_boundary():
    names = T.header_functions()
    for required in ("tdh_init", "tdh_init_blocks", "tdh_set_eos_table", "tdh_step_level", "tdh_reduce_dt"):
        assert required in names


def test_library_exports_every_header_symbol():
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtdh.so not built")
    L = ctypes.CDLL(T.LIB_PATH)
    missing = [n for n in T.header_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_arena_size_and_mesh_validation_without_gpu():
    """tdh_arena_bytes is pure host logic: check it against the layout sizes."""
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtdh.so not built")
    from paper_2609_37859_amd import workloads as W
    L = T.lib()
    cfg = W.Config(dual=1)
    mesh = W.uniform_mesh(2, 1, 1, 16, 0.1)
    c = T.make_config(cfg)
    m, keep = T.make_mesh(mesh)
    nb = L.tdh_arena_bytes(ctypes.byref(c), ctypes.byref(m))
    total = 2 * 6 * 16 ** 3 * 8
    imp = 2 * 6 * 6 * 16 ** 2 * 8
    assert nb >= 3 * total + 2 * imp
    bad = W.uniform_mesh(2, 1, 1, 12, 0.1)  # 12 is not a power of two
    m2, keep2 = T.make_mesh(bad)
    assert L.tdh_arena_bytes(ctypes.byref(c), ctypes.byref(m2)) == 0
    # two refinement levels: levels 0 and 1 accepted, anything else refused
    ref = np.zeros((2, 2, 2), dtype=bool)
    ref[1, 0, 1] = True
    amr = W.amr_mesh((2, 2, 2), 8, 0.1, ref)
    m3, keep3 = T.make_mesh(amr)
    assert L.tdh_arena_bytes(ctypes.byref(c), ctypes.byref(m3)) >= 3 * 6 * 8 ** 3 * 8 * amr.nblocks
    amr.rlev = amr.rlev.copy()
    amr.rlev[0] = 2
    m4, keep4 = T.make_mesh(amr)
    assert L.tdh_arena_bytes(ctypes.byref(c), ctypes.byref(m4)) == 0


def test_library_allocates_no_device_memory():
    """Every device byte a context uses is the caller's (arena, table buffer,
    gravity workspace) or the static per-GPU array of the allocation-free
    reduction: no source of the library calls a device allocator."""
    import re
    csrc = os.path.join(os.path.dirname(T.__file__), "csrc")
    pat = re.compile(r"\bhip(Malloc|MallocAsync|MallocManaged|ExtMallocWithFlags|MallocPitch|Malloc3D|HostMalloc|"
                     r"MallocFromPoolAsync|Free|FreeAsync|HostFree)\s*\(")
    hits = []
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".hpp")):
            for n, line in enumerate(open(os.path.join(csrc, f)), 1):
                if pat.search(line):
                    hits.append(f"{f}:{n}: {line.strip()}")
    assert not hits, hits
