"""Python binding of libtdh (include/tdh.h): argument marshalling only.

Every step of the update runs in the HIP library; PyTorch provides the device
arena and the stream.  There is no fallback: if libtdh.so is missing or a
call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdh.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tdh.h")


class TdhError(RuntimeError):
    pass


class tdh_config(C.Structure):
    _fields_ = [("eos_kind", C.c_int), ("dual", C.c_int), ("grav_kind", C.c_int), ("n_lat", C.c_int),
                ("gamma", C.c_double), ("eta1", C.c_double), ("eta2", C.c_double), ("cfl", C.c_double),
                ("rho_floor", C.c_double), ("p_floor", C.c_double), ("e_floor", C.c_double),
                ("merge_frac", C.c_double), ("gm_bh", C.c_double), ("r_soft", C.c_double), ("r_exc", C.c_double),
                ("bh_x0", C.c_double * 3), ("v_frame", C.c_double * 3),
                ("inv_mode", C.c_int), ("newton_max_iter", C.c_int), ("riemann", C.c_int),
                ("ghost_dense", C.c_int)]


class tdh_mesh(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("bc", C.c_int * 3),
                ("x0", C.c_double * 3), ("dx", C.c_double * 3), ("nblocks", C.c_int),
                ("blk", C.POINTER(C.c_int)), ("rlev", C.POINTER(C.c_int))]


class tdh_stats(C.Structure):
    _fields_ = [("block_updates", C.c_int64), ("cell_updates", C.c_int64), ("windows", C.c_int64),
                ("sub_cycles", C.c_int64), ("kernel_launches", C.c_int64), ("graph_captures", C.c_int64),
                ("capture_ms", C.c_double)]


_lib = None


def header_functions():
    """Names of the functions include/tdh.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tdh_[a-z0-9_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TdhError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc for gfx950)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, d, i, st = C.c_void_p, C.c_double, C.c_int, C.c_int
    ctx = vp
    sig = {
        "tdh_arena_bytes": ([P(tdh_config), P(tdh_mesh)], C.c_size_t),
        "tdh_init": ([P(tdh_config), vp, P(ctx)], st),
        "tdh_init_blocks": ([ctx, P(tdh_mesh), vp, C.c_size_t, P(d), P(d)], st),
        "tdh_set_eos_table": ([ctx, i, i, d, d, d, d, P(d), P(d), P(d), vp, C.c_size_t], st),
        "tdh_table_bytes": ([i, i], C.c_size_t),
        "tdh_reduce_dt": ([ctx, P(d), P(d), P(C.c_int8), P(i)], st),
        "tdh_reduce_dt_static": ([ctx, P(d), P(d), P(C.c_int8), P(i)], st),
        "tdh_set_levels": ([ctx, P(C.c_int8)], st),
        "tdh_step_level": ([ctx, i, d], st),
        "tdh_run_window": ([ctx, d, i, i], st),
        "tdh_get_time": ([ctx, P(d)], st),
        "tdh_set_time": ([ctx, d], st),
        "tdh_get_state": ([ctx, P(d)], st),
        "tdh_set_state": ([ctx, P(d)], st),
        "tdh_get_seed_cells": ([ctx, P(C.c_int32)], st),
        "tdh_gravity_workspace_bytes": ([ctx, P(C.c_size_t)], st),
        "tdh_gravity_solve": ([ctx, vp, C.c_size_t, d, i, d, i, P(i), P(d)], st),
        "tdh_get_potential": ([ctx, P(d)], st),
        "tdh_remap": ([ctx, ctx], st),
        "tdh_galilean_boost": ([ctx, P(d), d], st),
        "tdh_frame_acceleration": ([ctx, d, P(d)], st),
        "tdh_eos_invert_batch": ([ctx, vp, vp, vp, vp, vp, C.c_int64, i], st),
        "tdh_eos_eval_batch": ([ctx, vp, vp, vp, vp, C.c_int64], st),
        "tdh_get_stats": ([ctx, P(tdh_stats)], st),
        "tdh_last_error": ([ctx], C.c_char_p),
        "tdh_destroy": ([ctx], None),
        "tdh_num_tiles": ([], i),
        "tdh_tile_shape": ([i, P(i)], st),
        "tdh_set_tile": ([ctx, i], st),
        "tdh_get_tile": ([ctx, P(i)], st),
        "tdh_autotune": ([ctx, i, P(i), P(C.c_float)], st),
        "tdh_set_timing": ([ctx, i], st),
        "tdh_get_stage_time": ([ctx, P(d), P(C.c_int64)], st),
        "tdh_mlp_init": ([ctx, P(C.c_float), d, d, d, d, d, d], st),
        "tdh_mlp_train": ([ctx, vp, vp, C.c_int64, i, i, C.c_float, C.c_uint64, P(C.c_float)], st),
        "tdh_mlp_get_params": ([ctx, P(C.c_float)], st),
        "tdh_mlp_forward": ([ctx, vp, vp, C.c_int64], st),
        "tdh_mlp_loss_grad": ([ctx, vp, vp, C.c_int64, P(C.c_float), P(C.c_float)], st),
        "tdh_mlp_enable_seed": ([ctx, i], st),
        "tdh_mlp_adam_step": ([ctx, P(C.c_float), C.c_float], st),
    }
    for name, (args, res) in sig.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(cfg, inv_mode=0, newton_max_iter=4) -> tdh_config:
    c = tdh_config()
    for f, _ in tdh_config._fields_:
        if f == "inv_mode":
            c.inv_mode = inv_mode
        elif f == "newton_max_iter":
            c.newton_max_iter = newton_max_iter
        elif f in ("bh_x0", "v_frame"):
            getattr(c, f)[:] = [float(x) for x in getattr(cfg, f)]
        else:
            setattr(c, f, getattr(cfg, f))
    return c


def make_mesh(mesh):
    """tdh_mesh of a workloads.Mesh, and the arrays it points into (keep them alive)."""
    blk = np.ascontiguousarray(mesh.blk, dtype=np.int32)
    m = tdh_mesh()
    m.nx, m.ny, m.nz = mesh.nx, mesh.ny, mesh.nz
    m.bc[:] = list(mesh.bc)
    m.x0[:] = list(mesh.x0)
    m.dx[:] = list(mesh.dx)
    m.nblocks = mesh.nblocks
    m.blk = blk.ctypes.data_as(C.POINTER(C.c_int))
    keep = [blk]
    if getattr(mesh, "rlev", None) is not None:
        rlev = np.ascontiguousarray(mesh.rlev, dtype=np.int32)
        m.rlev = rlev.ctypes.data_as(C.POINTER(C.c_int))
        keep.append(rlev)
    return m, keep


class Context:
    """One library context on one GPU, owning a torch arena for the state."""

    def __init__(self, cfg, mesh, state, phi=None, table=None, inv_mode=0, newton_max_iter=4, device="cuda:0",
                 stream=None):
        import torch
        self.torch = torch
        self.L = lib()
        self.cfg, self.mesh = cfg, mesh
        self.nv = cfg.nv
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        # a stream of our own (default priority): graph capture needs a non-legacy stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._cfg = make_config(cfg, inv_mode, newton_max_iter)
        self._mesh, self._blk = make_mesh(mesh)
        nbytes = self.L.tdh_arena_bytes(C.byref(self._cfg), C.byref(self._mesh))
        if nbytes == 0:
            raise TdhError("tdh_arena_bytes rejected the mesh")
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self.arena.record_stream(self.stream)
        base = self.arena.data_ptr()
        self._arena_ptr = (base + 255) & ~255
        self.ctx = C.c_void_p()
        self._check(self.L.tdh_init(C.byref(self._cfg), C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx)),
                    "tdh_init", ctx=False)
        if table is not None:
            self.set_eos_table(table)
        st = np.ascontiguousarray(state, dtype=np.float64)
        if st.size != mesh.offsets(self.nv)[-1]:
            raise TdhError("state has the wrong size for this mesh")
        ph = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
        self._check(self.L.tdh_init_blocks(self.ctx, C.byref(self._mesh), C.c_void_p(self._arena_ptr), nbytes,
                                           _dp(st), None if ph is None else _dp(ph)), "tdh_init_blocks")

    def _enter(self, *tensors):
        """Order the library stream after torch's current stream (inputs ready)
        and keep the tensors alive for the library stream."""
        cur = self.torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        for t in tensors:
            t.record_stream(self.stream)

    def _dev64(self, t):
        return t.to(self.device, self.torch.float64).contiguous()

    def _leave(self):
        """Order torch's current stream after the library stream (outputs ready)."""
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _check(self, rc, what, ctx=True):
        if rc != 0:
            msg = self.L.tdh_last_error(self.ctx if ctx else None)
            raise TdhError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def set_eos_table(self, t):
        """Install the table; its packed device copy lives in a torch buffer
        owned here (the library allocates no device memory)."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (t.lP, t.le, t.lc2)]
        nbytes = self.L.tdh_table_bytes(t.nrho, t.nT)
        if nbytes == 0:
            raise TdhError("tdh_table_bytes rejected the table dimensions")
        buf = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        buf.record_stream(self.stream)
        ptr = (buf.data_ptr() + 255) & ~255
        self._check(self.L.tdh_set_eos_table(self.ctx, t.nrho, t.nT, t.lr0, t.dlr, t.lT0, t.dlT, *map(_dp, arrs),
                                             C.c_void_p(ptr), nbytes), "tdh_set_eos_table")
        old = getattr(self, "_table_buf", None)
        if old is not None:
            old.record_stream(self.stream)  # queued work may still read it
        self._table_buf = buf

    def reduce_dt(self, static=False):
        """CFL reduction and level assignment: (dt_block, dt0, levels, Lmax).
        static=True calls the allocation-free variant (tdh_reduce_dt_static)."""
        nb = self.mesh.nblocks
        dtb = np.zeros(nb)
        lev = np.zeros(nb, dtype=np.int8)
        dt0 = C.c_double()
        lmax = C.c_int()
        fn, name = (self.L.tdh_reduce_dt_static, "tdh_reduce_dt_static") if static else \
            (self.L.tdh_reduce_dt, "tdh_reduce_dt")
        self._check(fn(self.ctx, _dp(dtb), C.byref(dt0), lev.ctypes.data_as(C.POINTER(C.c_int8)), C.byref(lmax)), name)
        return dtb, dt0.value, lev.astype(np.int32), lmax.value

    def set_levels(self, levels):
        lev = np.ascontiguousarray(levels, dtype=np.int8)
        self._check(self.L.tdh_set_levels(self.ctx, lev.ctypes.data_as(C.POINTER(C.c_int8))), "tdh_set_levels")

    def step_level(self, level, dt):
        self._check(self.L.tdh_step_level(self.ctx, int(level), float(dt)), "tdh_step_level")

    def run_window(self, dt_coarse, batched=True, graph=False):
        self._check(self.L.tdh_run_window(self.ctx, float(dt_coarse), int(batched), int(graph)), "tdh_run_window")

    @property
    def time(self):
        t = C.c_double()
        self._check(self.L.tdh_get_time(self.ctx, C.byref(t)), "tdh_get_time")
        return t.value

    @time.setter
    def time(self, t):
        self._check(self.L.tdh_set_time(self.ctx, float(t)), "tdh_set_time")

    def get_state(self):
        out = np.empty(self.mesh.offsets(self.nv)[-1])
        self._check(self.L.tdh_get_state(self.ctx, _dp(out)), "tdh_get_state")
        return out

    def gravity_solve(self, four_pi_G, max_cycles, tol=0.0, warm=True):
        """Self-gravity potential of the current state into the stored potential
        (multigrid V-cycles, periodic).  The workspace (a device tensor owned
        here) keeps the solution, the warm start of the next call.  Returns
        (cycles run, RMS defects before and after each cycle)."""
        torch = self.torch
        nbytes = C.c_size_t()
        self._check(self.L.tdh_gravity_workspace_bytes(self.ctx, C.byref(nbytes)), "tdh_gravity_workspace_bytes")
        fresh = getattr(self, "_mg_work", None) is None or self._mg_work.numel() < nbytes.value + 256
        if fresh:
            self._mg_work = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
            self._mg_work.record_stream(self.stream)
        ptr = (self._mg_work.data_ptr() + 255) & ~255
        cyc = C.c_int()
        defects = np.zeros(max_cycles + 1)
        self._enter()
        self._check(self.L.tdh_gravity_solve(self.ctx, C.c_void_p(ptr), nbytes.value, float(four_pi_G),
                                             int(max_cycles), float(tol), int(warm and not fresh), C.byref(cyc),
                                             _dp(defects)), "tdh_gravity_solve")
        return cyc.value, defects[:cyc.value + 1]

    def potential_global(self):
        """The last solve's potential on the global grid [nz, ny, nx] (from the
        workspace, which holds it in red-black order)."""
        m = self.mesh
        n = m.nx * m.ny * m.nz
        ptr = (self._mg_work.data_ptr() + 255) & ~255
        base = self._mg_work.data_ptr()
        t = self._mg_work[ptr - base:ptr - base + 8 * n].view(self.torch.float64)
        self.sync()
        raw = t.cpu().numpy()
        k, j, i = np.meshgrid(np.arange(m.nz), np.arange(m.ny), np.arange(m.nx), indexing="ij")
        nat = (k * m.ny + j) * m.nx + i
        return raw[((i + j + k) & 1) * (n // 2) + (nat >> 1)]

    def remap_from(self, src):
        """This context's state becomes the restart remap of src's state."""
        self._check(self.L.tdh_remap(self.ctx, src.ctx), "tdh_remap")

    def galilean_boost(self, V, rho_skip):
        Va = np.ascontiguousarray(V, dtype=np.float64)
        self._check(self.L.tdh_galilean_boost(self.ctx, _dp(Va), float(rho_skip)), "tdh_galilean_boost")

    def frame_acceleration(self, rho_min):
        A = np.zeros(3)
        self._check(self.L.tdh_frame_acceleration(self.ctx, float(rho_min), _dp(A)), "tdh_frame_acceleration")
        return A

    def get_potential(self):
        out = np.empty(int(sum((int(n) + 2) ** 3 for n in self.mesh.blk[:, 0])))
        self._check(self.L.tdh_get_potential(self.ctx, _dp(out)), "tdh_get_potential")
        return out

    def seed_cells(self):
        """Seed table cells held for the current state (inv_mode 3), per cell."""
        out = np.empty(self.mesh.ncells, dtype=np.int32)
        self._check(self.L.tdh_get_seed_cells(self.ctx, out.ctypes.data_as(C.POINTER(C.c_int32))),
                    "tdh_get_seed_cells")
        return out

    def set_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        self._check(self.L.tdh_set_state(self.ctx, _dp(U)), "tdh_set_state")

    def eos_invert(self, lr, le, mode=0):
        torch = self.torch
        lr = lr.to(self.device, torch.float64).contiguous()
        le = le.to(self.device, torch.float64).contiguous()
        n = lr.numel()
        lT = torch.empty(n, dtype=torch.float64, device=self.device)
        j = torch.empty(n, dtype=torch.int32, device=self.device)
        it = torch.empty(n, dtype=torch.int32, device=self.device)
        self._enter(lr, le, lT, j, it)
        self._check(self.L.tdh_eos_invert_batch(self.ctx, lr.data_ptr(), le.data_ptr(), lT.data_ptr(), j.data_ptr(),
                                                it.data_ptr(), n, int(mode)), "tdh_eos_invert_batch")
        self._leave()
        return lT, j, it

    def eos_eval(self, rho, U):
        torch = self.torch
        rho = rho.to(self.device, torch.float64).contiguous()
        U = U.to(self.device, torch.float64).contiguous()
        P = torch.empty_like(rho)
        cs = torch.empty_like(rho)
        self._enter(rho, U, P, cs)
        self._check(self.L.tdh_eos_eval_batch(self.ctx, rho.data_ptr(), U.data_ptr(), P.data_ptr(), cs.data_ptr(),
                                              rho.numel()), "tdh_eos_eval_batch")
        self._leave()
        return P, cs

    def set_tile(self, tile_id):
        self._check(self.L.tdh_set_tile(self.ctx, int(tile_id)), "tdh_set_tile")

    def get_tile(self):
        t = C.c_int()
        self._check(self.L.tdh_get_tile(self.ctx, C.byref(t)), "tdh_get_tile")
        return t.value

    def autotune(self, reps=3):
        nt = self.L.tdh_num_tiles()
        ms = (C.c_float * nt)()
        best = C.c_int()
        self._check(self.L.tdh_autotune(self.ctx, int(reps), C.byref(best), ms), "tdh_autotune")
        return best.value, [float(x) for x in ms]

    def set_timing(self, on=True):
        self._check(self.L.tdh_set_timing(self.ctx, int(on)), "tdh_set_timing")

    def stage_time(self):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.L.tdh_get_stage_time(self.ctx, C.byref(ms), C.byref(n)), "tdh_get_stage_time")
        return ms.value, n.value

    # --- learned seed network ---
    def mlp_init(self, params, ranges):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == 4417
        self._check(self.L.tdh_mlp_init(self.ctx, p.ctypes.data_as(C.POINTER(C.c_float)), *map(float, ranges)),
                    "tdh_mlp_init")

    def mlp_train(self, x, lT, steps, batch=4096, lr=1e-3, seed=1):
        """x: device float64 [n, 2] (log10 rho, log10 e); lT: device float64 [n]."""
        x, lT = self._dev64(x), self._dev64(lT)
        loss = np.zeros(steps, dtype=np.float32)
        self._enter(x, lT)
        self._check(self.L.tdh_mlp_train(self.ctx, x.data_ptr(), lT.data_ptr(), x.shape[0], int(steps), int(batch),
                                         float(lr), int(seed), loss.ctypes.data_as(C.POINTER(C.c_float))),
                    "tdh_mlp_train")
        return loss

    def mlp_loss_grad(self, x, lT):
        x, lT = self._dev64(x), self._dev64(lT)
        g = np.zeros(4417, dtype=np.float32)
        loss = C.c_float()
        self._enter(x, lT)
        self._check(self.L.tdh_mlp_loss_grad(self.ctx, x.data_ptr(), lT.data_ptr(), x.shape[0], C.byref(loss),
                                             g.ctypes.data_as(C.POINTER(C.c_float))), "tdh_mlp_loss_grad")
        return loss.value, g

    def mlp_adam_step(self, grad, lr):
        g = np.ascontiguousarray(grad, dtype=np.float32)
        assert g.size == 4417
        self._check(self.L.tdh_mlp_adam_step(self.ctx, g.ctypes.data_as(C.POINTER(C.c_float)), float(lr)),
                    "tdh_mlp_adam_step")

    def mlp_forward(self, x):
        torch = self.torch
        x = self._dev64(x)
        out = torch.empty(x.shape[0], dtype=torch.float64, device=self.device)
        self._enter(x, out)
        self._check(self.L.tdh_mlp_forward(self.ctx, x.data_ptr(), out.data_ptr(), x.shape[0]), "tdh_mlp_forward")
        self._leave()
        return out

    def mlp_params(self):
        p = np.zeros(4417, dtype=np.float32)
        self._check(self.L.tdh_mlp_get_params(self.ctx, p.ctypes.data_as(C.POINTER(C.c_float))), "tdh_mlp_get_params")
        return p

    def mlp_enable_seed(self, on=True):
        self._check(self.L.tdh_mlp_enable_seed(self.ctx, int(on)), "tdh_mlp_enable_seed")

    def stats(self):
        s = tdh_stats()
        self._check(self.L.tdh_get_stats(self.ctx, C.byref(s)), "tdh_get_stats")
        return {f: getattr(s, f) for f, _ in tdh_stats._fields_}

    def sync(self):
        self.stream.synchronize()

    def close(self):
        if self.ctx:
            self.L.tdh_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_sync_steps(ctx: Context, nsteps, dts=None):
    """nsteps synchronous steps; dt from the library's CFL reduction unless given."""
    used = []
    for s in range(nsteps):
        if dts is None:
            _, dt, _, _ = ctx.reduce_dt()
        else:
            dt = float(dts[s])
        ctx.step_level(0, dt)
        used.append(dt)
    return np.array(used)


def tile_shapes():
    L = lib()
    out = []
    for t in range(L.tdh_num_tiles()):
        d = (C.c_int * 4)()
        L.tdh_tile_shape(t, d)
        out.append(tuple(d))
    return out
