"""Pins of the oracle's restart remap, Galilean boost and frame-acceleration
estimate (Sec. Domain remapping and frame conversion, eqs remap-cell-average,
galilean-boost; Sec. Moving-frame dynamics and BH treatment, eq
frame-acceleration) against facts fixed outside them."""
import math

import numpy as np

from paper_2609_37859_amd import workloads as W


def _vortex_state(mesh, cfg, rho0=1.0, p0=0.6):
    """Orszag-Tang-like velocity field v = (-sin 2 pi y, sin 2 pi x, 0) on a
    uniform, slightly perturbed density (the hydro part of the paper's remap
    example)."""
    def fn(x, y, z):
        rho = rho0 * (1 + 0.1 * np.cos(2 * np.pi * (x + z)))
        return W.ideal_conserved(rho, -np.sin(2 * np.pi * y), np.sin(2 * np.pi * x), 0 * x, p0 + 0 * x,
                                 cfg.gamma, cfg.dual == 1)
    return W.pack_state(mesh, cfg.nv, fn)


def _sums(mesh, nv, U, cfg):
    g = W.to_global(mesh, nv, U)
    K = 0.5 * (g[1] ** 2 + g[2] ** 2 + g[3] ** 2) / g[0]
    vol = mesh.dx[0] * mesh.dx[1] * mesh.dx[2]
    return {"M": math.fsum(g[0].ravel()) * vol, "E": math.fsum(g[4].ravel()) * vol,
            "K": math.fsum(K.ravel()) * vol, "U": math.fsum((g[4] - K).ravel()) * vol}


def test_remap_onto_the_same_grid_is_the_identity(orc):
    """The same global grid cut into other blocks: every value copied exactly."""
    cfg = W.Config(dual=1)
    src = W.uniform_mesh(2, 2, 2, 16, 1.0 / 32)
    dst = W.uniform_mesh(4, 4, 4, 8, 1.0 / 32)
    U = _vortex_state(src, cfg)
    V = orc.remap(cfg, src, U, dst)
    assert np.array_equal(W.to_global(dst, 6, V), W.to_global(src, 6, U))


def test_remap_reproduces_linear_fields(orc):
    """Linear density, momentum and thermal energy on an outflow box, remapped
    onto a finer grid shifted by a third of a source cell: midpoint sampling of
    the trilinear interpolant is exact for linear fields, so interior target
    cells get the fields' values at their centres."""
    cfg = W.Config(dual=1)
    src = W.uniform_mesh(2, 2, 2, 8, 0.1, bc=(1, 1, 1))
    dst = W.uniform_mesh(2, 2, 2, 8, 0.06, x0=(0.1 / 3, 0.1 / 3, 0.1 / 3), bc=(1, 1, 1))
    lin = lambda x, y, z: (1.0 + 0.3 * x - 0.2 * y + 0.1 * z, 0.5 + x - 2 * z, -0.4 + y, 0.2 * z,
                           2.0 + 0.5 * x + 0.25 * y - 0.1 * z)

    def fn(x, y, z):
        rho, mx, my, mz, u = lin(x, y, z)
        return [rho, mx, my, mz, u + 0.5 * (mx * mx + my * my + mz * mz) / rho, u]
    U = W.pack_state(src, 6, fn)
    V = orc.remap(cfg, src, U, dst)
    G = W.to_global(dst, 6, V)
    want = np.zeros_like(G)
    for b in range(dst.nblocks):
        x, y, z = W.cell_centres(dst, b)
        n, ox, oy, oz = dst.blk[b]
        q = fn(x, y, z)
        for v in range(6):
            want[v, oz:oz + n, oy:oy + n, ox:ox + n] = q[v]
    # interior: every sample's stencil inside the source domain (0.05 .. 1.55 in source units)
    c = (np.arange(16) + 0.5) * 0.06 + 0.1 / 3
    inner = (c - 0.015 > 0.05) & (c + 0.015 < 1.55)
    sel = np.ix_(inner, inner, inner)
    for v in range(6):
        assert np.allclose(G[v][sel], want[v][sel], rtol=1e-13, atol=1e-13), v


def test_coarsening_carries_thermal_energy(orc):
    """The paper's remap example in hydro form: onto a grid twice as coarse,
    mass and internal energy are kept to rounding (each target cell's eight
    samples are the source cell centres), and the total energy falls by
    exactly the kinetic energy of the velocity structure the coarse cells
    cannot represent (a total-energy remap would turn that into heat)."""
    cfg = W.Config()
    src = W.uniform_mesh(2, 2, 2, 16, 1.0 / 32)
    dst = W.uniform_mesh(2, 2, 2, 8, 1.0 / 16)
    U = _vortex_state(src, cfg)
    V = orc.remap(cfg, src, U, dst)
    a, b = _sums(src, 5, U, cfg), _sums(dst, 5, V, cfg)
    assert abs(b["M"] - a["M"]) <= 1e-14 * a["M"]
    assert abs(b["U"] - a["U"]) <= 1e-13 * a["U"]
    lost = a["K"] - b["K"]
    assert lost > 1e-3 * a["K"]                        # coarsening loses kinetic energy
    assert abs((a["E"] - b["E"]) - lost) <= 1e-12 * a["E"]
    print("kinetic energy lost to coarsening, per cent of the internal energy:", 100 * lost / a["U"])


def test_remap_outside_and_excision(orc):
    """Target cells whose centres lie outside a non-periodic source domain get
    the floor state; cells inside the excision sphere get the sink state."""
    cfg = W.Config(dual=1, grav_kind=2, gm_bh=1.0, r_soft=0.01, r_exc=0.1, bh_x0=(0.5, 0.5, 0.5),
                   v_frame=(0.2, 0.0, 0.0), rho_floor=1e-6, p_floor=1e-8)
    src = W.uniform_mesh(2, 2, 2, 8, 1.0 / 16, bc=(1, 1, 1))
    dst = W.uniform_mesh(3, 2, 2, 8, 1.0 / 16, bc=(1, 1, 1))  # one more block of x beyond the source
    U = _vortex_state(src, cfg)
    t = 0.5
    V = orc.remap(cfg, src, U, dst, t=t)
    G = W.to_global(dst, 6, V)
    uf = cfg.p_floor / (cfg.gamma - 1)
    assert np.all(G[0][:, :, 16:] == cfg.rho_floor) and np.all(G[4][:, :, 16:] == uf)
    c = (np.arange(16) + 0.5) / 16
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    inside = (X - (0.5 - 0.2 * t)) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2 < 0.01
    assert inside.sum() > 0
    assert np.all(G[0][:, :, :16][inside] == cfg.rho_floor) and np.all(G[1][:, :, :16][inside] == 0.0)
    # the coincident grid copies every other cell but those of the band inside
    # the face the target extends beyond (x = 1: two source cells, 14 and 15)
    keep = ~inside
    keep[:, :, 14:] = False
    assert np.array_equal(G[:, :, :, :16][:, keep], W.to_global(src, 6, U)[:, keep])


def test_remap_blends_into_the_floor_across_a_band(orc):
    """Target domain larger than the source on both sides of x (outflow): the
    remapped state reaches the floor state smoothly.  Along x, density and
    thermal pressure fall monotonically from the source values to the floor
    values over the band inside each extended face and are unchanged beyond
    it; density and pressure move by the same fraction of their way to the
    floor (one blending weight); the velocity goes to rest; and where the
    target does not extend past a face (y, z) nothing is blended."""
    cfg = W.Config(rho_floor=1e-6, p_floor=1e-8)
    src = W.uniform_mesh(2, 2, 2, 8, 1.0 / 16, bc=(1, 1, 1))
    dst = W.uniform_mesh(4, 2, 2, 8, 1.0 / 16, x0=(-0.5, 0.0, 0.0), bc=(1, 1, 1))
    rho0, P0, v0 = 2.0, 0.5, 0.3

    def fn(x, y, z):
        return W.ideal_conserved(rho0 + 0 * x, v0 + 0 * x, 0 * x, 0 * x, P0 + 0 * x, cfg.gamma, False)
    U = W.pack_state(src, 5, fn)
    G = W.to_global(dst, 5, orc.remap(cfg, src, U, dst))
    rho = G[0]
    P = (cfg.gamma - 1) * (G[4] - 0.5 * (G[1] ** 2 + G[2] ** 2 + G[3] ** 2) / G[0])
    for a in (rho, P, G[1]):                       # uniform across y and z
        assert np.all(a == a[:1, :1, :])
    r, p, m = rho[0, 0], P[0, 0], G[1][0, 0]
    # x cells 0..7 and 24..31 lie outside the source: floor; 8..23 inside
    assert np.all(r[:8] == cfg.rho_floor) and np.all(r[24:] == cfg.rho_floor) and np.all(m[:8] == 0)
    assert np.all(r[10:22] == rho0) and np.allclose(p[10:22], P0, rtol=1e-14)      # beyond the band
    band = np.r_[8:10, 22:24]
    assert np.all((r[band] > cfg.rho_floor) & (r[band] < rho0))
    assert r[8] < r[9] and r[23] < r[22]                                       # rising into the domain
    fr = (r[band] - cfg.rho_floor) / (rho0 - cfg.rho_floor)
    fp = (p[band] - cfg.p_floor) / (P0 - cfg.p_floor)
    assert np.allclose(fr, fp, rtol=1e-12)
    assert np.allclose(m[band], fr * rho0 * v0, rtol=1e-12)                   # velocity brought to rest the same way
    assert np.allclose(fr[:2], fr[2:][::-1], rtol=1e-12)                       # symmetric faces


def test_galilean_boost(orc):
    """Velocities shift by V, the internal energy E - |m|^2/2rho is unchanged,
    floor-density cells are untouched, and boosting back restores the state."""
    cfg = W.Config(dual=1)
    mesh = W.uniform_mesh(2, 1, 1, 8, 1.0 / 16)
    U = _vortex_state(mesh, cfg)
    g = W.to_global(mesh, 6, U)
    V = np.array([0.3, -1.2, 2.0])
    B = orc.galilean_boost(cfg, mesh, U, V, rho_skip=1.0)
    h = W.to_global(mesh, 6, B)
    move = g[0] > 1.0
    assert move.sum() > 0 and (~move).sum() > 0
    for d in range(3):
        assert np.allclose((h[1 + d] / h[0])[move], (g[1 + d] / g[0])[move] + V[d], rtol=0, atol=1e-14)
    Ku = lambda q: q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
    assert np.allclose(Ku(h)[move], Ku(g)[move], rtol=1e-12, atol=1e-12)
    assert np.array_equal(h[:, ~move], g[:, ~move]) and np.array_equal(h[5], g[5])
    back = W.to_global(mesh, 6, orc.galilean_boost(cfg, mesh, B, -V, rho_skip=1.0))
    assert np.allclose(back, g, rtol=1e-13, atol=1e-13)


def test_frame_acceleration(orc):
    """One dense cell: the frame acceleration is the point mass's field at its
    centre, -GM r / (r^2 + r_soft^2)^(3/2); two dense cells: the mass-weighted
    mean; floor-density and excised cells do not count."""
    cfg = W.Config(grav_kind=2, gm_bh=2.0, r_soft=0.05, r_exc=0.1, bh_x0=(0.25, 0.5, 0.5), v_frame=(0.1, 0, 0))
    mesh = W.uniform_mesh(1, 1, 1, 8, 1.0 / 8)
    rho = np.full((8, 8, 8), 1e-8)
    rho[2, 3, 6] = 2.0
    rho[5, 1, 1] = 3.0
    rho[3, 3, 1] = 50.0   # centre (0.1875, 0.4375, 0.4375): inside the excision sphere at t = 0.5
    U = W.pack_state(mesh, 5, lambda x, y, z: W.ideal_conserved(
        rho[np.floor(z * 8).astype(int), np.floor(y * 8).astype(int), np.floor(x * 8).astype(int)],
        0 * x, 0 * x, 0 * x, 1.0 + 0 * x, cfg.gamma, False))
    t = 0.5
    bh = np.array([0.25 - 0.1 * t, 0.5, 0.5])

    def g(i, j, k):
        r = np.array([(i + 0.5) / 8, (j + 0.5) / 8, (k + 0.5) / 8]) - bh
        return -cfg.gm_bh * r / (r @ r + cfg.r_soft ** 2) ** 1.5
    A = orc.frame_acceleration(cfg, mesh, U, rho_min=1e-4, t=t)
    want = (2.0 * g(6, 3, 2) + 3.0 * g(1, 1, 5)) / 5.0
    assert np.allclose(A, want, rtol=1e-13, atol=0), (A, want)
