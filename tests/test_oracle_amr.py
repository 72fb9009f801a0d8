"""Pins of the oracle's two-level (coarse-fine) LAT (Sec. LAT method): the
factor rule f_fine <= f_coarse <= 2 f_fine, ghost states of neighbours on
another refinement level (restriction of the stored histories, time
interpolation, then prolongation), and the flux correction at coarse-fine
faces.

The pins hold the oracle to properties the mathematics fixes, not to its own
formulas:
  * prolongation reproduces linear data exactly, and the 2x2x2 children of a
    coarse cell average back to it (the operator conserves);
  * a limited prolongation leaves no slope along an axis where the coarse
    cell is a local extremum;
  * restriction of linear data is the coarse cell's centre value;
  * the factor assignment is the greatest one under the CFL bins that obeys
    the neighbour rules (a shortest-path computation here);
  * uniform flow stays uniform bit for bit through mixed levels and factors;
  * a periodic run conserves mass, momentum and energy to rounding;
  * a uniform gas accelerated by a uniform field stays spatially uniform when
    ghosts use the RK2 dense output (which is exact for the quadratic-in-time
    energy), and follows v = g t exactly.
"""
import math

import numpy as np
import pytest

from paper_2609_37859_amd import workloads as W

N = 8


def _mesh(refined, nb=(4, 4, 4), bc=(1, 1, 1), dx=0.125):
    ref = np.zeros(nb[::-1], dtype=bool)
    for cx, cy, cz in refined:
        ref[cz, cy, cx] = True
    return W.amr_mesh(nb, N, dx, ref, bc=bc)


def _level0_box(mesh, b):
    """Extent of block b in level-0 cells: lo[3], edge."""
    r = mesh.level(b)
    n = int(mesh.blk[b, 0])
    return np.array([int(mesh.blk[b, 1 + d]) for d in range(3)]) / 2 ** r, n / 2 ** r


def _covering_level(mesh, xyz):
    """Refinement level of the block whose box contains point xyz."""
    for b in range(mesh.nblocks):
        lo, e = _level0_box(mesh, b)
        p = (np.asarray(xyz) - np.asarray(mesh.x0)) / np.asarray(mesh.dx)
        if np.all(p >= lo) and np.all(p < lo + e):
            return mesh.level(b)
    return None


def _linear_state(mesh, nv, seed):
    rng = np.random.default_rng(seed)
    c0 = rng.uniform(2.0, 3.0, nv)
    g = rng.uniform(-0.5, 0.5, (nv, 3))

    def fn(x, y, z):
        return [c0[v] + g[v, 0] * x + g[v, 1] * y + g[v, 2] * z for v in range(nv)]
    return W.pack_state(mesh, nv, fn), fn


def test_amr_mesh_geometry():
    mesh = _mesh([(1, 1, 1)])
    assert mesh.nblocks == 63 + 8 and mesh.refined
    fine = [b for b in range(mesh.nblocks) if mesh.level(b) == 1]
    assert len(fine) == 8
    vol = sum(W.block_volume(mesh, b) * N ** 3 for b in range(mesh.nblocks))
    assert vol == pytest.approx((4 * N * 0.125) ** 3, rel=1e-15)
    # the eight children of a coarse cell average to its centre
    x, y, z = W.cell_centres(mesh, fine[0])
    assert x[0, 0, :2].mean() == pytest.approx((N + 0.5) * 0.125, rel=1e-15)


@pytest.mark.parametrize("refined", [[(1, 1, 1)], [(1, 1, 1), (2, 1, 1), (1, 2, 2)]])
def test_ghosts_of_linear_data_are_exact(orc, refined):
    """Restriction and limited prolongation reproduce a linear field: every
    ghost cell (face, edge and corner, either level) holds the field at its
    centre; only ghosts beyond the outflow edges are excluded."""
    mesh = _mesh(refined)
    cfg = W.Config(dual=0)
    U, fn = _linear_state(mesh, cfg.nv, seed=3)
    hi = np.array([mesh.nx, mesh.ny, mesh.nz]) * np.array(mesh.dx)
    checked = 0
    for b in range(mesh.nblocks):
        pad = orc.ghost_fill(cfg, mesh, U, b)
        x, y, z = W.cell_centres(mesh, b, ghost=2)
        inside = (x > 0) & (x < hi[0]) & (y > 0) & (y < hi[1]) & (z > 0) & (z < hi[2])
        exp = np.stack([np.asarray(q) for q in fn(x, y, z)])
        err = np.abs(pad - exp)[:, inside].max()
        assert err <= 1e-14 * 4, (b, err)
        checked += 1
    assert checked == mesh.nblocks


def _fine_ghost_groups(mesh, b):
    """For fine block b: map coarse cell (level-0 global index) -> list of pad
    indices (k, j, i) of the fine ghost cells inside it that lie on the
    coarse side (their level-0 cell is covered by a level-0 block)."""
    n = int(mesh.blk[b, 0])
    o = mesh.blk[b, 1:4].astype(int)
    groups = {}
    for kk in range(-2, n + 2):
        for jj in range(-2, n + 2):
            for ii in range(-2, n + 2):
                G = o + np.array([ii, jj, kk])
                c0 = tuple(G // 2)
                centre = (np.array(c0) + 0.5) * np.array(mesh.dx)
                if _covering_level(mesh, centre) != 0:
                    continue
                groups.setdefault(c0, []).append((kk + 2, jj + 2, ii + 2))
    return groups


def test_prolongation_conserves_and_limits(orc):
    """The eight prolonged children of a coarse cell average to the coarse
    value (random data), and where the coarse data have an extremum along x
    the two x-children agree."""
    mesh = _mesh([(1, 1, 1)])
    cfg = W.Config(dual=0)
    rng = np.random.default_rng(11)
    U = np.ascontiguousarray(rng.uniform(1.0, 2.0, mesh.ncells * cfg.nv))
    coarse_val = {}
    for c in range(mesh.nblocks):
        if mesh.level(c):
            continue
        q = W.unpack_block(mesh, cfg.nv, U, c)
        o = mesh.blk[c, 1:4].astype(int)
        for k in range(N):
            for j in range(N):
                for i in range(N):
                    coarse_val[(o[0] + i, o[1] + j, o[2] + k)] = q[:, k, j, i]
    fine = [b for b in range(mesh.nblocks) if mesh.level(b) == 1]
    full = 0
    for b in fine:
        pad = orc.ghost_fill(cfg, mesh, U, b)
        for c0, cells in _fine_ghost_groups(mesh, b).items():
            if len(cells) != 8:
                continue
            full += 1
            kids = np.stack([pad[:, k, j, i] for k, j, i in cells])
            assert np.allclose(kids.mean(axis=0), coarse_val[c0], rtol=2e-16 * 8, atol=0)
    assert full >= 6 * 16
    # extremum along x: a field with a ridge at one coarse column
    def ridge(x, y, z):
        xc = (N + 2.5) * 0.125  # centre of coarse cell i = N + 2 (inside the first fine block's x range)
        return [2.0 + 0.1 * y + 0.05 * z - (x - xc) ** 2 * (1.0 + 0 * x) for _ in range(cfg.nv)]
    U2 = W.pack_state(mesh, cfg.nv, ridge)
    b = fine[0]  # fine block with origin (2N, 2N, 2N); its y- face neighbour is coarse
    pad = orc.ghost_fill(cfg, mesh, U2, b)
    # ghost row below the block (y side, pad j = 0, 1) at the fine x-children of coarse i = N + 2
    ii = np.array([2 * (N + 2), 2 * (N + 2) + 1]) - 2 * N + 2
    for kk in range(2, N + 2):
        for jj in (0, 1):
            a, c = pad[:, kk, jj, ii[0]], pad[:, kk, jj, ii[1]]
            assert np.array_equal(a, c)
    # a monotone coarse column gives distinct children
    assert not np.array_equal(pad[:, 2, 0, ii[0] - 2], pad[:, 2, 0, ii[1] - 2])


def _adjacent(mesh, a, b):
    """Boxes in level-0 units touch (face, edge or corner), periodic axes wrapped."""
    if a == b:
        return False
    Ns = (mesh.nx, mesh.ny, mesh.nz)
    la, ea = _level0_box(mesh, a)
    lb, eb = _level0_box(mesh, b)
    for d in range(3):
        shifts = (-Ns[d], 0, Ns[d]) if mesh.bc[d] == 0 else (0,)
        if not any(lb[d] + s <= la[d] + ea and la[d] <= lb[d] + s + eb for s in shifts):
            return False
    return True


def test_factor_rule_across_levels_is_greatest_admissible(orc):
    """eq lat-factor then the neighbour rules: same level |e_b - e_c| <= 1,
    coarse-fine e_fine <= e_coarse <= e_fine + 1 (f = 2^e).  The oracle's
    relaxation must reach the greatest admissible exponents below the CFL
    bins, which is a shortest-path problem: e_b = min_c (e0_c + dist(b, c)),
    dist over the constraint graph (Floyd-Warshall here)."""
    mesh = _mesh([(1, 1, 1), (2, 1, 1), (0, 3, 2)], bc=(0, 1, 0))
    nb = mesh.nblocks
    adj = [[c for c in range(nb) if _adjacent(mesh, b, c)] for b in range(nb)]
    INF = 10 ** 6
    D = np.full((nb, nb), INF, dtype=np.int64)
    np.fill_diagonal(D, 0)
    for b in range(nb):
        for c in adj[b]:
            rb, rc = mesh.level(b), mesh.level(c)
            w = 0 if rb > rc else 1  # e_b <= e_c + w
            D[b, c] = min(D[b, c], w)
    for m in range(nb):
        D = np.minimum(D, D[:, m:m + 1] + D[m:m + 1, :])
    rng = np.random.default_rng(5)
    cfg = W.Config(n_lat=4, merge_frac=0.0)
    split = 0
    for trial in range(4):
        dtb = 1e-3 * 2.0 ** rng.uniform(0, 6, nb)
        lev, L, dt0 = orc.lat_assign(cfg, mesh, dtb)
        e0 = np.array([min(4, math.frexp(t / dtb.min())[1] - 1) for t in dtb])
        expect = (e0[None, :] + D).min(axis=1)
        got = L - lev
        assert np.array_equal(got, expect), trial
        for b in range(nb):
            for c in adj[b]:
                if mesh.level(b) == 1 and mesh.level(c) == 0:
                    assert got[b] <= got[c] <= got[b] + 1
        split += sum(mesh.level(b) == 1 and mesh.level(c) == 0 and got[b] < got[c]
                     for b in range(nb) for c in adj[b])
    assert split > 0  # coarse-fine faces with f_coarse = 2 f_fine occur


def _levels_for(mesh, fine_lev, coarse_lev):
    return np.array([fine_lev if mesh.level(b) else coarse_lev for b in range(mesh.nblocks)], dtype=np.int32)


def _mixed_levels(mesh):
    """LAT levels (level = Lmax - exponent, Lmax = 2) obeying both rules: fine
    blocks on LAT level 2 (factor 1); coarse blocks touching a fine one on 1
    (factor 2); other coarse blocks on 1 or 0 by x position, so same-level
    mixed-factor faces exist too."""
    nb = mesh.nblocks
    lev = np.zeros(nb, dtype=np.int32)
    fine = [b for b in range(nb) if mesh.level(b)]
    for b in fine:
        lev[b] = 2
    for b in range(nb):
        if mesh.level(b) == 0:
            near = any(_adjacent(mesh, b, c) for c in fine)
            lev[b] = 1 if near or mesh.blk[b, 1] // N == 0 else 0
    for b in range(nb):
        for c in range(nb):
            if _adjacent(mesh, b, c):
                eb, ec = 2 - lev[b], 2 - lev[c]
                if mesh.level(b) == mesh.level(c):
                    assert abs(eb - ec) <= 1
                elif mesh.level(b) == 1:
                    assert eb <= ec <= eb + 1
    return lev


@pytest.mark.parametrize("ghost_dense", [0, 1])
def test_uniform_flow_stays_uniform_across_levels(orc, ghost_dense):
    mesh = _mesh([(1, 1, 1), (2, 1, 1)], bc=(0, 0, 0))
    cfg = W.Config(dual=1, ghost_dense=ghost_dense)
    U = W.uniform_state(mesh, cfg)
    lev = _mixed_levels(mesh)
    U2, nupd = orc.lat_window(cfg, mesh, U, lev, 1e-3)
    assert nupd == sum(1 << int(l) for l in lev)
    assert np.array_equal(U, U2)


def _totals(mesh, nv, U):
    """Volume integrals of rho, m and E of a state with nv variables per cell."""
    t = []
    for v in range(5):
        t.append(math.fsum(float(W.block_volume(mesh, b)) * float(x)
                           for b in range(mesh.nblocks) for x in W.unpack_block(mesh, nv, U, b)[v].ravel()))
    return np.array(t)


@pytest.mark.parametrize("sync", [False, True])
@pytest.mark.parametrize("ghost_dense", [0, 1])
def test_coarse_fine_reflux_conserves(orc, sync, ghost_dense):
    """Periodic box with refined regions (one touching another across a
    periodic edge): the coarse side's flux correction makes the volume
    integrals of rho, m and E exact to rounding (eq lat-flux-impulse applied at
    coarse-fine faces), synchronised or with mixed factors."""
    mesh = _mesh([(0, 1, 1), (3, 1, 1), (1, 2, 2)], bc=(0, 0, 0))
    cfg = W.Config(dual=1, ghost_dense=ghost_dense)
    U = W.random_smooth_state(mesh, cfg, seed=9, amp=0.3)
    lev = np.zeros(mesh.nblocks, dtype=np.int32) if sync else _mixed_levels(mesh)
    dt0 = 2e-3 if sync else 1e-3
    t0 = _totals(mesh, cfg.nv, U)
    U2, _ = orc.lat_window(cfg, mesh, U, lev, dt0)
    t1 = _totals(mesh, cfg.nv, U2)
    scale = np.array([t0[0], t0[0], t0[0], t0[0], t0[4]])
    assert np.all(np.abs(t1 - t0) <= 1e-14 * scale), (t1 - t0) / scale
    assert not np.array_equal(U, U2)


@pytest.mark.parametrize("mixed", [False, True])
def test_uniform_gravity_across_levels(orc, mixed):
    """Uniform gas at rest in a uniform field (linear stored potential, whose
    ghost layer continues the linear function across the periodic seam): the
    exact solution stays uniform with v = g t.  Ghost states taken at the
    wrong history (a stage-1 state for a start state, a start state for a
    mid-step one) give density errors of order dt |g| dt / dx ~ 1e-5 here.
      * synchronised (every block one step of 4 dt0): restriction and
        prolongation of uniform histories are exact, so the run is uniform to
        rounding and v = g t;
      * fine blocks with factor 1 beside coarse blocks with factor 2: the
        fine stage-2 input is the Euler predictor, the coarse neighbour's
        dense output at the same time the exact state; their energies differ
        by rho |g|^2 dt_c^2 / 2 (dt_c = 2 dt0), which moves the density by
        about that pressure difference / (2 c) * dt0 / dx_fine ~ 6e-10."""
    mesh = _mesh([(1, 1, 1), (2, 1, 1)], bc=(0, 0, 0))
    g = np.array([0.3, -0.2, 0.1])
    cfg = W.Config(dual=0, grav_kind=1, ghost_dense=1)
    phi = W.pack_potential(mesh, lambda x, y, z: -(g[0] * x + g[1] * y + g[2] * z))
    U = W.pack_state(mesh, 5, lambda x, y, z: W.ideal_conserved(1.0 + 0 * x, 0 * x, 0 * x, 0 * x, 1.0 + 0 * x,
                                                                cfg.gamma, False))
    if mixed:
        lev, dt0, T = _levels_for(mesh, 1, 0), 1e-3, 2e-3
    else:
        lev, dt0, T = np.zeros(mesh.nblocks, np.int32), 4e-3, 4e-3
    U2, _ = orc.lat_window(cfg, mesh, U, lev, dt0, phi=phi)
    drho = max(np.abs(W.unpack_block(mesh, 5, U2, b)[0] - 1.0).max() for b in range(mesh.nblocks))
    dv = max(np.abs(W.unpack_block(mesh, 5, U2, b)[1 + d] - g[d] * T).max() / abs(g[d] * T)
             for b in range(mesh.nblocks) for d in range(3))
    if mixed:
        assert drho <= 5e-9 and dv <= 1e-4, (drho, dv)
    else:
        assert drho <= 1e-14 and dv <= 1e-12, (drho, dv)
