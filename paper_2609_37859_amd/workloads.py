"""Seeded, synthetic inputs shared by the GPU path and the oracle.

This module holds no part of the finite-volume method: it builds run
parameters, mesh descriptions, an equation-of-state table, potentials and
initial states.  Both the GPU library and the CPU oracle consume what it
returns; neither imports the other.

Workload shapes follow the paper: 32^3-zone MeshBlocks, the floor ratios and
dual-energy thresholds of Table 1, the H/He composition X=0.7, Y=0.3 of the
tabulated EOS (Sec. Tabulated EOS construction), the 1e3 Msun black hole and
the LAT level structure (Table 1, Sec. LAT method).  The paper's own EOS
tables, checkpoints and production data are not available; every state here
is synthetic.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# CODATA 2018 / IAU constants, cgs
K_B = 1.380649e-16
H_PLANCK = 6.62607015e-27
M_E = 9.1093837015e-28
M_U = 1.66053906660e-24
EV = 1.602176634e-12
G_NEWTON = 6.67430e-8
M_SUN = 1.98847e33
R_SUN = 6.957e10
CHI_H = 13.598434 * EV
CHI_HE1 = 24.587389 * EV
CHI_HE2 = 54.417765 * EV

# variable indices of the conserved state
IDN, IM1, IM2, IM3, IEN, IAX = range(6)


@dataclasses.dataclass
class Config:
    """Run parameters (mirrors the C-ABI configuration struct field by field)."""
    eos_kind: int = 0          # 0 ideal gas, 1 table
    dual: int = 0              # dual-energy on/off
    grav_kind: int = 0         # 0 none, 1 stored potential, 2 softened point mass
    n_lat: int = 0             # N_LAT
    gamma: float = 5.0 / 3.0
    eta1: float = 1e-3
    eta2: float = 1e-4
    cfl: float = 0.3
    rho_floor: float = 1e-10
    p_floor: float = 1e-12
    e_floor: float = 0.0       # specific-energy floor (table EOS)
    merge_frac: float = 0.0
    gm_bh: float = 0.0
    r_soft: float = 0.0
    r_exc: float = 0.0
    bh_x0: tuple = (0.0, 0.0, 0.0)
    v_frame: tuple = (0.0, 0.0, 0.0)
    riemann: int = 0           # 0 HLLC, 1 HLLE
    ghost_dense: int = 0       # LAT ghosts of a neighbour mid-step: 0 linear in time, 1 RK2 dense output

    @property
    def nv(self) -> int:
        return 6 if self.dual else 5


@dataclasses.dataclass
class Mesh:
    """Cubic blocks aligned to a lattice of the smallest block edge (in cells
    of refinement level 0).  A block on refinement level r has cell widths
    dx / 2^r and its origin counted in level-r cells; nx, ny, nz and dx are
    level 0's."""
    nx: int
    ny: int
    nz: int
    bc: tuple                  # per axis: 0 periodic, 1 outflow
    x0: tuple
    dx: tuple
    blk: np.ndarray            # int32 [nblocks, 4] = n, ox, oy, oz
    rlev: np.ndarray = None    # int32 [nblocks] refinement level (0 or 1); None: all on level 0

    @property
    def nblocks(self) -> int:
        return int(self.blk.shape[0])

    @property
    def refined(self) -> bool:
        return self.rlev is not None and bool(np.any(self.rlev != 0))

    def level(self, b: int) -> int:
        return 0 if self.rlev is None else int(self.rlev[b])

    def block_cells(self) -> np.ndarray:
        return self.blk[:, 0].astype(np.int64) ** 3

    def offsets(self, nv: int) -> np.ndarray:
        sizes = nv * self.block_cells()
        return np.concatenate([[0], np.cumsum(sizes)])

    @property
    def ncells(self) -> int:
        return int(self.block_cells().sum())


@dataclasses.dataclass
class EosTable:
    nrho: int
    nT: int
    lr0: float
    dlr: float
    lT0: float
    dlT: float
    lP: np.ndarray             # [nrho, nT] log10 P
    le: np.ndarray             # [nrho, nT] log10 e (specific internal energy)
    lc2: np.ndarray            # [nrho, nT] log10 c_s^2
    e_floor: float             # smallest specific energy every row reaches (T = T_min)


# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------
def uniform_mesh(nbx, nby, nbz, n, dx, x0=(0.0, 0.0, 0.0), bc=(0, 0, 0)) -> Mesh:
    blk = []
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                blk.append((n, bx * n, by * n, bz * n))
    if np.isscalar(dx):
        dx = (dx, dx, dx)
    return Mesh(nbx * n, nby * n, nbz * n, tuple(bc), tuple(map(float, x0)), tuple(map(float, dx)),
                np.asarray(blk, dtype=np.int32))


def mixed_mesh(regions, rn, split, dx, x0=(0.0, 0.0, 0.0), bc=(1, 1, 1)) -> Mesh:
    """Regions of rn^3 cells on a (rx, ry, rz) grid; regions flagged in ``split``
    (bool array [rz, ry, rx]) become eight (rn/2)^3 blocks."""
    rx, ry, rz = regions
    h = rn // 2
    blk = []
    for cz in range(rz):
        for cy in range(ry):
            for cx in range(rx):
                ox, oy, oz = cx * rn, cy * rn, cz * rn
                if split[cz, cy, cx]:
                    for sz in range(2):
                        for sy in range(2):
                            for sx in range(2):
                                blk.append((h, ox + sx * h, oy + sy * h, oz + sz * h))
                else:
                    blk.append((rn, ox, oy, oz))
    if np.isscalar(dx):
        dx = (dx, dx, dx)
    return Mesh(rx * rn, ry * rn, rz * rn, tuple(bc), tuple(map(float, x0)), tuple(map(float, dx)),
                np.asarray(blk, dtype=np.int32))


def amr_mesh(nb, n, dx, refine, x0=(0.0, 0.0, 0.0), bc=(0, 0, 0)) -> Mesh:
    """Two refinement levels.  Level 0 is a (nbx, nby, nbz) grid of regions of
    n^3 cells of width dx; a region flagged in ``refine`` (bool array
    [nbz, nby, nbx]) is covered instead by eight level-1 blocks of n^3 cells
    of width dx/2.  Every block holds n^3 cells; blocks are listed region by
    region (x fastest), a refined region's eight in x-fastest order."""
    nbx, nby, nbz = nb
    blk, lev = [], []
    for cz in range(nbz):
        for cy in range(nby):
            for cx in range(nbx):
                if refine[cz, cy, cx]:
                    for sz in range(2):
                        for sy in range(2):
                            for sx in range(2):
                                blk.append((n, 2 * cx * n + sx * n, 2 * cy * n + sy * n, 2 * cz * n + sz * n))
                                lev.append(1)
                else:
                    blk.append((n, cx * n, cy * n, cz * n))
                    lev.append(0)
    if np.isscalar(dx):
        dx = (dx, dx, dx)
    return Mesh(nbx * n, nby * n, nbz * n, tuple(bc), tuple(map(float, x0)), tuple(map(float, dx)),
                np.asarray(blk, dtype=np.int32), np.asarray(lev, dtype=np.int32))


def block_volume(mesh: Mesh, b: int) -> float:
    """Cell volume of block b."""
    return float(np.prod([np.ldexp(d, -mesh.level(b)) for d in mesh.dx]))


def cell_centres(mesh: Mesh, b: int, ghost: int = 0):
    """Cell-centre coordinates of block b (optionally with ghost layers), as
    3-D arrays indexed [k, j, i]."""
    n, ox, oy, oz = (int(v) for v in mesh.blk[b])
    r = np.arange(-ghost, n + ghost, dtype=np.float64)
    h = [np.ldexp(d, -mesh.level(b)) for d in mesh.dx]
    xs = mesh.x0[0] + (ox + r + 0.5) * h[0]
    ys = mesh.x0[1] + (oy + r + 0.5) * h[1]
    zs = mesh.x0[2] + (oz + r + 0.5) * h[2]
    z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")
    return x, y, z


def pack_state(mesh: Mesh, nv: int, fn) -> np.ndarray:
    """Concatenate blocks; fn(x, y, z) returns a list of nv conserved arrays."""
    out = []
    for b in range(mesh.nblocks):
        x, y, z = cell_centres(mesh, b)
        q = fn(x, y, z)
        out.append(np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), x.shape) for v in q[:nv]]).ravel())
    return np.ascontiguousarray(np.concatenate(out))


def unpack_block(mesh: Mesh, nv: int, U: np.ndarray, b: int) -> np.ndarray:
    off = mesh.offsets(nv)
    n = int(mesh.blk[b, 0])
    return U[off[b]:off[b + 1]].reshape(nv, n, n, n)


def to_global(mesh: Mesh, nv: int, U: np.ndarray) -> np.ndarray:
    """Assemble the block-ordered state of a single-level mesh into a
    [nv, nz, ny, nx] array."""
    if mesh.refined:
        raise ValueError("to_global needs a single-level mesh")
    g = np.empty((nv, mesh.nz, mesh.ny, mesh.nx))
    for b in range(mesh.nblocks):
        n, ox, oy, oz = (int(v) for v in mesh.blk[b])
        g[:, oz:oz + n, oy:oy + n, ox:ox + n] = unpack_block(mesh, nv, U, b)
    return g


def pack_potential(mesh: Mesh, fn) -> np.ndarray:
    """Cell-centred potential per block with one ghost layer, [(n+2)^3] each."""
    out = []
    for b in range(mesh.nblocks):
        x, y, z = cell_centres(mesh, b, ghost=1)
        out.append(np.asarray(fn(x, y, z), dtype=np.float64).ravel())
    return np.ascontiguousarray(np.concatenate(out))


def ideal_conserved(rho, vx, vy, vz, P, gamma, with_aux):
    U = P / (gamma - 1.0)
    E = U + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    q = [rho, rho * vx, rho * vy, rho * vz, E]
    if with_aux:
        q.append(U)
    return q


# ---------------------------------------------------------------------------
# Saha hydrogen-helium equation of state (data generator for the EOS table)
# ---------------------------------------------------------------------------
def _saha_core(rho, T, X=0.7, Y=0.3):
    rho = np.asarray(rho, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    rho, T = np.broadcast_arrays(rho, T)
    nH = X * rho / M_U
    nHe = Y * rho / (4.0 * M_U)
    kT = K_B * T
    lnLam = 1.5 * np.log(2.0 * math.pi * M_E * kT / H_PLANCK ** 2)
    lnSH = lnLam - CHI_H / kT
    lnS1 = lnLam + math.log(4.0) - CHI_HE1 / kT
    lnS2 = lnLam - CHI_HE2 / kT

    def fractions(lne):
        xH = 1.0 / (1.0 + np.exp(lne - lnSH))
        la = lnS1 - lne
        lb = lnS2 - lne
        # He fractions y0:y1:y2 = 1 : a : a b, normalised in log space
        m = np.maximum(np.maximum(0.0, la), la + lb)
        d = np.exp(-m) + np.exp(la - m) + np.exp(la + lb - m)
        y1 = np.exp(la - m) / d
        y2 = np.exp(la + lb - m) / d
        return xH, y1, y2

    lo = np.full(rho.shape, math.log(1e-60))
    hi = np.log(nH + 2.0 * nHe) + 1e-12
    for _ in range(64):  # the bracket spans < 200 in ln n_e: 64 halvings reach ~1e-17
        mid = 0.5 * (lo + hi)
        xH, y1, y2 = fractions(mid)
        f = nH * xH + nHe * (y1 + 2.0 * y2) - np.exp(mid)
        pos = f > 0.0
        lo = np.where(pos, mid, lo)
        hi = np.where(pos, hi, mid)
    lne = 0.5 * (lo + hi)
    xH, y1, y2 = fractions(lne)
    ne = np.exp(lne)
    ntot = nH + nHe + ne
    P = ntot * kT
    e = (1.5 * ntot * kT + nH * xH * CHI_H + nHe * (y1 * CHI_HE1 + y2 * (CHI_HE1 + CHI_HE2))) / rho
    return P, e, xH, y1, y2, ne


def saha_pe(rho, T):
    """Pressure and specific internal energy (zero point: neutral atoms)."""
    P, e, *_ = _saha_core(rho, T)
    return P, e


def saha_gamma1(rho, T, h=1e-3):
    """First adiabatic exponent by the identity Gamma1 = chi_rho + chi_T^2 P / (rho T c_V),
    with the logarithmic derivatives taken by 5-point central differences."""
    rho = np.asarray(rho, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    lr, lt = np.log(rho), np.log(T)
    w = np.array([1.0, -8.0, 8.0, -1.0]) / (12.0 * h)
    st = np.array([-2.0, -1.0, 1.0, 2.0]) * h
    lnP_r = sum(wi * np.log(saha_pe(np.exp(lr + s), T)[0]) for wi, s in zip(w, st))
    lnP_t = sum(wi * np.log(saha_pe(rho, np.exp(lt + s))[0]) for wi, s in zip(w, st))
    de_dlnT = sum(wi * saha_pe(rho, np.exp(lt + s))[1] for wi, s in zip(w, st))
    P, e = saha_pe(rho, T)
    cV = de_dlnT / T
    return lnP_r + lnP_t ** 2 * P / (rho * T * cV)


def saha_table(nrho=256, nT=256, lr=(-12.0, 2.0), lt=(3.0, 8.0)) -> EosTable:
    """256x256 node table in (log10 rho, log10 T) of log10 P, log10 e, log10 c_s^2
    for Saha ionisation of H and He (X=0.7, Y=0.3) with recombination energy."""
    lrs = np.linspace(lr[0], lr[1], nrho)
    lts = np.linspace(lt[0], lt[1], nT)
    LR, LT = np.meshgrid(lrs, lts, indexing="ij")
    rho, T = 10.0 ** LR, 10.0 ** LT
    P, e = saha_pe(rho, T)
    g1 = saha_gamma1(rho, T)
    cs2 = g1 * P / rho
    le = np.log10(e)
    if not np.all(np.diff(le, axis=1) > 0):
        raise RuntimeError("log e is not increasing in T on every density row")
    return EosTable(nrho, nT, lr[0], (lr[1] - lr[0]) / (nrho - 1), lt[0], (lt[1] - lt[0]) / (nT - 1),
                    np.ascontiguousarray(np.log10(P)), np.ascontiguousarray(le),
                    np.ascontiguousarray(np.log10(cs2)), float(np.max(e[:, 0])))


def ideal_table(gamma=5.0 / 3.0, mu=0.6, nrho=64, nT=64, lr=(-12.0, 2.0), lt=(3.0, 8.0)) -> EosTable:
    """Ideal gas written as a table: every field is linear in (log rho, log T),
    so bilinear interpolation reproduces it exactly."""
    lrs = np.linspace(lr[0], lr[1], nrho)
    lts = np.linspace(lt[0], lt[1], nT)
    LR, LT = np.meshgrid(lrs, lts, indexing="ij")
    a = K_B / (mu * M_U)
    lP = LR + LT + math.log10(a)
    le = LT + math.log10(a / (gamma - 1.0)) + 0.0 * LR
    lc2 = LT + math.log10(gamma * a) + 0.0 * LR
    return EosTable(nrho, nT, lr[0], (lr[1] - lr[0]) / (nrho - 1), lt[0], (lt[1] - lt[0]) / (nT - 1),
                    np.ascontiguousarray(lP), np.ascontiguousarray(le), np.ascontiguousarray(lc2),
                    float(10.0 ** le[:, 0].max()))


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def entropy_wave_c1(n=32):
    """One periodic 32^3 block on [0,1]^3, ideal gas gamma=5/3:
    rho = 1 + 0.1 sin(2 pi x), v = (1, 0.5, 0.25), P = 1."""
    cfg = Config(eos_kind=0, dual=0, gamma=5.0 / 3.0, cfl=0.3, rho_floor=1e-10, p_floor=1e-12)
    mesh = uniform_mesh(1, 1, 1, n, 1.0 / n)

    def fn(x, y, z):
        rho = 1.0 + 0.1 * np.sin(2.0 * math.pi * x)
        return ideal_conserved(rho, 1.0, 0.5, 0.25, 1.0 + 0.0 * x, cfg.gamma, False)

    return cfg, mesh, pack_state(mesh, cfg.nv, fn)


def stream_c2(table: EosTable, nb=4, n=32, dx=1e10, mach=1e7):
    """Cold Gaussian stream along x through the box centre: rho = 1e-12 + 1e-3
    exp(-r_perp^2 / 2 sigma^2), sigma = 8 cells, T = 1e4 K everywhere, uniform
    velocity of Mach 1e7 (w.r.t. the peak) along (1, 0.5, 0.25); periodic."""
    cfg = Config(eos_kind=1, dual=1, gamma=5.0 / 3.0, cfl=0.3, eta1=1e-3, eta2=1e-4,
                 rho_floor=1e-12, p_floor=0.0, e_floor=table.e_floor)
    mesh = uniform_mesh(nb, nb, nb, n, dx)
    L = nb * n * dx
    sig = 8.0 * dx
    d = np.array([1.0, 0.5, 0.25])
    d /= np.linalg.norm(d)
    cs_pk = math.sqrt(float(saha_gamma1(1e-3, 1e4)) * float(saha_pe(1e-3, 1e4)[0]) / 1e-3)
    v = mach * cs_pk * d

    def fn(x, y, z):
        r2 = (y - 0.5 * L) ** 2 + (z - 0.5 * L) ** 2
        rho = 1e-12 + 1e-3 * np.exp(-r2 / (2.0 * sig * sig))
        _, e = saha_pe(rho, 1e4)
        U = rho * e
        E = U + 0.5 * rho * float(v @ v)
        return [rho, rho * v[0], rho * v[1], rho * v[2], E, U]

    return cfg, mesh, pack_state(mesh, cfg.nv, fn)


def lane_emden(n=1.5, dxi=1e-4):
    """Lane-Emden solution theta(xi) by classical RK4 from the series start;
    returns (xi grid, theta, xi1, -xi1^2 theta'(xi1))."""
    xi = dxi
    th = 1.0 - xi * xi / 6.0 + n * xi ** 4 / 120.0
    dth = -xi / 3.0 + n * xi ** 3 / 30.0
    xs, ts = [0.0, xi], [1.0, th]

    def f(x, y):
        t, dt = y
        return np.array([dt, -(max(t, 0.0) ** n) - 2.0 * dt / x])

    y = np.array([th, dth])
    while y[0] > 0.0:
        k1 = f(xi, y)
        k2 = f(xi + 0.5 * dxi, y + 0.5 * dxi * k1)
        k3 = f(xi + 0.5 * dxi, y + 0.5 * dxi * k2)
        k4 = f(xi + dxi, y + dxi * k3)
        yn = y + dxi / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        if yn[0] <= 0.0:
            frac = y[0] / (y[0] - yn[0])
            xi1 = xi + frac * dxi
            dth1 = y[1] + frac * (yn[1] - y[1])
            xs.append(xi1)
            ts.append(0.0)
            return np.array(xs), np.array(ts), xi1, -xi1 * xi1 * dth1
        xi += dxi
        y = yn
        xs.append(xi)
        ts.append(y[0])
    raise RuntimeError("unreachable")


def polytrope_c3(nb=8, n=32, mass=M_SUN, radius=R_SUN, npoly=1.5):
    """n=1.5 Lane-Emden star (1 Msun, 1 Rsun) at rest in a 1e-10 rho_c / 1e-12 P_c
    atmosphere, under its own fixed potential; [-2 Rsun, 2 Rsun]^3, outflow."""
    xi, th, xi1, om = lane_emden(npoly)
    a = radius / xi1
    rho_c = mass / (4.0 * math.pi * a ** 3 * om)
    K = 4.0 * math.pi * G_NEWTON * a * a * rho_c ** (1.0 - 1.0 / npoly) / (npoly + 1.0)
    P_c = K * rho_c ** (1.0 + 1.0 / npoly)
    L = 4.0 * radius
    dx = L / (nb * n)
    cfg = Config(eos_kind=0, dual=0, gamma=5.0 / 3.0, cfl=0.3, grav_kind=1, n_lat=3,
                 rho_floor=1e-12 * rho_c, p_floor=1e-14 * P_c)
    mesh = uniform_mesh(nb, nb, nb, n, dx, x0=(-2 * radius,) * 3, bc=(1, 1, 1))
    rho_atm, P_atm = 1e-10 * rho_c, 1e-12 * P_c

    def theta(r):
        return np.interp(r / a, xi, th, right=0.0)

    def phi(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        inside = -G_NEWTON * mass / radius - (npoly + 1.0) * K * rho_c ** (1.0 / npoly) * theta(r)
        return np.where(r < radius, inside, -G_NEWTON * mass / np.maximum(r, 1e-30))

    def fn(x, y, z):
        r = np.sqrt(x * x + y * y + z * z)
        t = theta(r)
        rho = np.maximum(rho_c * t ** npoly, rho_atm)
        P = np.maximum(K * rho_c ** (1.0 + 1.0 / npoly) * t ** (npoly + 1.0), P_atm)
        return ideal_conserved(rho, 0.0 * x, 0.0 * x, 0.0 * x, P, cfg.gamma, False)

    info = dict(rho_c=rho_c, P_c=P_c, K=K, a=a, xi1=xi1, omega=om)
    return cfg, mesh, pack_state(mesh, cfg.nv, fn), pack_potential(mesh, phi), info


def polytrope_c3_saha(table: EosTable, nb=8, n=32, mass=M_SUN, radius=R_SUN, npoly=1.5):
    """The polytrope of polytrope_c3 (same mesh, density, pressure and fixed
    potential) with the Saha H/He EOS: at every radius the temperature whose
    Saha pressure equals the polytrope's pressure (bisection in log T, clamped
    to the table's range), and the internal energy density rho e(rho, T) there;
    cells take the values of their centre's radius.  Dual energy off."""
    cfg0, mesh, _, phi, info = polytrope_c3(nb, n, mass, radius, npoly)
    xi, th, xi1, om = lane_emden(npoly)
    a = info["a"]
    rho_c, P_c, K = info["rho_c"], info["P_c"], info["K"]
    r = np.linspace(0.0, 2.0 * math.sqrt(3.0) * radius, 8193)
    t = np.interp(r / a, xi, th, right=0.0)
    rho = np.maximum(rho_c * t ** npoly, 1e-10 * rho_c)
    P = np.maximum(K * rho_c ** (1.0 + 1.0 / npoly) * t ** (npoly + 1.0), 1e-12 * P_c)
    lo = np.full(r.shape, table.lT0)
    hi = np.full(r.shape, table.lT0 + (table.nT - 1) * table.dlT)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        p_mid, _ = saha_pe(rho, 10.0 ** mid)
        up = p_mid < P
        lo = np.where(up, mid, lo)
        hi = np.where(up, hi, mid)
    _, e = saha_pe(rho, 10.0 ** (0.5 * (lo + hi)))
    U_r = rho * e
    cfg = dataclasses.replace(cfg0, eos_kind=1, e_floor=table.e_floor, p_floor=0.0)

    def fn(x, y, z):
        rr = np.sqrt(x * x + y * y + z * z)
        d = np.interp(rr, r, rho)
        return [d, 0.0 * x, 0.0 * x, 0.0 * x, np.interp(rr, r, U_r)]

    return cfg, mesh, pack_state(mesh, cfg.nv, fn), phi, info


def high_mach_wave(ncell=64, nt=4, v_adv=1e8, amp=0.1, dual=1):
    """Periodic entropy wave with rho_bar = P = 1 advected at V = 1e8 along x
    (gamma = 5/3, Mach ~7.75e7); blocks of nt^3 cells, uniform in y and z."""
    cfg = Config(eos_kind=0, dual=dual, gamma=5.0 / 3.0, cfl=0.3, eta1=1e-3, eta2=1e-4,
                 rho_floor=1e-10, p_floor=1e-20)
    mesh = uniform_mesh(ncell // nt, 1, 1, nt, 1.0 / ncell)

    def fn(x, y, z):
        rho = 1.0 + amp * np.sin(2.0 * math.pi * x)
        return ideal_conserved(rho, v_adv + 0.0 * x, 0.0 * x, 0.0 * x, 1.0 + 0.0 * x, cfg.gamma, bool(dual))

    return cfg, mesh, pack_state(mesh, cfg.nv, fn)


def jeans_wave(nx=64, nt=8, n=8, a=1e-3, lam_ratio=0.8):
    """Linear Jeans wave along x (Sec. Self-gravity validation, eqs jeans-initial,
    jeans-analytic), adiabatic: rho = 1 + a cos(kx), P = 1/gamma + c^2 a cos(kx)
    with c = 1, at rest, wavelength = the box (k = 2 pi), on a periodic
    nx x nt x nt grid of n^3 blocks; 4 pi G = (lam_ratio k c)^2 puts the mode at
    lambda / lambda_J = lam_ratio.  Returns (cfg, mesh, U, zero potential,
    four_pi_G)."""
    cfg = Config(grav_kind=1, gamma=5.0 / 3.0, cfl=0.3, rho_floor=1e-10, p_floor=1e-12)
    mesh = uniform_mesh(nx // n, nt // n, nt // n, n, 1.0 / nx)
    k = 2 * np.pi
    U = pack_state(mesh, 5, lambda x, y, z: ideal_conserved(1 + a * np.cos(k * x), 0 * x, 0 * x, 0 * x,
                                                          1 / cfg.gamma + a * np.cos(k * x), cfg.gamma, False))
    phi0 = pack_potential(mesh, lambda x, y, z: 0 * x)
    return cfg, mesh, U, phi0, (lam_ratio * k) ** 2


def sound_wave(ncell, nt=4, amp=1e-6, gamma=5.0 / 3.0):
    """Linear sound wave along x: rho = 1 + a sin, v = c a sin, P = 1/gamma + c^2 a sin (c = 1)."""
    cfg = Config(eos_kind=0, dual=0, gamma=gamma, cfl=0.3, rho_floor=1e-10, p_floor=1e-20)
    mesh = uniform_mesh(ncell // nt, 1, 1, nt, 1.0 / ncell)
    P0 = 1.0 / gamma

    def fn(x, y, z):
        s = amp * np.sin(2.0 * math.pi * x)
        return ideal_conserved(1.0 + s, s, 0.0 * x, 0.0 * x, P0 + s, gamma, False)

    return cfg, mesh, pack_state(mesh, cfg.nv, fn)


def sod_mirrored(ncell=256, nt=4, gamma=1.4):
    """Sod shock tube along x, mirrored so the domain is periodic: left state
    (rho, v, P) = (1, 0, 1) for 0.25 <= x < 0.75, right state (0.125, 0, 0.1)
    elsewhere; blocks of nt^3 cells, uniform in y and z."""
    cfg = Config(eos_kind=0, dual=0, gamma=gamma, cfl=0.3, rho_floor=1e-10, p_floor=1e-20)
    mesh = uniform_mesh(ncell // nt, 1, 1, nt, 1.0 / ncell)

    def fn(x, y, z):
        inner = (x >= 0.25) & (x < 0.75)
        rho = np.where(inner, 1.0, 0.125)
        P = np.where(inner, 1.0, 0.1)
        return ideal_conserved(rho, 0.0 * x, 0.0 * x, 0.0 * x, P, gamma, False)

    return cfg, mesh, pack_state(mesh, cfg.nv, fn)


def uniform_state(mesh: Mesh, cfg: Config, rho=1.3, v=(0.7, -0.2, 0.4), P=0.9):
    def fn(x, y, z):
        return ideal_conserved(rho + 0.0 * x, v[0], v[1], v[2], P + 0.0 * x, cfg.gamma, bool(cfg.dual))
    return pack_state(mesh, cfg.nv, fn)


def random_smooth_state(mesh: Mesh, cfg: Config, seed: int, amp=0.2, modes=3):
    """Smooth random periodic perturbation of a uniform ideal-gas state."""
    rng = np.random.default_rng(seed)
    L = (mesh.nx * mesh.dx[0], mesh.ny * mesh.dx[1], mesh.nz * mesh.dx[2])
    coef = rng.normal(size=(6, modes, 3))
    phase = rng.uniform(0, 2 * math.pi, size=(6, modes))

    def field(c, x, y, z):
        s = 0.0 * x
        for m in range(modes):
            k = 2 * math.pi * np.round(coef[c, m] * 1.5)
            s = s + np.sin(k[0] * x / L[0] + k[1] * y / L[1] + k[2] * z / L[2] + phase[c, m]) / modes
        return s

    def fn(x, y, z):
        rho = 1.0 + amp * field(0, x, y, z)
        vx, vy, vz = (0.5 * amp * field(c, x, y, z) for c in (1, 2, 3))
        P = 1.0 + amp * field(4, x, y, z)
        return ideal_conserved(rho, vx, vy, vz, P, cfg.gamma, bool(cfg.dual))

    return pack_state(mesh, cfg.nv, fn)


# ---------------------------------------------------------------------------
# learned EOS seed: training samples, initial parameters, normalisation
# ---------------------------------------------------------------------------
def amr_blast(nb=(4, 4, 4), n=8, refined=((1, 1, 1), (2, 1, 1), (1, 2, 1), (2, 2, 2)), seed=5, amp=0.2,
              hot=30.0, dual=1, n_lat=2, ghost_dense=0, riemann=0):
    """Two-level workload of the coarse-fine LAT: a periodic unit-length box
    (along x) of nb level-0 regions of n^3 cells, the listed regions (x, y, z
    region indices) refined into eight level-1 blocks of n^3 cells.  Ideal
    gas (gamma 5/3) with a smooth random perturbation of amplitude amp
    (random_smooth_state) and an over-pressured Gaussian (peak pressure
    1 + hot, width one level-0 region / 4) at the centre of the first refined
    region: its sound speed and the halved fine cells give the refined blocks
    the smallest CFL steps, so a LAT window mixes factors across refinement
    levels and on each level.  Returns (cfg, mesh, U)."""
    cfg = Config(dual=dual, gamma=5.0 / 3.0, cfl=0.3, n_lat=n_lat, rho_floor=1e-10, p_floor=1e-12,
                 ghost_dense=ghost_dense, riemann=riemann)
    ref = np.zeros(nb[::-1], dtype=bool)
    for cx, cy, cz in refined:
        ref[cz, cy, cx] = True
    dx = 1.0 / (nb[0] * n)
    mesh = amr_mesh(nb, n, dx, ref, bc=(0, 0, 0))
    base = random_smooth_state(mesh, dataclasses.replace(cfg, dual=0), seed=seed, amp=amp)
    cx, cy, cz = refined[0]
    c = [(cx + 0.5) * n * dx, (cy + 0.5) * n * dx, (cz + 0.5) * n * dx]
    w = 0.25 * n * dx
    out = []
    off = mesh.offsets(5)
    for b in range(mesh.nblocks):
        x, y, z = cell_centres(mesh, b)
        q = base[off[b]:off[b + 1]].reshape(5, *x.shape)
        rho = q[0]
        K = 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho
        P = (q[4] - K) * (cfg.gamma - 1.0)
        P = P + hot * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * w * w))
        U = P / (cfg.gamma - 1.0)
        blk = [q[0], q[1], q[2], q[3], U + K] + ([U] if dual else [])
        out.append(np.stack(blk).ravel())
    return cfg, mesh, np.ascontiguousarray(np.concatenate(out))


def seed_ranges(table: EosTable):
    """(log rho lo, hi, log e lo, hi, log T lo, hi) used to normalise to [-1, 1]."""
    return (table.lr0, table.lr0 + (table.nrho - 1) * table.dlr, float(table.le.min()), float(table.le.max()),
            table.lT0, table.lT0 + (table.nT - 1) * table.dlT)


def seed_training_samples(table: EosTable, n: int, seed: int) -> np.ndarray:
    """[n, 2] (log10 rho, log10 e): log rho uniform over the table, log e uniform
    between the table's values at its lowest and highest temperature for that
    density (the tighter of the two bracketing rows)."""
    rng = np.random.default_rng(seed)
    lr = rng.uniform(table.lr0, table.lr0 + (table.nrho - 1) * table.dlr, n)
    i = np.clip(np.floor((lr - table.lr0) / table.dlr).astype(np.int64), 0, table.nrho - 2)
    # bounds from the stored nodes of the two bracketing rows (inside both rows' range)
    le_lo = np.maximum(table.le[i, 0], table.le[i + 1, 0])
    le_hi = np.minimum(table.le[i, -1], table.le[i + 1, -1])
    u = rng.uniform(0.0, 1.0, n)
    le = le_lo + u * (le_hi - le_lo)
    return np.ascontiguousarray(np.stack([lr, le], 1))


def mlp_init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, fp32 [4417] in the library's order."""
    rng = np.random.default_rng(seed)
    p = np.zeros(4417, dtype=np.float64)
    p[0:128] = rng.normal(0.0, math.sqrt(2.0 / 2.0), 128)
    p[192:4288] = rng.normal(0.0, math.sqrt(2.0 / 64.0), 4096)
    p[4352:4416] = rng.normal(0.0, math.sqrt(1.0 / 64.0), 64)
    return p.astype(np.float32)


# Region box (x0, x1, y0, y1, z0, z1) of the production-shaped run's 13 x 17 x 9
# region grid that holds 512 blocks (112 x 32^3 + 400 x 16^3, 5.3 M cells): the
# full z extent, y from 4 to 13 (the stream axis at y = 8.5 and the black hole
# at y = 11 regions) and the two x regions about the centre.  Its timing sample
# for the CPU oracle and its parity case.
C5_SUBDOMAIN_512 = (5, 7, 4, 13, 0, 9)
# region box of the two-level run that holds coarse and refined regions across
# the stream's lower edge (14 level-0 + 80 level-1 blocks of 32^3, 3.1 M cells)
AMR_SUBDOMAIN = (4, 7, 5, 9, 2, 4)


def _debris_setup(table: EosTable, regions, rn, n_split, dxr, vfr, dv, rho_pk, T, stream_frac, sig_cells):
    """Region selection, run parameters and initial data of the debris-stream
    runs: (dx, flagged regions [rz, ry, rx], cfg, fn(x, y, z) -> conserved)."""
    dx = dxr * R_SUN
    rx, ry, rz = regions
    L = np.array([rx, ry, rz]) * rn * dx
    c = 0.5 * L
    bh0 = np.array([c[0], c[1] + 20.0 * R_SUN, c[2]])
    # flag the regions whose centres are nearest the stream axis or the BH path
    cz, cy, cx = np.meshgrid(np.arange(rz), np.arange(ry), np.arange(rx), indexing="ij")
    pc = np.stack([(cx + 0.5) * rn * dx, (cy + 0.5) * rn * dx, (cz + 0.5) * rn * dx], -1)
    d_axis = np.hypot(pc[..., 1] - c[1], pc[..., 2] - c[2]) + np.maximum(np.abs(pc[..., 0] - c[0]) - stream_frac * L[0], 0)
    d_bh = np.hypot(pc[..., 1] - bh0[1], pc[..., 2] - bh0[2])
    score = np.minimum(d_axis, d_bh) + 1e-6 * (cx + rx * (cy + ry * cz))  # deterministic ties
    order = np.argsort(score.ravel(), kind="stable")
    flag = np.zeros(rx * ry * rz, dtype=bool)
    flag[order[:n_split]] = True
    flag = flag.reshape(rz, ry, rx)
    cfg = Config(eos_kind=1, dual=1, grav_kind=2, n_lat=3, cfl=0.3, eta1=1e-3, eta2=1e-4,
                 rho_floor=1e-10 * rho_pk * 0.5, p_floor=0.0, e_floor=table.e_floor, merge_frac=0.0,
                 gm_bh=G_NEWTON * 1e3 * M_SUN, r_soft=0.1 * dx, r_exc=4.0 * dx, bh_x0=tuple(bh0),
                 v_frame=(vfr, 0.0, 0.0))
    # specific energy at T on a fine log-density grid (data for the initial state)
    lg = np.linspace(math.log10(cfg.rho_floor) - 0.1, math.log10(rho_pk) + 0.1, 4096)
    _, eg = saha_pe(10.0 ** lg, T)
    a_s = stream_frac * L[0]
    sig = sig_cells * dx

    def fn(x, y, z):
        q = ((x - c[0]) / a_s) ** 2 + ((y - c[1]) / sig) ** 2 + ((z - c[2]) / sig) ** 2
        theta = np.clip(1.0 - q, 0.0, 1.0)
        rho = np.maximum(rho_pk * theta ** 1.5, 1e-10 * rho_pk)
        e = 10.0 ** np.interp(np.log10(rho), lg, np.log10(eg))
        U = rho * e
        inside = theta > 0
        vx = np.where(inside, dv * (x - c[0]) / a_s, 0.0)
        return [rho, rho * vx, 0 * x, 0 * x, U + 0.5 * rho * vx * vx, U]

    return dx, flag, cfg, fn


def debris_stream_c5(table: EosTable, regions=(13, 17, 9), rn=32, n_split=301, dxr=0.25, vfr=1e8, dv=3e7,
                     rho_pk=1e-3, T=1e4, stream_frac=0.3, sig_cells=8.0, box=None):
    """Production-shaped run: 13 x 17 x 9 regions of 32^3 cells at dx = 0.25 Rsun;
    the 301 regions nearest the stream axis and the black-hole path are split
    into eight 16^3 blocks (1688 x 32^3 + 2408 x 16^3 = 4096 blocks, 65.2 M
    cells).  A tidally stretched n = 1.5 stream (ellipsoid with semi-axes
    0.3 L_x, 8 dx, 8 dx; rho = rho_pk theta^1.5, T = 1e4 K) with a linear
    velocity spread v_x = dV (x - x_c) / (0.3 L_x) lies in a 1e-10 rho_pk
    background at rest; a 1e3 Msun point mass starts 20 Rsun from the stream
    centre and moves at -V_fr along x (uniform frame velocity V_fr); excision
    radius 4 dx, softening 0.1 dx; outflow boundaries.

    box = (x0, x1, y0, y1, z0, z1) keeps only those regions of the region grid
    (the same cells, split decisions, coordinates and initial data as in the
    whole run), with outflow boundaries at the box faces."""
    dx, split, cfg, fn = _debris_setup(table, regions, rn, n_split, dxr, vfr, dv, rho_pk, T, stream_frac, sig_cells)
    if box is None:
        mesh = mixed_mesh(regions, rn, split, dx, bc=(1, 1, 1))
    else:
        x0, x1, y0, y1, z0, z1 = box
        mesh = mixed_mesh((x1 - x0, y1 - y0, z1 - z0), rn, split[z0:z1, y0:y1, x0:x1], dx,
                          x0=(x0 * rn * dx, y0 * rn * dx, z0 * rn * dx), bc=(1, 1, 1))
    return cfg, mesh, pack_state(mesh, cfg.nv, fn)


def debris_stream_amr(table: EosTable, regions=(13, 17, 9), rn=32, n_refine=301, dxr=0.25, vfr=1e8, dv=3e7,
                      rho_pk=1e-3, T=1e4, stream_frac=0.3, sig_cells=8.0, box=None):
    """The production-shaped run on two refinement levels: the 301 regions of
    debris_stream_c5 that it splits are refined instead, each into eight
    level-1 blocks of 32^3 cells at dx / 2 (1688 level-0 + 2408 level-1 blocks,
    all 32^3: 4096 blocks, 134.2 M cells); stream, point mass, frame,
    excision radius (4 level-0 cells) and boundaries as there.  box as there."""
    dx, ref, cfg, fn = _debris_setup(table, regions, rn, n_refine, dxr, vfr, dv, rho_pk, T, stream_frac, sig_cells)
    if box is None:
        mesh = amr_mesh(regions, rn, dx, ref, bc=(1, 1, 1))
    else:
        x0, x1, y0, y1, z0, z1 = box
        mesh = amr_mesh((x1 - x0, y1 - y0, z1 - z0), rn, dx, ref[z0:z1, y0:y1, x0:x1],
                        x0=(x0 * rn * dx, y0 * rn * dx, z0 * rn * dx), bc=(1, 1, 1))
    return cfg, mesh, pack_state(mesh, cfg.nv, fn)
