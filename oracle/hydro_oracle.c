/*
 * FP64 CPU oracle for the MeshBlock finite-volume update of
 * "An End-to-End Numerical Framework for Tidal Disruption Events with AthenaK".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark load this library.  The product path never does.
 *
 * It is deliberately plain: every RK stage copies each block into an explicit
 * ghost-padded array, converts to primitives, computes every face flux and
 * then updates every cell, in that order, in IEEE double precision with round
 * to nearest and no floating-point contraction (built with -ffp-contract=off).
 * It shares no code, header or table with the GPU library; the two meet only
 * in the input data (mesh description, state, EOS table, potential).
 *
 * What each part follows:
 *   - hydro scheme: RK2 + PLM + Riemann solver, floors        (Table 1)
 *   - conserved-to-primitive + dual-energy switch             (Sec. Dual-energy evolution,
 *                                                              eqs dual-econs, dual-primitive-switch)
 *   - aux-energy flux and face velocity                        (eqs dual-flux, dual-face-velocity)
 *   - compression source, ideal (analytic) and tabulated       (eqs dual-compression-continuous,
 *                                                              dual-divv, dual-tabulated-compression)
 *   - resynchronisation                                        (eq dual-sync)
 *   - gravity source, centred momentum / flux-form energy      (eqs lat-grav-momentum, lat-grav-energy)
 *   - softened point-mass potential and excision               (eq bh-softened-gravity)
 *   - tabulated EOS in (log rho, log T), inverted in energy    (Sec. Tabulated EOS construction,
 *                                                              eqs eos-table-range, eos-table-fields)
 *   - LAT base step, factors, windows, ghost time
 *     interpolation, reflux with gravity work                  (Sec. LAT method; eqs lat-base-dt,
 *                                                              lat-factor, lat-flux-impulse,
 *                                                              lat-mass-impulse-mismatch, lat-grav-reflux)
 *   - two refinement levels under LAT: the coarse-fine factor
 *     rule, ghost states restricted from finer histories,
 *     interpolated in time and prolonged into finer ghosts,
 *     and the coarse side's flux correction at coarse-fine
 *     faces                                                    (Sec. LAT method)
 * Prolongation is piecewise linear with minmod-limited slopes on the
 * conserved variables, restriction the mean of the 2x2x2 children: the
 * paper names the operations and their order, not the operators.
 * The Riemann solver is HLLC (Toro, Riemann Solvers and Numerical Methods for
 * Fluid Dynamics, 3rd ed., Sec. 10.4, with Davis wave-speed estimates) or, by
 * configuration, the HLLE solver of the paper's production runs (Table 1;
 * Toro Sec. 10.3 with the same wave-speed estimates); the PLM limiter is van
 * Leer's harmonic mean; RK2 is Heun's (SSP) method.
 *
 * State layout: blocks are cubic (edge n), stored one after another, each as
 * nv arrays of n^3 doubles with x fastest.  nv = 5 (rho, mx, my, mz, E) or 6
 * (plus the auxiliary internal energy density A when dual energy is on).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { IDN = 0, IM1 = 1, IM2 = 2, IM3 = 3, IEN = 4, IAX = 5 };

typedef struct {
  int eos_kind;   /* 0 ideal gas, 1 table */
  int dual;       /* dual-energy on (1) / off (0) */
  int grav_kind;  /* 0 none, 1 stored cell-centred potential, 2 softened point mass */
  int n_lat;      /* largest LAT exponent N_LAT */
  double gamma, eta1, eta2, cfl;
  double rho_floor, p_floor, e_floor; /* e_floor: specific-energy floor, table EOS */
  double merge_frac;
  double gm_bh, r_soft, r_exc;
  double bh_x0[3], v_frame[3];
  int riemann;     /* 0 HLLC, 1 HLLE */
  int ghost_dense; /* LAT ghosts of a neighbour mid-step: 0 linear in time, 1 RK2 dense output */
} orc_cfg;

typedef struct {
  int nx, ny, nz;  /* global cells of refinement level 0 */
  int bc[3];       /* 0 periodic, 1 outflow (zero gradient) */
  double x0[3], dx[3]; /* cell widths of refinement level 0 */
  int nblocks;
  const int *blk;  /* [nblocks][4] = n, ox, oy, oz (global cell origin at the block's level) */
  const int *rlev; /* [nblocks] refinement level of each block (0 or 1; NULL: all 0); level r has
                      cell widths dx / 2^r and global extents (nx, ny, nz) * 2^r */
} orc_mesh;

typedef struct {
  int nrho, nT;
  double lr0, dlr, lT0, dlT; /* log10 axes: node i at lr0 + i*dlr */
  const double *lP, *le, *lc2; /* [nrho][nT], T contiguous */
} orc_table;

/* ------------------------------------------------------------------ */
/* mesh bookkeeping                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
  const orc_cfg *cfg;
  const orc_mesh *m;
  const orc_table *tab;
  int nv;
  int lat, lx, ly, lz; /* lattice edge in level-0 cells, lattice cells per axis */
  int *lmap;     /* lattice cell -> block */
  int *rl;       /* refinement level of each block */
  int rmax;      /* largest refinement level */
  size_t *off;   /* state offset of each block (doubles) */
  size_t *poff;  /* potential offset of each block */
  size_t *ioff;  /* impulse offset of each block */
  size_t total, ptotal, itotal;
} mesh_t;

static void mesh_free(mesh_t *M) {
  free(M->lmap); free(M->rl); free(M->off); free(M->poff); free(M->ioff);
  memset(M, 0, sizeof *M);
}

/* cell width along d of refinement level r (exact: a power-of-two scaling) */
static double dx_r(const orc_mesh *m, int r, int d) { return ldexp(m->dx[d], -r); }

static int mesh_build(mesh_t *M, const orc_cfg *cfg, const orc_mesh *m, const orc_table *tab) {
  memset(M, 0, sizeof *M);
  M->cfg = cfg; M->m = m; M->tab = tab;
  M->nv = cfg->dual ? 6 : 5;
  if (m->nblocks <= 0) return -1;
  M->rl = malloc(m->nblocks * sizeof(int));
  /* lattice edge: the smallest block extent in level-0 cells */
  int lat = 1 << 30;
  for (int b = 0; b < m->nblocks; b++) {
    int r = m->rlev ? m->rlev[b] : 0;
    int n = m->blk[4 * b];
    if (r < 0 || r > 1 || n % (1 << r)) { free(M->rl); M->rl = NULL; return -1; }
    M->rl[b] = r;
    if (r > M->rmax) M->rmax = r;
    if ((n >> r) < lat) lat = n >> r;
  }
  if (lat < 2 || m->nx % lat || m->ny % lat || m->nz % lat) { mesh_free(M); return -1; }
  M->lat = lat; M->lx = m->nx / lat; M->ly = m->ny / lat; M->lz = m->nz / lat;
  size_t nl = (size_t)M->lx * M->ly * M->lz;
  M->lmap = malloc(nl * sizeof(int));
  M->off = malloc((m->nblocks + 1) * sizeof(size_t));
  M->poff = malloc((m->nblocks + 1) * sizeof(size_t));
  M->ioff = malloc((m->nblocks + 1) * sizeof(size_t));
  for (size_t i = 0; i < nl; i++) M->lmap[i] = -1;
  size_t o = 0, po = 0, io = 0;
  for (int b = 0; b < m->nblocks; b++) {
    int r = M->rl[b];
    int n = m->blk[4 * b], ox = m->blk[4 * b + 1], oy = m->blk[4 * b + 2], oz = m->blk[4 * b + 3];
    int L = lat << r; /* lattice edge in this block's cells */
    if (n % L || ox % L || oy % L || oz % L) { mesh_free(M); return -1; }
    if (ox < 0 || oy < 0 || oz < 0 || ox + n > (m->nx << r) || oy + n > (m->ny << r) || oz + n > (m->nz << r)) {
      mesh_free(M); return -1;
    }
    for (int c = oz / L; c < (oz + n) / L; c++)
      for (int bb = oy / L; bb < (oy + n) / L; bb++)
        for (int a = ox / L; a < (ox + n) / L; a++) {
          size_t li = ((size_t)c * M->ly + bb) * M->lx + a;
          if (M->lmap[li] != -1) { mesh_free(M); return -1; }
          M->lmap[li] = b;
        }
    M->off[b] = o; o += (size_t)M->nv * n * n * n;
    M->poff[b] = po; po += (size_t)(n + 2) * (n + 2) * (n + 2);
    M->ioff[b] = io; io += (size_t)6 * M->nv * n * n;
  }
  for (size_t i = 0; i < nl; i++) if (M->lmap[i] < 0) { mesh_free(M); return -1; }
  M->off[m->nblocks] = o; M->poff[m->nblocks] = po; M->ioff[m->nblocks] = io;
  M->total = o; M->ptotal = po; M->itotal = io;
  return 0;
}

/* Apply the domain boundary to a global cell index; returns 0 when the index
 * lies outside an outflow edge (then it is clamped onto the edge cell). */
static int wrap_axis(int g, int N, int bc) {
  if (bc == 0) { g %= N; if (g < 0) g += N; return g; }
  if (g < 0) return 0;
  if (g >= N) return N - 1;
  return g;
}

/* Block covering global cell (gx, gy, gz) of refinement level r (indices
 * already inside the level's extents); its level may differ from r. */
static int covering_block(const mesh_t *M, int r, int gx, int gy, int gz) {
  int L = M->lat << r;
  return M->lmap[((size_t)(gz / L) * M->ly + gy / L) * M->lx + gx / L];
}

/* global cell of level r -> owning block and local index, for a cell whose
 * covering block is on level r (every cell of a single-level mesh) */
static void locate_r(const mesh_t *M, int r, int gx, int gy, int gz, int *b, int *i, int *j, int *k) {
  const orc_mesh *m = M->m;
  gx = wrap_axis(gx, m->nx << r, m->bc[0]);
  gy = wrap_axis(gy, m->ny << r, m->bc[1]);
  gz = wrap_axis(gz, m->nz << r, m->bc[2]);
  int bb = covering_block(M, r, gx, gy, gz);
  *b = bb;
  *i = gx - m->blk[4 * bb + 1];
  *j = gy - m->blk[4 * bb + 2];
  *k = gz - m->blk[4 * bb + 3];
}

static void locate(const mesh_t *M, int gx, int gy, int gz, int *b, int *i, int *j, int *k) {
  locate_r(M, 0, gx, gy, gz, b, i, j, k);
}

/* whether the neighbour across a face is a real cell (not beyond an outflow edge) */
static int inside_axis(int g, int N, int bc) { return bc == 0 || (g >= 0 && g < N); }

/* ------------------------------------------------------------------ */
/* equation of state                                                   */
/* ------------------------------------------------------------------ */

/* internal-energy-density floor (Table 1 floors; table: rho * e_floor) */
static double u_floor(const orc_cfg *c, double rho) {
  if (c->eos_kind == 0) return c->p_floor / (c->gamma - 1.0);
  return rho * c->e_floor;
}

static void table_rho_cell(const orc_table *T, double lr, int *i, double *w) {
  double lrmax = T->lr0 + (T->nrho - 1) * T->dlr;
  if (lr < T->lr0) lr = T->lr0;
  if (lr > lrmax) lr = lrmax;
  double x = (lr - T->lr0) / T->dlr;
  int ii = (int)floor(x);
  if (ii > T->nrho - 2) ii = T->nrho - 2;
  if (ii < 0) ii = 0;
  *i = ii; *w = x - ii;
}

/* Alternative roundings, for the tests only (they measure how strongly a
 * workload amplifies rounding differences: the conditioning of a comparison).
 * Bit 0: the linear interpolation (1 - w) x + w y is taken as one fused
 * multiply-add w y + (1 - w) x instead of two rounded products and a rounded
 * sum.  Bit 1: the EOS's base-10 logarithms and powers are evaluated in long
 * double and rounded once to double instead of by the double-precision
 * library routines.  Each is an equally valid evaluation of the same formula,
 * one rounding apart; the default (0) is the plain definition. */
static int g_interp_fused = 0, g_math_long = 0;
void orc_set_interp_rounding(int mode) {
  g_interp_fused = mode & 1;
  g_math_long = (mode >> 1) & 1;
}
static double log10_e(double x) { return g_math_long ? (double)log10l((long double)x) : log10(x); }
static double pow10_e(double y) { return g_math_long ? (double)powl(10.0L, (long double)y) : pow(10.0, y); }

static double lerp(double w, double x, double y) {
  return g_interp_fused ? fma(w, y, (1.0 - w) * x) : (1.0 - w) * x + w * y;
}

/* value of a table field at density weight w between rows i, i+1, at T node j */
static double tcol(const double *F, int nT, int i, double w, int j) {
  return lerp(w, F[(size_t)i * nT + j], F[(size_t)(i + 1) * nT + j]);
}

/* Inversion e -> T at fixed density.  The answer is defined as the largest T
 * node j in [0, nT-2] whose interpolated log e does not exceed the target,
 * after the target is clamped into the column's range; this is found by
 * bisection.  Returns j and the in-cell weight wT. */
static void table_invert(const orc_table *T, int i, double w, double le, int *jout, double *wT) {
  int nT = T->nT;
  double lo_v = tcol(T->le, nT, i, w, 0), hi_v = tcol(T->le, nT, i, w, nT - 1);
  if (le < lo_v) le = lo_v;
  if (le > hi_v) le = hi_v;
  int lo = 0, hi = nT - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (tcol(T->le, nT, i, w, mid) <= le) lo = mid; else hi = mid;
  }
  double a = tcol(T->le, nT, i, w, lo), b = tcol(T->le, nT, i, w, lo + 1);
  *jout = lo;
  *wT = (le - a) / (b - a);
}

static double tbil(const double *F, int nT, int i, double w, int j, double wT) {
  return lerp(wT, tcol(F, nT, i, w, j), tcol(F, nT, i, w, j + 1));
}

/* (rho, U) -> pressure and adiabatic sound speed */
static void eos_pc(const orc_cfg *c, const orc_table *T, double rho, double U, double *P, double *cs) {
  if (c->eos_kind == 0) {
    double Ue = U;
    double uf = u_floor(c, rho);
    if (Ue < uf) Ue = uf;
    *P = (c->gamma - 1.0) * Ue;
    *cs = sqrt(c->gamma * (*P) / rho);
    return;
  }
  int i, j; double w, wT;
  double Ue = U;
  double uf = u_floor(c, rho);
  if (Ue < uf) Ue = uf; /* keeps the logarithm defined; the inversion clamps into the table */
  table_rho_cell(T, log10_e(rho), &i, &w);
  table_invert(T, i, w, log10_e(Ue / rho), &j, &wT);
  *P = pow10_e(tbil(T->lP, T->nT, i, w, j, wT));
  *cs = pow10_e(0.5 * tbil(T->lc2, T->nT, i, w, j, wT));
}

/* ------------------------------------------------------------------ */
/* cell primitives and the Riemann problem                             */
/* ------------------------------------------------------------------ */

/* conserved -> (rho, vx, vy, vz, U_EOS[, A]) with the dual-energy switch */
static void c2p(const orc_cfg *c, const double *q, double *w) {
  double rho = q[IDN];
  double vx = q[IM1] / rho, vy = q[IM2] / rho, vz = q[IM3] / rho;
  double K = 0.5 * (q[IM1] * q[IM1] + q[IM2] * q[IM2] + q[IM3] * q[IM3]) / rho;
  double Uc = q[IEN] - K;
  double Ueos = Uc;
  if (c->dual) {
    if (!(Uc > 0.0 && Uc > c->eta1 * q[IEN])) Ueos = q[IAX];
    w[5] = q[IAX];
  }
  w[0] = rho; w[1] = vx; w[2] = vy; w[3] = vz; w[4] = Ueos;
}

static double vanleer(double dm, double dp) {
  double p = dm * dp;
  return p > 0.0 ? 2.0 * p / (dm + dp) : 0.0;
}

/* HLLC flux for states rotated so that index 1 is the face normal.
 * wl, wr: (rho, un, ut1, ut2, U, [A]); returns flux (rho, mn, mt1, mt2, E).
 * Davis wave speeds; contact tie S_M = 0 takes the left star state. */
static void hllc(const double *wl, double pl, double cl, const double *wr, double pr, double cr, double *f) {
  double rl = wl[0], ul = wl[1], vl = wl[2], zl = wl[3];
  double rr = wr[0], ur = wr[1], vr = wr[2], zr = wr[3];
  double El = wl[4] + 0.5 * rl * (ul * ul + vl * vl + zl * zl);
  double Er = wr[4] + 0.5 * rr * (ur * ur + vr * vr + zr * zr);
  double sl = fmin(ul - cl, ur - cr);
  double sr = fmax(ul + cl, ur + cr);
  double fl[5] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, rl * ul * zl, (El + pl) * ul};
  double fr[5] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, rr * ur * zr, (Er + pr) * ur};
  if (sl >= 0.0) { memcpy(f, fl, sizeof fl); return; }
  if (sr <= 0.0) { memcpy(f, fr, sizeof fr); return; }
  double sm = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) / (rl * (sl - ul) - rr * (sr - ur));
  if (sm >= 0.0) {
    double a = rl * (sl - ul) / (sl - sm);
    double us[5] = {a, a * sm, a * vl, a * zl, a * (El / rl + (sm - ul) * (sm + pl / (rl * (sl - ul))))};
    double u0[5] = {rl, rl * ul, rl * vl, rl * zl, El};
    for (int v = 0; v < 5; v++) f[v] = fl[v] + sl * (us[v] - u0[v]);
  } else {
    double a = rr * (sr - ur) / (sr - sm);
    double us[5] = {a, a * sm, a * vr, a * zr, a * (Er / rr + (sm - ur) * (sm + pr / (rr * (sr - ur))))};
    double u0[5] = {rr, rr * ur, rr * vr, rr * zr, Er};
    for (int v = 0; v < 5; v++) f[v] = fr[v] + sr * (us[v] - u0[v]);
  }
}

/*
 * HLLE flux (Harten, Lax and van Leer; Einfeldt's positive wave-speed bounds,
 * here the same Davis estimates as the HLLC solver), Toro (2009) eq. 10.21:
 * F_L if S_L >= 0, F_R if S_R <= 0, else
 * (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L).
 * The paper's production runs use this solver (Table 1).
 */
static void hlle(const double *wl, double pl, double cl, const double *wr, double pr, double cr, double *f) {
  double rl = wl[0], ul = wl[1], vl = wl[2], zl = wl[3];
  double rr = wr[0], ur = wr[1], vr = wr[2], zr = wr[3];
  double El = wl[4] + 0.5 * rl * (ul * ul + vl * vl + zl * zl);
  double Er = wr[4] + 0.5 * rr * (ur * ur + vr * vr + zr * zr);
  double sl = fmin(ul - cl, ur - cr);
  double sr = fmax(ul + cl, ur + cr);
  double fl[5] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, rl * ul * zl, (El + pl) * ul};
  double fr[5] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, rr * ur * zr, (Er + pr) * ur};
  if (sl >= 0.0) { memcpy(f, fl, sizeof fl); return; }
  if (sr <= 0.0) { memcpy(f, fr, sizeof fr); return; }
  double ul5[5] = {rl, rl * ul, rl * vl, rl * zl, El};
  double ur5[5] = {rr, rr * ur, rr * vr, rr * zr, Er};
  for (int v = 0; v < 5; v++) f[v] = (sr * fl[v] - sl * fr[v] + sl * sr * (ur5[v] - ul5[v])) / (sr - sl);
}

/* ------------------------------------------------------------------ */
/* gravity and excision geometry                                       */
/* ------------------------------------------------------------------ */
/* centre of global cell g (level r) along d */
static double cell_x(const orc_mesh *m, int r, int d, int g) { return m->x0[d] + (g + 0.5) * dx_r(m, r, d); }

static double bh_pos(const orc_cfg *c, int d, double t) { return c->bh_x0[d] - c->v_frame[d] * t; }

/* softened point-mass potential at a cell centre (eq bh-softened-gravity) */
static double phi_point(const orc_cfg *c, const orc_mesh *m, int r, int gx, int gy, int gz, double t) {
  double dx = cell_x(m, r, 0, gx) - bh_pos(c, 0, t);
  double dy = cell_x(m, r, 1, gy) - bh_pos(c, 1, t);
  double dz = cell_x(m, r, 2, gz) - bh_pos(c, 2, t);
  return -c->gm_bh / sqrt(dx * dx + dy * dy + dz * dz + c->r_soft * c->r_soft);
}

static int excised(const orc_cfg *c, const orc_mesh *m, int r, int gx, int gy, int gz, double t) {
  if (c->grav_kind != 2 || !(c->r_exc > 0.0)) return 0;
  double dx = cell_x(m, r, 0, gx) - bh_pos(c, 0, t);
  double dy = cell_x(m, r, 1, gy) - bh_pos(c, 1, t);
  double dz = cell_x(m, r, 2, gz) - bh_pos(c, 2, t);
  return dx * dx + dy * dy + dz * dz < c->r_exc * c->r_exc;
}

/* potential at local cell (i,j,k) of block b, i,j,k in [-1, n] */
static double phi_at(const mesh_t *M, const double *phi, int b, int i, int j, int k, double t) {
  const orc_mesh *m = M->m;
  int n = m->blk[4 * b];
  if (M->cfg->grav_kind == 1) {
    int np = n + 2;
    return phi[M->poff[b] + ((size_t)(k + 1) * np + (j + 1)) * np + (i + 1)];
  }
  return phi_point(M->cfg, m, M->rl[b], m->blk[4 * b + 1] + i, m->blk[4 * b + 2] + j, m->blk[4 * b + 3] + k, t);
}

/* ------------------------------------------------------------------ */
/* one RK stage on one block                                           */
/* ------------------------------------------------------------------ */
#define PADX(n) ((n) + 4)
static inline size_t pidx(int n, int i, int j, int k) { /* i,j,k in [-2, n+2) */
  int np = n + 4;
  return ((size_t)(k + 2) * np + (j + 2)) * np + (i + 2);
}
static inline size_t cidx(int n, int i, int j, int k) { return ((size_t)k * n + j) * n + i; }
static inline size_t fidx(int n, int a, int b) { return (size_t)b * n + a; }

/*
 * Stage update of block b.
 *   qpad  : stage-input conserved state with 2 ghost layers, [nv][(n+4)^3]
 *   qbase : state at the start of the step (stage 2 only), [nv][n^3]
 *   stage : 1 -> out = q + dt L(q);  2 -> out = 1/2 qbase + 1/2 (q + dt L(q))
 *   t     : time at which the stage's right-hand side is evaluated
 *   bflux : boundary-face fluxes [6 faces][nv][n^2] (face = 2*dir + side)
 */
static void block_stage(const mesh_t *M, const double *phi, int b, const double *qpad, const double *qbase,
                        int stage, double dt, double t, double *out, double *bflux) {
  const orc_cfg *c = M->cfg;
  const orc_mesh *m = M->m;
  const orc_table *T = M->tab;
  const int nv = M->nv;
  const int n = m->blk[4 * b];
  const int o[3] = {m->blk[4 * b + 1], m->blk[4 * b + 2], m->blk[4 * b + 3]};
  const size_t np3 = (size_t)PADX(n) * PADX(n) * PADX(n);
  const size_t n3 = (size_t)n * n * n;
  const size_t nf = (size_t)(n + 1) * n * n; /* faces per direction */
  const double dxb[3] = {dx_r(m, M->rl[b], 0), dx_r(m, M->rl[b], 1), dx_r(m, M->rl[b], 2)};

  double *W = malloc(np3 * nv * sizeof(double));
  double *F = malloc(3 * nf * (nv + 1) * sizeof(double)); /* fluxes + face velocity */
  unsigned char *exm = calloc(np3, 1);

  /* primitives on the padded block */
  for (size_t p = 0; p < np3; p++) {
    double q[6], w[6];
    for (int v = 0; v < nv; v++) q[v] = qpad[v * np3 + p];
    c2p(c, q, w);
    for (int v = 0; v < nv; v++) W[v * np3 + p] = w[v];
  }
  if (c->grav_kind == 2 && c->r_exc > 0.0) {
    for (int k = -2; k < n + 2; k++)
      for (int j = -2; j < n + 2; j++)
        for (int i = -2; i < n + 2; i++)
          exm[pidx(n, i, j, k)] = (unsigned char)excised(c, m, M->rl[b], o[0] + i, o[1] + j, o[2] + k, t);
  }

  /* face fluxes: direction d, face index a in [0, n] between cells a-1 and a */
  for (int d = 0; d < 3; d++) {
    int perm[3]; /* velocity components in (normal, t1, t2) order */
    perm[0] = 1 + d; perm[1] = 1 + (d + 1) % 3; perm[2] = 1 + (d + 2) % 3;
    for (int t2 = 0; t2 < n; t2++)
      for (int t1 = 0; t1 < n; t1++)
        for (int a = 0; a <= n; a++) {
          size_t pc[4];
          for (int s = 0; s < 4; s++) {
            int ii[3];
            ii[d] = a - 2 + s; ii[(d + 1) % 3] = t1; ii[(d + 2) % 3] = t2;
            pc[s] = pidx(n, ii[0], ii[1], ii[2]);
          }
          /* PLM on each primitive: left state from cell a-1, right from a */
          double wl[6], wr[6];
          for (int v = 0; v < nv; v++) {
            double q0 = W[v * np3 + pc[0]], q1 = W[v * np3 + pc[1]];
            double q2 = W[v * np3 + pc[2]], q3 = W[v * np3 + pc[3]];
            double sL = vanleer(q1 - q0, q2 - q1);
            double sR = vanleer(q2 - q1, q3 - q2);
            wl[v] = q1 + 0.5 * sL;
            wr[v] = q2 - 0.5 * sR;
          }
          /* rotate to (rho, un, ut1, ut2, U, A) */
          double rl[6], rr[6];
          rl[0] = wl[0]; rr[0] = wr[0];
          for (int s = 0; s < 3; s++) { rl[1 + s] = wl[perm[s]]; rr[1 + s] = wr[perm[s]]; }
          rl[4] = wl[4]; rr[4] = wr[4];
          double pl, cl, pr, cr;
          eos_pc(c, T, rl[0], rl[4], &pl, &cl);
          eos_pc(c, T, rr[0], rr[4], &pr, &cr);
          double fr5[5];
          if (c->riemann == 1) hlle(rl, pl, cl, rr, pr, cr, fr5);
          else hllc(rl, pl, cl, rr, pr, cr, fr5);
          double fl[7];
          fl[IDN] = fr5[0];
          for (int s = 0; s < 3; s++) fl[perm[s]] = fr5[1 + s];
          fl[IEN] = fr5[4];
          /* upwind state by the sign of the mass flux; tie -> left */
          const double *wu = fr5[0] >= 0.0 ? wl : wr;
          if (c->dual) fl[IAX] = fr5[0] * (wu[5] / wu[0]);
          double vf = fr5[0] / wu[0];
          /* excision is a one-way sink: a face between an active and an
           * excised cell keeps its flux unless the mass flux leaves the sink */
          unsigned char eL = exm[pc[1]], eR = exm[pc[2]];
          if (eL != eR) {
            int into = eR ? (fr5[0] >= 0.0) : (fr5[0] <= 0.0);
            if (!into) { for (int v = 0; v < nv; v++) fl[v] = 0.0; vf = 0.0; }
          }
          int ii[3];
          ii[d] = a; ii[(d + 1) % 3] = t1; ii[(d + 2) % 3] = t2;
          /* face array index: (a, t1, t2) with a fastest */
          size_t fi = ((size_t)t2 * n + t1) * (n + 1) + a;
          for (int v = 0; v < nv; v++) F[((size_t)d * (nv + 1) + v) * nf + fi] = fl[v];
          F[((size_t)d * (nv + 1) + nv) * nf + fi] = vf;
          (void)ii;
        }
  }

  /* boundary-face fluxes for the LAT impulse (face = 2*d + side) */
  if (bflux) {
    for (int d = 0; d < 3; d++)
      for (int side = 0; side < 2; side++) {
        int a = side ? n : 0;
        for (int t2 = 0; t2 < n; t2++)
          for (int t1 = 0; t1 < n; t1++) {
            size_t fi = ((size_t)t2 * n + t1) * (n + 1) + a;
            /* face-cell index over the two transverse axes in increasing axis order */
            int ax[3]; ax[(d + 1) % 3] = t1; ax[(d + 2) % 3] = t2;
            int u0 = d == 0 ? ax[1] : ax[0];
            int u1 = d == 2 ? ax[1] : ax[2];
            for (int v = 0; v < nv; v++)
              bflux[((size_t)(2 * d + side) * nv + v) * n * n + fidx(n, u0, u1)] =
                  F[((size_t)d * (nv + 1) + v) * nf + fi];
          }
      }
  }

  /* cell update */
  const double tau = stage == 1 ? dt : 0.5 * dt;
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) {
        int lc[3] = {i, j, k};
        size_t p = pidx(n, i, j, k);
        double rhs[6] = {0, 0, 0, 0, 0, 0};
        double divv = 0.0;
        for (int d = 0; d < 3; d++) {
          int tt1 = lc[(d + 1) % 3], tt2 = lc[(d + 2) % 3];
          size_t fm = ((size_t)tt2 * n + tt1) * (n + 1) + lc[d];
          size_t fp = fm + 1;
          for (int v = 0; v < nv; v++) {
            const double *Fv = F + ((size_t)d * (nv + 1) + v) * nf;
            rhs[v] -= (Fv[fp] - Fv[fm]) / dxb[d];
          }
          const double *Vf = F + ((size_t)d * (nv + 1) + nv) * nf;
          divv += (Vf[fp] - Vf[fm]) / dxb[d];
          if (c->grav_kind) {
            int im[3] = {i, j, k}, ip[3] = {i, j, k};
            im[d] -= 1; ip[d] += 1;
            double pm = phi_at(M, phi, b, im[0], im[1], im[2], t);
            double p0 = phi_at(M, phi, b, i, j, k, t);
            double pp = phi_at(M, phi, b, ip[0], ip[1], ip[2], t);
            double rho_i = qpad[IDN * np3 + p];
            rhs[IM1 + d] -= rho_i * (pp - pm) / (2.0 * dxb[d]);
            const double *Fr = F + ((size_t)d * (nv + 1) + IDN) * nf;
            rhs[IEN] -= (Fr[fp] * (pp - p0) + Fr[fm] * (p0 - pm)) / (2.0 * dxb[d]);
          }
        }
        double qn[6];
        for (int v = 0; v < nv; v++) {
          double qs = qpad[v * np3 + p] + dt * rhs[v];
          qn[v] = stage == 1 ? qs : 0.5 * qbase[v * n3 + cidx(n, i, j, k)] + 0.5 * qs;
        }
        if (c->dual) {
          /* compression of the auxiliary energy over this stage's time */
          double rho_in = qpad[IDN * np3 + p];
          if (c->eos_kind == 0) {
            qn[IAX] = qn[IAX] * exp(-(c->gamma - 1.0) * divv * tau);
          } else {
            double Pa, ca;
            /* eos_pc floors its energy argument before the table call */
            eos_pc(c, T, rho_in, qn[IAX], &Pa, &ca);
            qn[IAX] = qn[IAX] - Pa * divv * tau;
          }
          double uf = u_floor(c, qn[IDN] > c->rho_floor ? qn[IDN] : c->rho_floor);
          if (qn[IAX] < uf) qn[IAX] = uf;
        }
        /* floors */
        if (qn[IDN] < c->rho_floor) qn[IDN] = c->rho_floor;
        {
          double w[6];
          c2p(c, qn, w);
          double uf = u_floor(c, qn[IDN]);
          if (w[4] < uf) {
            qn[IEN] += uf - w[4];
            if (c->dual && qn[IAX] < uf) qn[IAX] = uf;
          }
        }
        /* resynchronisation against the stage-input total energy of the 7-point neighbourhood */
        if (c->dual) {
          double emax = qpad[IEN * np3 + p];
          for (int d = 0; d < 3; d++) {
            int im[3] = {i, j, k}, ip[3] = {i, j, k};
            im[d] -= 1; ip[d] += 1;
            double e1 = qpad[IEN * np3 + pidx(n, im[0], im[1], im[2])];
            double e2 = qpad[IEN * np3 + pidx(n, ip[0], ip[1], ip[2])];
            if (e1 > emax) emax = e1;
            if (e2 > emax) emax = e2;
          }
          double K = 0.5 * (qn[IM1] * qn[IM1] + qn[IM2] * qn[IM2] + qn[IM3] * qn[IM3]) / qn[IDN];
          double Uc = qn[IEN] - K;
          if (Uc > 0.0 && Uc > c->eta2 * emax) qn[IAX] = Uc;
        }
        for (int v = 0; v < nv; v++) out[v * n3 + cidx(n, i, j, k)] = qn[v];
      }
  free(W); free(F); free(exm);
}

/* reset excised cells to the zero-momentum floor state */
static void excise_reset(const mesh_t *M, int b, double *q, double t) {
  const orc_cfg *c = M->cfg;
  const orc_mesh *m = M->m;
  if (c->grav_kind != 2 || !(c->r_exc > 0.0)) return;
  int n = m->blk[4 * b];
  size_t n3 = (size_t)n * n * n;
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) {
        if (!excised(c, m, M->rl[b], m->blk[4 * b + 1] + i, m->blk[4 * b + 2] + j, m->blk[4 * b + 3] + k, t)) continue;
        size_t p = cidx(n, i, j, k);
        double uf = u_floor(c, c->rho_floor);
        q[IDN * n3 + p] = c->rho_floor;
        q[IM1 * n3 + p] = 0.0; q[IM2 * n3 + p] = 0.0; q[IM3 * n3 + p] = 0.0;
        q[IEN * n3 + p] = uf;
        if (c->dual) q[IAX * n3 + p] = uf;
      }
}

/* ------------------------------------------------------------------ */
/* CFL time step per block (eq lat-base-dt uses its minimum)           */
/* ------------------------------------------------------------------ */
int orc_cfl(const orc_cfg *cfg, const orc_mesh *m, const orc_table *tab, const double *U, const double *phi, double t,
            double *dt_block) {
  mesh_t M;
  if (mesh_build(&M, cfg, m, tab)) return -1;
  int nb = m->nblocks;
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < nb; b++) {
    int n = m->blk[4 * b];
    size_t n3 = (size_t)n * n * n;
    const double *q = U + M.off[b];
    double best = INFINITY;
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
          if (excised(cfg, m, M.rl[b], m->blk[4 * b + 1] + i, m->blk[4 * b + 2] + j, m->blk[4 * b + 3] + k, t)) continue;
          size_t p = cidx(n, i, j, k);
          double qq[6], w[6];
          for (int v = 0; v < M.nv; v++) qq[v] = q[v * n3 + p];
          c2p(cfg, qq, w);
          double P, cs;
          eos_pc(cfg, tab, w[0], w[4], &P, &cs);
          for (int d = 0; d < 3; d++) {
            double s = dx_r(m, M.rl[b], d) / (fabs(w[1 + d]) + cs);
            if (s < best) best = s;
          }
          /* source-term limit: the gravitational acceleration may move the gas
           * at most one cell width within the step, sqrt(dx_min / |g|) */
          if (cfg->grav_kind) {
            double g2 = 0.0;
            for (int d = 0; d < 3; d++) {
              int ip[3] = {i, j, k}, im[3] = {i, j, k};
              ip[d] += 1; im[d] -= 1;
              double gd = (phi_at(&M, phi, b, ip[0], ip[1], ip[2], t) - phi_at(&M, phi, b, im[0], im[1], im[2], t)) /
                          (2.0 * dx_r(m, M.rl[b], d));
              g2 += gd * gd;
            }
            double dmin = fmin(dx_r(m, M.rl[b], 0), fmin(dx_r(m, M.rl[b], 1), dx_r(m, M.rl[b], 2)));
            if (g2 > 0.0) {
              double s = sqrt(dmin / sqrt(g2));
              if (s < best) best = s;
            }
          }
        }
    dt_block[b] = cfg->cfl * best;
  }
  mesh_free(&M);
  return 0;
}

/* ------------------------------------------------------------------ */
/* LAT level assignment (eq lat-factor, bin merging, neighbour limit)  */
/* ------------------------------------------------------------------ */

/* blocks sharing a face, edge or corner (periodic wrap; nothing beyond outflow
 * edges), whatever their refinement level: the lattice cells (level-0 units)
 * around the block's extent */
static int *adjacency(const mesh_t *M, int *deg_out_max) {
  const orc_mesh *m = M->m;
  int nb = m->nblocks, maxd = 64;
  int *adj = malloc((size_t)nb * maxd * sizeof(int));
  int N[3] = {m->nx, m->ny, m->nz};
  for (int b = 0; b < nb; b++) {
    int cnt = 0;
    int r = M->rl[b], L = M->lat;
    int n0 = m->blk[4 * b] >> r; /* extent in level-0 cells */
    int o[3] = {m->blk[4 * b + 1] >> r, m->blk[4 * b + 2] >> r, m->blk[4 * b + 3] >> r};
    for (int cz = o[2] - L; cz < o[2] + n0 + L; cz += L)
      for (int cy = o[1] - L; cy < o[1] + n0 + L; cy += L)
        for (int cx = o[0] - L; cx < o[0] + n0 + L; cx += L) {
          int g[3] = {cx, cy, cz}, ok = 1;
          for (int d = 0; d < 3; d++) {
            if (!inside_axis(g[d], N[d], m->bc[d])) ok = 0;
            else g[d] = wrap_axis(g[d], N[d], m->bc[d]);
          }
          if (!ok) continue;
          int nb2 = covering_block(M, 0, g[0], g[1], g[2]);
          if (nb2 == b) continue;
          int seen = 0;
          for (int s2 = 0; s2 < cnt; s2++) if (adj[b * maxd + s2] == nb2) seen = 1;
          if (!seen && cnt < maxd - 1) adj[b * maxd + cnt++] = nb2;
        }
    adj[b * maxd + cnt] = -1;
  }
  *deg_out_max = maxd;
  return adj;
}

/* Admissible pair of LAT exponents e (factor 2^e) for adjacent blocks b, c:
 * on the same refinement level at most one apart; across a coarse-fine
 * interface f_fine <= f_coarse <= 2 f_fine (Sec. LAT method). */
static int exps_admissible(const mesh_t *M, int b, int c, int eb, int ec) {
  int rb = M->rl[b], rc = M->rl[c];
  if (rb == rc) return abs(eb - ec) <= 1;
  if (rb > rc) return eb <= ec && ec <= eb + 1; /* b fine, c coarse */
  return ec <= eb && eb <= ec + 1;               /* b coarse, c fine */
}

/*
 * dt_block -> levels.  exps[b] = min(N_LAT, floor(log2(dt_b / dt0))) is taken
 * with ilogb (exact), bins are merged from the top while they hold fewer than
 * merge_frac * N blocks, then neighbours are limited by relaxation to the
 * fixed point: one exponent apart on one refinement level, and
 * f_fine <= f_coarse <= 2 f_fine across refinement levels (Sec. LAT method).
 * The relaxation only lowers exponents, so it ends at the greatest admissible
 * assignment below the CFL bins.  Output level = Lmax - exponent, so level 0
 * is the coarsest (largest step) and Lmax the finest.  Returns Lmax.
 */
int orc_lat_assign(const orc_cfg *cfg, const orc_mesh *m, const double *dt_block, int *levels, double *dt0_out) {
  mesh_t M;
  if (mesh_build(&M, cfg, m, NULL)) return -1;
  int nb = m->nblocks;
  double dt0 = INFINITY;
  for (int b = 0; b < nb; b++) if (dt_block[b] < dt0) dt0 = dt_block[b];
  int *e = malloc(nb * sizeof(int));
  for (int b = 0; b < nb; b++) {
    double r = dt_block[b] / dt0;
    int k = ilogb(r);
    if (k > cfg->n_lat) k = cfg->n_lat;
    if (k < 0) k = 0;
    e[b] = k;
  }
  /* merge sparse top bins */
  for (;;) {
    int top = 0, cnt = 0;
    for (int b = 0; b < nb; b++) if (e[b] > top) top = e[b];
    if (top == 0) break;
    for (int b = 0; b < nb; b++) if (e[b] == top) cnt++;
    if ((double)cnt >= cfg->merge_frac * nb) break;
    for (int b = 0; b < nb; b++) if (e[b] == top) e[b] = top - 1;
  }
  /* neighbour limit, relaxed to its fixed point: e_b <= e_c + 1 for every
   * neighbour c on the same refinement level or a finer one, and e_b <= e_c
   * for a fine block b next to a coarser c (f_fine <= f_coarse <= 2 f_fine) */
  int maxd;
  int *adj = adjacency(&M, &maxd);
  for (int changed = 1; changed;) {
    changed = 0;
    for (int b = 0; b < nb; b++)
      for (int s = 0; adj[b * maxd + s] >= 0; s++) {
        int cN = adj[b * maxd + s];
        int cap = M.rl[b] > M.rl[cN] ? e[cN] : e[cN] + 1;
        if (e[b] > cap) { e[b] = cap; changed = 1; }
      }
  }
  int Lmax = 0;
  for (int b = 0; b < nb; b++) if (e[b] > Lmax) Lmax = e[b];
  for (int b = 0; b < nb; b++) levels[b] = Lmax - e[b];
  if (dt0_out) *dt0_out = dt0;
  free(e); free(adj); mesh_free(&M);
  return Lmax;
}

/* ------------------------------------------------------------------ */
/* LAT window (and the synchronous step as its one-level special case) */
/* ------------------------------------------------------------------ */
typedef struct {
  mesh_t *M;
  const double *phi;
  double *Qend, *Qstart, *Q1, *Qnew, *imp, *bf1, *bf2;
  int *f;      /* factor per block (in dt0 units) */
} lat_t;

/* Heun's method has the continuous extension (dense output) with weights
 * b1 = th - th^2/2, b2 = th^2/2 on its two stage slopes; written with the
 * stored start, stage-1 and end states of the step it is
 * Q(th) = (1 - th) Qn + th (1 - th) Q1 + th^2 Q_{n+1}, second order in time.
 * The weights are nonnegative and sum to one, so the value is a convex
 * combination of three admissible states: its density, energies and (the
 * internal energy being concave in the conserved variables) internal energy
 * stay positive. */
static double dense_value(double qn, double q1, double qe, double th) {
  return (1.0 - th) * qn + th * (1.0 - th) * q1 + th * th * qe;
}

/* Value at the reader's stage time of a neighbour quantity whose stored
 * history is qs (start of the neighbour's step), q1 (its stage-1 output) and
 * qe (its latest state): the reader nbk-neighbour relation at sub-cycle k in
 * phase ph (1 or 2) with factors fb (reader) and fn (neighbour).  A neighbour
 * that is mid-step at the reader's stage time uses its RK2 dense output with
 * ghost_dense, else the linear interpolation of start and end (Sec. LAT
 * method). */
static double hist_interp(const lat_t *L, int reader, int nbk, double qs, double q1, double qe, int k, int ph) {
  int fb = L->f[reader], fn = L->f[nbk];
  int act = (k % fn) == 0;
  const int dense = L->M->cfg->ghost_dense;
  if (ph == 1) {
    if (act) return qe;
    int t0 = k - k % fn;
    double w = (double)(k - t0) / fn;
    if (dense) return dense_value(qs, q1, qe, w);
    return (1.0 - w) * qs + w * qe;
  }
  if (act) {
    if (fn <= fb) return q1;
    double w = (double)fb / fn;
    return (1.0 - w) * qe + w * q1;
  }
  int t0 = k - k % fn;
  double w = (double)(k + fb - t0) / fn;
  if (dense) return dense_value(qs, q1, qe, w);
  return (1.0 - w) * qs + w * qe;
}

/* conserved value of variable v at a cell of block nbk, as the reader sees it */
static double ghost_value(const lat_t *L, int reader, int nbk, size_t cell, int v, int k, int ph) {
  const mesh_t *M = L->M;
  int n = M->m->blk[4 * nbk];
  size_t o = M->off[nbk] + v * (size_t)n * n * n + cell;
  return hist_interp(L, reader, nbk, L->Qstart[o], L->Q1[o], L->Qend[o], k, ph);
}

/* global cell index g of level r along axis d mapped into the level's extents
 * (periodic wrap, or the nearest cell beyond an outflow edge) */
static int level_axis(const mesh_t *M, int r, int d, int g) {
  const orc_mesh *m = M->m;
  int N[3] = {m->nx, m->ny, m->nz};
  return wrap_axis(g, N[d] << r, m->bc[d]);
}

/*
 * Conserved state q[nv] of global cell G (level r, any index: it is wrapped
 * here) as the reader sees it at sub-cycle k, phase ph, whatever the level of
 * the block covering it (Sec. LAT method, coarse-fine interfaces):
 *  - covered on level r: the owner's history at the reader's stage time;
 *  - covered by a finer block: the owner's stored histories (start, stage 1,
 *    latest) are each restricted to the cell (mean of its 2x2x2 children,
 *    summed in k, j, i order), then interpolated in time;
 *  - covered by a coarser block: prolongation of the coarse cell containing G
 *    from level r-1 values taken at the same stage time, q_c + sum_d s_d d_d/4
 *    (axes in x, y, z order), with d_d the minmod of the two one-sided coarse
 *    differences along d and s_d = +1 for the upper child, -1 for the lower.
 */
static void cell_state(const lat_t *L, int reader, int r, const int G[3], int k, int ph, double *q) {
  const mesh_t *M = L->M;
  const orc_mesh *m = M->m;
  const int nv = M->nv;
  int g[3];
  for (int d = 0; d < 3; d++) g[d] = level_axis(M, r, d, G[d]);
  int c = covering_block(M, r, g[0], g[1], g[2]);
  int rc = M->rl[c];
  int n = m->blk[4 * c];
  size_t n3 = (size_t)n * n * n;
  if (rc == r) {
    size_t cell = cidx(n, g[0] - m->blk[4 * c + 1], g[1] - m->blk[4 * c + 2], g[2] - m->blk[4 * c + 3]);
    for (int v = 0; v < nv; v++) q[v] = ghost_value(L, reader, c, cell, v, k, ph);
    return;
  }
  if (rc == r + 1) {
    int base[3] = {2 * g[0] - m->blk[4 * c + 1], 2 * g[1] - m->blk[4 * c + 2], 2 * g[2] - m->blk[4 * c + 3]};
    for (int v = 0; v < nv; v++) {
      double hs = 0.0, h1 = 0.0, he = 0.0;
      for (int kz = 0; kz < 2; kz++)
        for (int jy = 0; jy < 2; jy++)
          for (int ix = 0; ix < 2; ix++) {
            size_t o = M->off[c] + v * n3 + cidx(n, base[0] + ix, base[1] + jy, base[2] + kz);
            hs += L->Qstart[o]; h1 += L->Q1[o]; he += L->Qend[o];
          }
      q[v] = hist_interp(L, reader, c, 0.125 * hs, 0.125 * h1, 0.125 * he, k, ph);
    }
    return;
  }
  /* rc == r - 1: prolongation from the coarse level */
  int gc[3] = {g[0] >> 1, g[1] >> 1, g[2] >> 1};
  double qc[6], qm[3][6], qp[3][6];
  cell_state(L, reader, r - 1, gc, k, ph, qc);
  for (int d = 0; d < 3; d++) {
    int a[3] = {gc[0], gc[1], gc[2]}, b2[3] = {gc[0], gc[1], gc[2]};
    a[d] -= 1; b2[d] += 1;
    cell_state(L, reader, r - 1, a, k, ph, qm[d]);
    cell_state(L, reader, r - 1, b2, k, ph, qp[d]);
  }
  for (int v = 0; v < nv; v++) {
    double val = qc[v];
    for (int d = 0; d < 3; d++) {
      double dl = qc[v] - qm[d][v], dr = qp[d][v] - qc[v];
      double mm = dl * dr <= 0.0 ? 0.0 : (fabs(dl) < fabs(dr) ? dl : dr);
      double s = (g[d] & 1) ? 0.25 : -0.25;
      val += s * mm;
    }
    q[v] = val;
  }
}

/* dense output of one value, for pins */
double orc_dense_value(double qn, double q1, double qe, double th) { return dense_value(qn, q1, qe, th); }

static void fill_pad(const lat_t *L, int b, int k, int ph, double *qpad) {
  const mesh_t *M = L->M;
  const orc_mesh *m = M->m;
  int n = m->blk[4 * b], r = M->rl[b];
  size_t np3 = (size_t)PADX(n) * PADX(n) * PADX(n);
  for (int kk = -2; kk < n + 2; kk++)
    for (int jj = -2; jj < n + 2; jj++)
      for (int ii = -2; ii < n + 2; ii++) {
        int G[3] = {m->blk[4 * b + 1] + ii, m->blk[4 * b + 2] + jj, m->blk[4 * b + 3] + kk};
        double q[6];
        cell_state(L, b, r, G, k, ph, q);
        for (int v = 0; v < M->nv; v++) qpad[v * np3 + pidx(n, ii, jj, kk)] = q[v];
      }
}

/* Neighbour across face (d, side) of local face cell (u0,u1) of block b:
 * returns the block covering the cell across, or -1 beyond an outflow edge.
 * (*u0n, *u1n) index the neighbour's face cell on its opposite face: the
 * coarse cell containing the one across for a coarser neighbour, the first
 * (lowest-index) of the 2x2 fine face cells for a finer one. */
static int face_neighbor(const mesh_t *M, int b, int d, int side, int u0, int u1, int *u0n, int *u1n, int *ci) {
  const orc_mesh *m = M->m;
  int n = m->blk[4 * b], r = M->rl[b];
  int loc[3];
  if (d == 0) { loc[1] = u0; loc[2] = u1; }
  if (d == 1) { loc[0] = u0; loc[2] = u1; }
  if (d == 2) { loc[0] = u0; loc[1] = u1; }
  loc[d] = side ? n - 1 : 0;
  int g[3] = {m->blk[4 * b + 1] + loc[0], m->blk[4 * b + 2] + loc[1], m->blk[4 * b + 3] + loc[2]};
  *ci = (int)cidx(n, loc[0], loc[1], loc[2]);
  g[d] += side ? 1 : -1;
  int N[3] = {m->nx << r, m->ny << r, m->nz << r};
  if (!inside_axis(g[d], N[d], m->bc[d])) return -1;
  for (int a = 0; a < 3; a++) g[a] = wrap_axis(g[a], N[a], m->bc[a]);
  int nbk = covering_block(M, r, g[0], g[1], g[2]);
  int rn = M->rl[nbk];
  int h[3];
  for (int a = 0; a < 3; a++) {
    if (rn == r) h[a] = g[a];
    else if (rn < r) h[a] = g[a] >> 1;
    else h[a] = a == d ? 2 * g[a] + (side ? 0 : 1) : 2 * g[a];
  }
  int ln[3] = {h[0] - m->blk[4 * nbk + 1], h[1] - m->blk[4 * nbk + 2], h[2] - m->blk[4 * nbk + 3]};
  *u0n = d == 0 ? ln[1] : ln[0];
  *u1n = d == 2 ? ln[1] : ln[2];
  return nbk;
}

/*
 * One LAT window of f_max = 2^Lmax sub-cycles of dt0 (Lmax = max level).
 * Block b with level l has factor f = 2^(Lmax - l).  Returns the number of
 * block updates performed, or -1 on invalid input.
 */
int64_t orc_lat_window(const orc_cfg *cfg, const orc_mesh *m, const orc_table *tab, double *U, const double *phi,
                       const int *levels, double dt0, double t0) {
  mesh_t M;
  if (mesh_build(&M, cfg, m, tab)) return -1;
  int nb = m->nblocks, nv = M.nv;
  int Lmax = 0;
  for (int b = 0; b < nb; b++) {
    if (levels[b] < 0 || levels[b] > 30) { mesh_free(&M); return -1; }
    if (levels[b] > Lmax) Lmax = levels[b];
  }
  /* neighbour levels must be admissible (exponent = Lmax - level) */
  {
    int maxd;
    int *adj = adjacency(&M, &maxd);
    for (int b = 0; b < nb; b++)
      for (int s = 0; adj[b * maxd + s] >= 0; s++) {
        int c = adj[b * maxd + s];
        if (!exps_admissible(&M, b, c, Lmax - levels[b], Lmax - levels[c])) { free(adj); mesh_free(&M); return -1; }
        if (abs(M.rl[b] - M.rl[c]) > 1) { free(adj); mesh_free(&M); return -1; }
      }
    free(adj);
  }
  lat_t L;
  L.M = &M; L.phi = phi;
  L.Qend = U;
  L.Qstart = malloc(M.total * sizeof(double));
  L.Q1 = calloc(M.total, sizeof(double));
  L.Qnew = malloc(M.total * sizeof(double));
  L.imp = calloc(M.itotal, sizeof(double));
  L.bf1 = calloc(M.itotal, sizeof(double));
  L.bf2 = calloc(M.itotal, sizeof(double));
  L.f = malloc(nb * sizeof(int));
  for (int b = 0; b < nb; b++) L.f[b] = 1 << (Lmax - levels[b]);
  memcpy(L.Qstart, U, M.total * sizeof(double));
  int fmax = 1 << Lmax;
  int64_t updates = 0;
  for (int k = 0; k < fmax; k++) {
    double tk = t0 + k * dt0;
    /* phase 1 */
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < nb; b++) {
      if (k % L.f[b]) continue;
      int n = m->blk[4 * b];
      size_t np3 = (size_t)PADX(n) * PADX(n) * PADX(n);
      double *qpad = malloc(np3 * nv * sizeof(double));
      fill_pad(&L, b, k, 1, qpad);
      block_stage(&M, phi, b, qpad, NULL, 1, L.f[b] * dt0, tk, L.Q1 + M.off[b], L.bf1 + M.ioff[b]);
      free(qpad);
    }
    /* phase 2 */
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < nb; b++) {
      if (k % L.f[b]) continue;
      int n = m->blk[4 * b];
      size_t np3 = (size_t)PADX(n) * PADX(n) * PADX(n);
      double *qpad = malloc(np3 * nv * sizeof(double));
      fill_pad(&L, b, k, 2, qpad);
      double dtb = L.f[b] * dt0;
      block_stage(&M, phi, b, qpad, L.Qend + M.off[b], 2, dtb, tk + dtb, L.Qnew + M.off[b], L.bf2 + M.ioff[b]);
      excise_reset(&M, b, L.Qnew + M.off[b], tk + dtb);
      free(qpad);
    }
    /* time-integrated boundary impulses (eq lat-flux-impulse) */
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < nb; b++) {
      if (k % L.f[b]) continue;
      int n = m->blk[4 * b];
      double dtb = L.f[b] * dt0;
      for (int d = 0; d < 3; d++) {
        double area = dx_r(m, M.rl[b], (d + 1) % 3) * dx_r(m, M.rl[b], (d + 2) % 3);
        for (int side = 0; side < 2; side++)
          for (int u1 = 0; u1 < n; u1++)
            for (int u0 = 0; u0 < n; u0++) {
              int u0n, u1n, ci;
              int nbk = face_neighbor(&M, b, d, side, u0, u1, &u0n, &u1n, &ci);
              if (nbk < 0) continue;
              int fw = L.f[b] > L.f[nbk] ? L.f[b] : L.f[nbk];
              int overwrite = (k % fw) == 0;
              for (int v = 0; v < nv; v++) {
                size_t ix = M.ioff[b] + ((size_t)(2 * d + side) * nv + v) * n * n + fidx(n, u0, u1);
                double Is = 0.5 * (L.bf1[ix] + L.bf2[ix]) * area * dtb;
                L.imp[ix] = overwrite ? Is : L.imp[ix] + Is;
              }
            }
      }
    }
    /* commit */
    for (int b = 0; b < nb; b++) {
      if (k % L.f[b]) continue;
      int n = m->blk[4 * b];
      size_t sz = (size_t)nv * n * n * n;
      memcpy(L.Qstart + M.off[b], L.Qend + M.off[b], sz * sizeof(double));
      memcpy(L.Qend + M.off[b], L.Qnew + M.off[b], sz * sizeof(double));
      updates++;
    }
    /* Flux corrections (eq lat-flux-impulse and the reflux after it) for
     * blocks completing at k+1: against neighbours on the same refinement
     * level that update more often, and against every finer neighbour, whose
     * 2x2 face impulses (summed in u1, u0 order) replace the coarse face's own;
     * a block never corrects against a coarser neighbour. */
    double tc = t0 + (k + 1) * dt0;
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < nb; b++) {
      if ((k + 1) % L.f[b]) continue;
      int n = m->blk[4 * b];
      size_t n3 = (size_t)n * n * n;
      int r = M.rl[b];
      double vol = dx_r(m, r, 0) * dx_r(m, r, 1) * dx_r(m, r, 2);
      /* cells in increasing index order, faces in order x-, x+, y-, y+, z-, z+ */
      for (int kk = 0; kk < n; kk++)
        for (int jj = 0; jj < n; jj++)
          for (int ii = 0; ii < n; ii++) {
            int lc[3] = {ii, jj, kk};
            for (int d = 0; d < 3; d++)
              for (int side = 0; side < 2; side++) {
                if (lc[d] != (side ? n - 1 : 0)) continue;
                int u0 = d == 0 ? jj : ii;
                int u1 = d == 2 ? jj : kk;
                int u0n, u1n, ci;
                int nbk = face_neighbor(&M, b, d, side, u0, u1, &u0n, &u1n, &ci);
                if (nbk < 0) continue;
                int rn = M.rl[nbk];
                if (rn < r || (rn == r && L.f[nbk] >= L.f[b])) continue;
                int nn = m->blk[4 * nbk];
                int w = rn > r ? 2 : 1;
                double sg = side ? 1.0 : -1.0;
                double dI[6];
                for (int v = 0; v < nv; v++) {
                  size_t ib = M.ioff[b] + ((size_t)(2 * d + side) * nv + v) * n * n + fidx(n, u0, u1);
                  size_t in = M.ioff[nbk] + ((size_t)(2 * d + (1 - side)) * nv + v) * nn * nn;
                  double In = 0.0;
                  for (int e1 = 0; e1 < w; e1++)
                    for (int e0 = 0; e0 < w; e0++) In += L.imp[in + fidx(nn, u0n + e0, u1n + e1)];
                  dI[v] = L.imp[ib] - In;
                }
                size_t p = cidx(n, ii, jj, kk);
                double *q = L.Qend + M.off[b];
                if (cfg->grav_kind) {
                  int ln[3] = {ii, jj, kk};
                  ln[d] += side ? 1 : -1;
                  double pn = phi_at(&M, phi, b, ln[0], ln[1], ln[2], tc);
                  double pi = phi_at(&M, phi, b, ii, jj, kk, tc);
                  q[IEN * n3 + p] += sg / (2.0 * vol) * dI[IDN] * (pn - pi);
                }
                for (int v = 0; v < nv; v++) q[v * n3 + p] += sg * dI[v] / vol;
              }
          }
    }
  }
  free(L.Qstart); free(L.Q1); free(L.Qnew); free(L.imp); free(L.bf1); free(L.bf2); free(L.f);
  mesh_free(&M);
  return updates;
}

/*
 * Synchronous RK2 steps: every block on one level.  dt_in (nullable) gives
 * the step sizes; otherwise each step takes min_b of the CFL time step.
 * The step sizes used are written to dt_out (nullable).
 */
int orc_run_sync(const orc_cfg *cfg, const orc_mesh *m, const orc_table *tab, double *U, const double *phi,
                 int nsteps, const double *dt_in, double *dt_out, double t0) {
  int nb = m->nblocks;
  int *lev = calloc(nb, sizeof(int));
  double *dtb = malloc(nb * sizeof(double));
  double t = t0;
  for (int s = 0; s < nsteps; s++) {
    double dt;
    if (dt_in) dt = dt_in[s];
    else {
      if (orc_cfl(cfg, m, tab, U, phi, t, dtb)) { free(lev); free(dtb); return -1; }
      dt = INFINITY;
      for (int b = 0; b < nb; b++) if (dtb[b] < dt) dt = dtb[b];
    }
    if (orc_lat_window(cfg, m, tab, U, phi, lev, dt, t) < 0) { free(lev); free(dtb); return -1; }
    if (dt_out) dt_out[s] = dt;
    t += dt;
  }
  free(lev); free(dtb);
  return 0;
}

/* ------------------------------------------------------------------ */
/* direct entry points to single pieces, for pins                      */
/* ------------------------------------------------------------------ */
void orc_eos_eval(const orc_cfg *cfg, const orc_table *tab, int64_t n, const double *rho, const double *U, double *P,
                  double *cs) {
  for (int64_t i = 0; i < n; i++) eos_pc(cfg, tab, rho[i], U[i], P + i, cs + i);
}

/* table-only inversion: log10 rho, log10 e -> (j, wT, log10 T) */
void orc_table_invert(const orc_table *tab, int64_t n, const double *lr, const double *le, int *j, double *wT,
                      double *lT) {
  for (int64_t q = 0; q < n; q++) {
    int i, jj; double w, wt;
    table_rho_cell(tab, lr[q], &i, &w);
    table_invert(tab, i, w, le[q], &jj, &wt);
    j[q] = jj; wT[q] = wt;
    lT[q] = tab->lT0 + (jj + wt) * tab->dlT;
  }
}

/* HLLC flux of one face for given primitive states (x-normal), for pins */
void orc_hllc_flux(const double *wl, double pl, double cl, const double *wr, double pr, double cr, double *f) {
  hllc(wl, pl, cl, wr, pr, cr, f);
}

/* HLLE flux of one face for given primitive states (x-normal), for pins */
void orc_hlle_flux(const double *wl, double pl, double cl, const double *wr, double pr, double cr, double *f) {
  hlle(wl, pl, cl, wr, pr, cr, f);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads the parallel loops over blocks use from now on (timing runs only;
   every thread count gives the same result, since blocks are independent). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/*
 * Ghost fill of block b with every stored history equal to U (a state at rest
 * in time, every block on one LAT level), for pins of the coarse-fine spatial
 * operators (restriction and prolongation).  out: [nv][(n+4)^3], the padded
 * block in the layout the stage update reads.  Returns 0, or -1 on invalid
 * input.
 */
int orc_ghost_fill(const orc_cfg *cfg, const orc_mesh *m, const double *U, int b, double *out) {
  mesh_t M;
  if (mesh_build(&M, cfg, m, NULL)) return -1;
  if (b < 0 || b >= m->nblocks) { mesh_free(&M); return -1; }
  lat_t L;
  memset(&L, 0, sizeof L);
  L.M = &M;
  L.Qstart = L.Q1 = L.Qend = (double *)U;
  L.f = malloc(m->nblocks * sizeof(int));
  for (int i = 0; i < m->nblocks; i++) L.f[i] = 1;
  fill_pad(&L, b, 0, 1, out);
  free(L.f);
  mesh_free(&M);
  return 0;
}
