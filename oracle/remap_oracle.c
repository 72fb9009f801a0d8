/*
 * FP64 CPU oracle for the restart remap, the Galilean boost and the
 * frame-acceleration estimate (Sec. Domain remapping and frame conversion,
 * eqs remap-state-vector, remap-cell-average, galilean-boost; Sec. Moving-frame
 * dynamics and BH treatment, eq frame-acceleration).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this library.
 *
 * Remap, for every target cell:
 *   - inside the BH excision sphere at time t (point-mass configurations):
 *     the sink state (rho_floor, 0, U_floor), as the hydro update's reset;
 *   - centre outside the source domain along a non-periodic axis: the floor
 *     state (rho_floor, 0, U_floor);
 *   - centre inside the source domain but within BAND source cells of a
 *     source face beyond which the target domain extends (a non-periodic axis
 *     whose target extent passes that face): the remapped state below blended
 *     toward the floor state, density, momentum and thermal energy density
 *     each as s q + (1 - s) q_floor with s = 3 u^2 - 2 u^3, u = the distance
 *     to the nearest such face in units of BAND source cells (clamped to
 *     [0, 1]); total energy rebuilt from the blended values.  The floor state
 *     is at rest, and for the ideal gas the thermal energy density is the
 *     pressure over (gamma - 1), so density and pressure go smoothly to the
 *     floor across the band (the band sits in the old domain's atmosphere);
 *   - target grid coincident with the source grid (same spacing, origin an
 *     integer number of cells away): the source cell's conserved values,
 *     copied (a remap onto the same grid is the identity);
 *   - otherwise the mean over N_qd = 8 sub-cell midpoints (+-1/4 of the
 *     target cell along each axis; z outer, x inner) of the trilinear
 *     interpolant of the source cell-centred density, momentum and thermal
 *     energy density (the auxiliary energy with dual energy on, E - |m|^2/2rho
 *     otherwise); the total energy is rebuilt as U + |m|^2/2rho and the
 *     auxiliary energy is U.  Interpolation stencils clamp at non-periodic
 *     source edges and wrap across periodic ones.
 * Trilinear interpolation: along x first, then y, then z, each as
 * (1 - w) a + w b.
 *
 * Galilean boost by V: rho' = rho, m' = m + rho V, E' = E + m.V + rho |V|^2/2,
 * skipped where rho <= rho_skip (floor-density gas); U_aux unchanged.
 *
 * Frame acceleration: A = sum rho g / sum rho over cells with rho > rho_min
 * outside the excision sphere, g = -grad of the softened point-mass potential
 * at the cell centre, g = -GM (r - r_bh) / (|r - r_bh|^2 + r_soft^2)^(3/2)
 * (uniform cells: the volume cancels).
 *
 * Plain loops in IEEE double precision, no contraction.  Shares no code with
 * the GPU library.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int eos_kind, dual, grav_kind, n_lat;
  double gamma, eta1, eta2, cfl;
  double rho_floor, p_floor, e_floor;
  double merge_frac;
  double gm_bh, r_soft, r_exc;
  double bh_x0[3], v_frame[3];
  int riemann, ghost_dense;
} orc_rcfg; /* same layout as the hydro oracle's configuration */

typedef struct {
  int nx, ny, nz;
  int bc[3];
  double x0[3], dx[3];
  int nblocks;
  const int *blk;
} orc_rmesh; /* same layout as the hydro oracle's mesh description */

static double u_floor_r(const orc_rcfg *c, double rho) {
  return c->eos_kind == 0 ? c->p_floor / (c->gamma - 1.0) : rho * c->e_floor;
}

static int excised_at(const orc_rcfg *c, const double *r, double t) {
  if (c->grav_kind != 2 || !(c->r_exc > 0.0)) return 0;
  double s = 0.0;
  for (int d = 0; d < 3; d++) {
    double q = r[d] - (c->bh_x0[d] - c->v_frame[d] * t);
    s += q * q;
  }
  return s < c->r_exc * c->r_exc;
}

/* global arrays [nv'][nz][ny][nx] of a block state: rho, mx, my, mz, E, A(or 0), U_th */
static double *gather(const orc_rmesh *m, int nv, const double *U) {
  size_t N = (size_t)m->nx * m->ny * m->nz;
  double *g = malloc(7 * N * sizeof(double));
  size_t off = 0;
  for (int b = 0; b < m->nblocks; b++) {
    int n = m->blk[4 * b];
    size_t n3 = (size_t)n * n * n;
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
          size_t l = ((size_t)k * n + j) * n + i;
          size_t p = ((size_t)(m->blk[4 * b + 3] + k) * m->ny + (m->blk[4 * b + 2] + j)) * m->nx +
                     (m->blk[4 * b + 1] + i);
          double q[6] = {0, 0, 0, 0, 0, 0};
          for (int v = 0; v < nv; v++) q[v] = U[off + v * n3 + l];
          for (int v = 0; v < 6; v++) g[v * N + p] = q[v];
          double K = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
          g[6 * N + p] = nv > 5 ? q[5] : q[4] - K;
        }
    off += (size_t)nv * n3;
  }
  return g;
}

#define BAND 2.0 /* width of the blending band in source cells */

/* Blending weight of a target centre c inside the source domain: 1 away from
   the source faces the target domain extends beyond, falling smoothly to 0 at
   them (section header). */
static double band_weight(const orc_rmesh *s, const orc_rmesh *d, const double *c) {
  int Ns[3] = {s->nx, s->ny, s->nz}, Nd[3] = {d->nx, d->ny, d->nz};
  double u = 1.0;
  for (int a = 0; a < 3; a++) {
    if (s->bc[a] == 0) continue;
    double lo = s->x0[a], hi = s->x0[a] + Ns[a] * s->dx[a];
    double dlo = d->x0[a], dhi = d->x0[a] + Nd[a] * d->dx[a];
    double w = BAND * s->dx[a];
    if (dlo < lo) { double v = (c[a] - lo) / w; if (v < u) u = v; }
    if (dhi > hi) { double v = (hi - c[a]) / w; if (v < u) u = v; }
  }
  if (u <= 0.0) return 0.0;
  if (u >= 1.0) return 1.0;
  return u * u * (3.0 - 2.0 * u);
}

static int src_index(int i, int n, int periodic) {
  if (periodic) return ((i % n) + n) % n;
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* trilinear interpolant of global field f at point r */
static double trilinear(const orc_rmesh *s, const double *f, const double *r) {
  int i0[3], i1[3];
  double w[3];
  int N[3] = {s->nx, s->ny, s->nz};
  for (int d = 0; d < 3; d++) {
    double xi = (r[d] - s->x0[d]) / s->dx[d] - 0.5;
    double fl = floor(xi);
    w[d] = xi - fl;
    i0[d] = src_index((int)fl, N[d], s->bc[d] == 0);
    i1[d] = src_index((int)fl + 1, N[d], s->bc[d] == 0);
  }
#define F(a, b, c) f[((size_t)(c) * s->ny + (b)) * s->nx + (a)]
  double a00 = (1.0 - w[0]) * F(i0[0], i0[1], i0[2]) + w[0] * F(i1[0], i0[1], i0[2]);
  double a10 = (1.0 - w[0]) * F(i0[0], i1[1], i0[2]) + w[0] * F(i1[0], i1[1], i0[2]);
  double a01 = (1.0 - w[0]) * F(i0[0], i0[1], i1[2]) + w[0] * F(i1[0], i0[1], i1[2]);
  double a11 = (1.0 - w[0]) * F(i0[0], i1[1], i1[2]) + w[0] * F(i1[0], i1[1], i1[2]);
#undef F
  double b0 = (1.0 - w[1]) * a00 + w[1] * a10;
  double b1 = (1.0 - w[1]) * a01 + w[1] * a11;
  return (1.0 - w[2]) * b0 + w[2] * b1;
}

int orc_remap(const orc_rcfg *cfg, const orc_rmesh *src, const double *Us, const orc_rmesh *dst, double *Ud,
              double t) {
  int nv = cfg->dual ? 6 : 5;
  double *g = gather(src, nv, Us);
  size_t Ns = (size_t)src->nx * src->ny * src->nz;
  /* coincident grids: same spacing, origins a whole number of cells apart */
  int coincident = 1, shift[3];
  for (int d = 0; d < 3; d++) {
    double s = (dst->x0[d] - src->x0[d]) / src->dx[d];
    if (dst->dx[d] != src->dx[d] || s != floor(s) || fabs(s) > 1e9) coincident = 0;
    else shift[d] = (int)s;
  }
  int Ns3[3] = {src->nx, src->ny, src->nz};
  size_t off = 0;
  for (int b = 0; b < dst->nblocks; b++) {
    int n = dst->blk[4 * b];
    size_t n3 = (size_t)n * n * n;
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
          int gi[3] = {dst->blk[4 * b + 1] + i, dst->blk[4 * b + 2] + j, dst->blk[4 * b + 3] + k};
          double c[3];
          for (int d = 0; d < 3; d++) c[d] = dst->x0[d] + (gi[d] + 0.5) * dst->dx[d];
          double q[6], uth0 = 0.0; /* conserved state; its thermal energy density */
          int outside = 0;
          for (int d = 0; d < 3; d++) {
            double lo = src->x0[d], hi = src->x0[d] + Ns3[d] * src->dx[d];
            if (src->bc[d] != 0 && (c[d] < lo || c[d] >= hi)) outside = 1;
          }
          if (excised_at(cfg, c, t) || outside) {
            double uf = u_floor_r(cfg, cfg->rho_floor);
            q[0] = cfg->rho_floor; q[1] = q[2] = q[3] = 0.0; q[4] = uf; q[5] = uf;
          } else if (coincident) {
            int si[3];
            for (int d = 0; d < 3; d++) si[d] = src_index(gi[d] + shift[d], Ns3[d], src->bc[d] == 0);
            size_t p = ((size_t)si[2] * src->ny + si[1]) * src->nx + si[0];
            for (int v = 0; v < 6; v++) q[v] = g[v * Ns + p];
            uth0 = g[6 * Ns + p];
          } else {
            double acc[5] = {0, 0, 0, 0, 0}; /* rho, mx, my, mz, U */
            for (int sz = 0; sz < 2; sz++)
              for (int sy = 0; sy < 2; sy++)
                for (int sx = 0; sx < 2; sx++) {
                  double r[3] = {c[0] + (sx ? 0.25 : -0.25) * dst->dx[0], c[1] + (sy ? 0.25 : -0.25) * dst->dx[1],
                                 c[2] + (sz ? 0.25 : -0.25) * dst->dx[2]};
                  acc[0] += trilinear(src, g + 0 * Ns, r);
                  acc[1] += trilinear(src, g + 1 * Ns, r);
                  acc[2] += trilinear(src, g + 2 * Ns, r);
                  acc[3] += trilinear(src, g + 3 * Ns, r);
                  acc[4] += trilinear(src, g + 6 * Ns, r);
                }
            for (int v = 0; v < 5; v++) acc[v] *= 0.125;
            q[0] = acc[0]; q[1] = acc[1]; q[2] = acc[2]; q[3] = acc[3];
            q[4] = acc[4] + 0.5 * (acc[1] * acc[1] + acc[2] * acc[2] + acc[3] * acc[3]) / acc[0];
            q[5] = acc[4];
            uth0 = acc[4];
          }
          if (!excised_at(cfg, c, t) && !outside) {
            double w = band_weight(src, dst, c);
            if (w < 1.0) {
              double uf = u_floor_r(cfg, cfg->rho_floor);
              double rho = w * q[0] + (1.0 - w) * cfg->rho_floor;
              double m[3] = {w * q[1], w * q[2], w * q[3]};
              double uth = w * uth0 + (1.0 - w) * uf;
              q[0] = rho; q[1] = m[0]; q[2] = m[1]; q[3] = m[2];
              q[4] = uth + 0.5 * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / rho;
              q[5] = uth;
            }
          }
          size_t l = ((size_t)k * n + j) * n + i;
          for (int v = 0; v < nv; v++) Ud[off + v * n3 + l] = q[v];
        }
    off += (size_t)nv * n3;
  }
  free(g);
  return 0;
}

void orc_galilean_boost(const orc_rcfg *cfg, const orc_rmesh *m, double *U, const double *V, double rho_skip) {
  int nv = cfg->dual ? 6 : 5;
  size_t off = 0;
  for (int b = 0; b < m->nblocks; b++) {
    int n = m->blk[4 * b];
    size_t n3 = (size_t)n * n * n;
    for (size_t l = 0; l < n3; l++) {
      double *q0 = U + off + l;
      double rho = q0[0];
      if (!(rho > rho_skip)) continue;
      double mx = q0[1 * n3], my = q0[2 * n3], mz = q0[3 * n3];
      double mv = (mx * V[0] + my * V[1]) + mz * V[2];
      double v2 = (V[0] * V[0] + V[1] * V[1]) + V[2] * V[2];
      q0[4 * n3] = (q0[4 * n3] + mv) + 0.5 * rho * v2;
      q0[1 * n3] = mx + rho * V[0];
      q0[2 * n3] = my + rho * V[1];
      q0[3 * n3] = mz + rho * V[2];
    }
    off += (size_t)nv * n3;
  }
}

void orc_frame_acceleration(const orc_rcfg *cfg, const orc_rmesh *m, const double *U, double rho_min, double t,
                            double *A) {
  int nv = cfg->dual ? 6 : 5;
  double sm = 0.0, sg[3] = {0.0, 0.0, 0.0};
  size_t off = 0;
  for (int b = 0; b < m->nblocks; b++) {
    int n = m->blk[4 * b];
    size_t n3 = (size_t)n * n * n;
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++) {
          double rho = U[off + ((size_t)k * n + j) * n + i];
          double c[3] = {m->x0[0] + (m->blk[4 * b + 1] + i + 0.5) * m->dx[0],
                         m->x0[1] + (m->blk[4 * b + 2] + j + 0.5) * m->dx[1],
                         m->x0[2] + (m->blk[4 * b + 3] + k + 0.5) * m->dx[2]};
          if (!(rho > rho_min) || excised_at(cfg, c, t)) continue;
          double dr[3], r2 = cfg->r_soft * cfg->r_soft;
          for (int d = 0; d < 3; d++) {
            dr[d] = c[d] - (cfg->bh_x0[d] - cfg->v_frame[d] * t);
            r2 += dr[d] * dr[d];
          }
          double f = -cfg->gm_bh / (r2 * sqrt(r2));
          sm += rho;
          for (int d = 0; d < 3; d++) sg[d] += rho * (f * dr[d]);
        }
    off += (size_t)nv * n3;
  }
  for (int d = 0; d < 3; d++) A[d] = sm > 0.0 ? sg[d] / sm : 0.0;
}
