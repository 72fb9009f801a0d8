/*
 * FP64 CPU oracle for the self-gravity solve (Sec. Self-gravity solver).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this library: only the tests,
 * the smoke check and the CPU baseline of the benchmark load it.
 *
 * Problem: the periodic Poisson problem A Phi = S on the mesh's uniform grid,
 * with A = -lap_h the positive-definite seven-point operator (eq
 * selfgrav-poisson) and S = -4 pi G (rho - mean rho): on a periodic domain the
 * source must have zero mean, so the mean density is subtracted (the periodic
 * form of the solve; isolated boundaries are not part of this oracle), in two
 * passes as the paper does (the second removes the first's rounding residue).
 * Anisotropic cells enter as the paper states: neighbours in y and z carry
 * weights wy = (dx/dy)^2, wz = (dx/dz)^2 and the centre 2 (1 + wy + wz).
 *
 * Method, in the paper's order: geometric multigrid V-cycles on a hierarchy
 * that halves every axis while all are even (down to at least 2 cells); the
 * smoother is red-black Gauss-Seidel (red = even i+j+k) over-relaxed with
 * omega = 1.15; two pre- and two post-smoothing sweeps on every level; the
 * defect d = S - A Phi (eq selfgrav-defect) is averaged over the eight child
 * cells onto the coarser level, where the correction is computed in
 * full-approximation form (coarse source R d + A_c R Phi, coarse start R Phi);
 * the correction (coarse result - R Phi) returns to the fine level by tricubic
 * interpolation (Lagrange cubics through the four nearest coarse centres per
 * axis, applied axis by axis); each V-cycle ends with one extra sweep on the
 * finest level.  The coarsest level is smoothed 2 (nx+ny+nz)^2 times.  The
 * defect is monitored by its root mean square over the finest cells.  After
 * the last cycle the potential is shifted to zero mean (on a periodic domain
 * it is defined up to a constant; only its differences enter the update).
 *
 * Every loop runs in a fixed order in IEEE double precision with no
 * floating-point contraction.  Shares no code with the GPU library.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int nx, ny, nz;
  int bc[3];
  double x0[3], dx[3];
  int nblocks;
  const int *blk; /* [nblocks][4] = n, ox, oy, oz */
} orc_gmesh;      /* same layout as the hydro oracle's mesh description */

#define MG_MAX_LEVELS 24
static const double kOmega = 1.15;

typedef struct {
  int nx, ny, nz;
  double hx2, wy, wz, c0; /* hx^2, anisotropy weights, centre coefficient */
  double *phi, *src, *tmp; /* tmp: the defect */
  double *rphi;             /* the restricted fine solution R phi (coarse levels) */
} level_t;

static size_t lidx(const level_t *L, int i, int j, int k) {
  i = ((i % L->nx) + L->nx) % L->nx;
  j = ((j % L->ny) + L->ny) % L->ny;
  k = ((k % L->nz) + L->nz) % L->nz;
  return ((size_t)k * L->ny + j) * L->nx + i;
}

/* weighted neighbour sum ((x- + x+) + wy (y- + y+)) + wz (z- + z+) */
static double nbsum(const level_t *L, const double *f, int i, int j, int k) {
  double sx = f[lidx(L, i - 1, j, k)] + f[lidx(L, i + 1, j, k)];
  double sy = f[lidx(L, i, j - 1, k)] + f[lidx(L, i, j + 1, k)];
  double sz = f[lidx(L, i, j, k - 1)] + f[lidx(L, i, j, k + 1)];
  return (sx + L->wy * sy) + L->wz * sz;
}

/* (A f)_ijk = (c0 f - nbsum) / hx^2 */
static double apply_A(const level_t *L, const double *f, int i, int j, int k) {
  return (L->c0 * f[lidx(L, i, j, k)] - nbsum(L, f, i, j, k)) / L->hx2;
}

/* one red-black sweep: red (even i+j+k) cells, then black */
static void rbgs_sweep(level_t *L) {
  for (int color = 0; color < 2; color++)
    for (int k = 0; k < L->nz; k++)
      for (int j = 0; j < L->ny; j++)
        for (int i = 0; i < L->nx; i++) {
          if (((i + j + k) & 1) != color) continue;
          size_t p = lidx(L, i, j, k);
          double gs = (nbsum(L, L->phi, i, j, k) + L->hx2 * L->src[p]) / L->c0;
          L->phi[p] = (1.0 - kOmega) * L->phi[p] + kOmega * gs;
        }
}

/* defect d = S - A phi into tmp */
static void defect(level_t *L) {
  for (int k = 0; k < L->nz; k++)
    for (int j = 0; j < L->ny; j++)
      for (int i = 0; i < L->nx; i++) {
        size_t p = lidx(L, i, j, k);
        L->tmp[p] = L->src[p] - apply_A(L, L->phi, i, j, k);
      }
}

/* mean of the eight children of coarse cell (i, j, k) */
static double child_mean(const level_t *F, const double *f, int i, int j, int k) {
  int I = 2 * i, J = 2 * j, K = 2 * k;
  double a = f[lidx(F, I, J, K)] + f[lidx(F, I + 1, J, K)];
  double b = f[lidx(F, I, J + 1, K)] + f[lidx(F, I + 1, J + 1, K)];
  double c = f[lidx(F, I, J, K + 1)] + f[lidx(F, I + 1, J, K + 1)];
  double d = f[lidx(F, I, J + 1, K + 1)] + f[lidx(F, I + 1, J + 1, K + 1)];
  return 0.125 * ((a + b) + (c + d));
}

/* cubic Lagrange weights (x 128) for a fine child at -1/4 (left) or +1/4
 * (right) of its parent's centre, through coarse centres parent-2..parent+1
 * (left) or parent-1..parent+2 (right) */
static const double kCubL[4] = {-5.0 / 128.0, 35.0 / 128.0, 105.0 / 128.0, -7.0 / 128.0};
static const double kCubR[4] = {-7.0 / 128.0, 105.0 / 128.0, 35.0 / 128.0, -5.0 / 128.0};

/* tricubic interpolation of coarse field e at fine cell (I, J, K) */
static double tricubic(const level_t *C, const double *e, int I, int J, int K) {
  int pi = I >> 1, pj = J >> 1, pk = K >> 1;
  const double *wx = (I & 1) ? kCubR : kCubL, *wy = (J & 1) ? kCubR : kCubL, *wz = (K & 1) ? kCubR : kCubL;
  int i0 = pi - ((I & 1) ? 1 : 2), j0 = pj - ((J & 1) ? 1 : 2), k0 = pk - ((K & 1) ? 1 : 2);
  double sz = 0.0;
  for (int c = 0; c < 4; c++) {
    double sy = 0.0;
    for (int b = 0; b < 4; b++) {
      double sx = 0.0;
      for (int a = 0; a < 4; a++) sx += wx[a] * e[lidx(C, i0 + a, j0 + b, k0 + c)];
      sy += wy[b] * sx;
    }
    sz += wz[c] * sy;
  }
  return sz;
}

static void vcycle(level_t *Ls, int l, int nlev) {
  level_t *L = &Ls[l];
  if (l == nlev - 1) {
    int sweeps = 2 * (L->nx + L->ny + L->nz) * (L->nx + L->ny + L->nz);
    for (int s = 0; s < sweeps; s++) rbgs_sweep(L);
    return;
  }
  level_t *C = &Ls[l + 1];
  rbgs_sweep(L);
  rbgs_sweep(L);
  defect(L);
  /* full approximation: coarse start R phi (kept in C->rphi), coarse source R d + A_c R phi */
  for (int k = 0; k < C->nz; k++)
    for (int j = 0; j < C->ny; j++)
      for (int i = 0; i < C->nx; i++) {
        size_t p = lidx(C, i, j, k);
        C->phi[p] = child_mean(L, L->phi, i, j, k);
        C->rphi[p] = C->phi[p];
        C->src[p] = child_mean(L, L->tmp, i, j, k);
      }
  for (int k = 0; k < C->nz; k++)
    for (int j = 0; j < C->ny; j++)
      for (int i = 0; i < C->nx; i++) {
        size_t p = lidx(C, i, j, k);
        C->src[p] = C->src[p] + apply_A(C, C->phi, i, j, k);
      }
  vcycle(Ls, l + 1, nlev);
  /* correction e = coarse result - R phi, interpolated back */
  size_t nc = (size_t)C->nx * C->ny * C->nz;
  for (size_t p = 0; p < nc; p++) C->rphi[p] = C->phi[p] - C->rphi[p];
  for (int K = 0; K < L->nz; K++)
    for (int J = 0; J < L->ny; J++)
      for (int I = 0; I < L->nx; I++) L->phi[lidx(L, I, J, K)] += tricubic(C, C->rphi, I, J, K);
  rbgs_sweep(L);
  rbgs_sweep(L);
}

static double rms_defect(level_t *L) {
  defect(L);
  size_t n = (size_t)L->nx * L->ny * L->nz;
  double s = 0.0;
  for (size_t p = 0; p < n; p++) s += L->tmp[p] * L->tmp[p];
  return sqrt(s / (double)n);
}

/* level dimensions: halve while every axis is even and stays >= 2 */
int orc_mg_levels(int nx, int ny, int nz, int *dims /* [MG_MAX_LEVELS][3] */) {
  int n = 0;
  for (;;) {
    dims[3 * n] = nx; dims[3 * n + 1] = ny; dims[3 * n + 2] = nz;
    n++;
    if (n == MG_MAX_LEVELS) break;
    if ((nx & 1) || (ny & 1) || (nz & 1) || nx < 4 || ny < 4 || nz < 4) break;
    nx /= 2; ny /= 2; nz /= 2;
  }
  return n;
}

static int build_levels(level_t *Ls, const orc_gmesh *m) {
  int dims[3 * MG_MAX_LEVELS];
  int nlev = orc_mg_levels(m->nx, m->ny, m->nz, dims);
  for (int l = 0; l < nlev; l++) {
    level_t *L = &Ls[l];
    L->nx = dims[3 * l]; L->ny = dims[3 * l + 1]; L->nz = dims[3 * l + 2];
    double s = (double)(1 << l);
    double hx = m->dx[0] * s, hy = m->dx[1] * s, hz = m->dx[2] * s;
    L->hx2 = hx * hx;
    L->wy = (hx / hy) * (hx / hy);
    L->wz = (hx / hz) * (hx / hz);
    L->c0 = 2.0 * (1.0 + L->wy + L->wz);
    size_t n = (size_t)L->nx * L->ny * L->nz;
    L->phi = calloc(n, sizeof(double));
    L->src = calloc(n, sizeof(double));
    L->tmp = calloc(n, sizeof(double));
    L->rphi = calloc(n, sizeof(double));
  }
  return nlev;
}

static void free_levels(level_t *Ls, int nlev) {
  for (int l = 0; l < nlev; l++) { free(Ls[l].phi); free(Ls[l].src); free(Ls[l].tmp); free(Ls[l].rphi); }
}

/*
 * Solve for the potential of the state U (blocks of nv arrays, density first).
 *   phi_global: [nz][ny][nx], in: start (warm != 0), out: solution
 *   phi_blocks: per block (n+2)^3 with one ghost layer (periodic), out (nullable)
 *   cycles: V-cycles run until the RMS defect <= tol or max_cycles
 *   defects: [max_cycles + 1] RMS defect before the first and after each cycle (nullable)
 * Returns the number of V-cycles run, or -1 if the mesh is not periodic.
 */
int orc_mg_solve(const orc_gmesh *m, int nv, const double *U, double four_pi_G, int max_cycles, double tol,
                 int warm, double *phi_global, double *phi_blocks, double *defects) {
  if (m->bc[0] || m->bc[1] || m->bc[2]) return -1;
  level_t Ls[MG_MAX_LEVELS];
  int nlev = build_levels(Ls, m);
  level_t *F = &Ls[0];
  size_t N = (size_t)m->nx * m->ny * m->nz;
  /* gather the density, its mean, and the source */
  double *rho = malloc(N * sizeof(double));
  size_t off = 0;
  for (int b = 0; b < m->nblocks; b++) {
    int n = m->blk[4 * b];
    for (int k = 0; k < n; k++)
      for (int j = 0; j < n; j++)
        for (int i = 0; i < n; i++)
          rho[lidx(F, m->blk[4 * b + 1] + i, m->blk[4 * b + 2] + j, m->blk[4 * b + 3] + k)] =
              U[off + ((size_t)k * n + j) * n + i];
    off += (size_t)nv * n * n * n;
  }
  double sum = 0.0;
  for (size_t p = 0; p < N; p++) sum += rho[p];
  double mean = sum / (double)N;
  for (size_t p = 0; p < N; p++) F->src[p] = -four_pi_G * (rho[p] - mean);
  free(rho);
  /* a second pass removes the rounding residue of the first from the operator's null space */
  double s2 = 0.0;
  for (size_t p = 0; p < N; p++) s2 += F->src[p];
  double mean2 = s2 / (double)N;
  for (size_t p = 0; p < N; p++) F->src[p] -= mean2;
  if (warm) memcpy(F->phi, phi_global, N * sizeof(double));
  double d = rms_defect(F);
  if (defects) defects[0] = d;
  int c = 0;
  while (c < max_cycles && !(d <= tol)) {
    vcycle(Ls, 0, nlev);
    rbgs_sweep(F);
    d = rms_defect(F);
    c++;
    if (defects) defects[c] = d;
  }
  double ps = 0.0;
  for (size_t p = 0; p < N; p++) ps += F->phi[p];
  double pm = ps / (double)N;
  for (size_t p = 0; p < N; p++) F->phi[p] -= pm;
  memcpy(phi_global, F->phi, N * sizeof(double));
  if (phi_blocks) {
    size_t po = 0;
    for (int b = 0; b < m->nblocks; b++) {
      int n = m->blk[4 * b], np = n + 2;
      for (int k = -1; k <= n; k++)
        for (int j = -1; j <= n; j++)
          for (int i = -1; i <= n; i++)
            phi_blocks[po + ((size_t)(k + 1) * np + (j + 1)) * np + (i + 1)] =
                F->phi[lidx(F, m->blk[4 * b + 1] + i, m->blk[4 * b + 2] + j, m->blk[4 * b + 3] + k)];
      po += (size_t)np * np * np;
    }
  }
  free_levels(Ls, nlev);
  return c;
}
