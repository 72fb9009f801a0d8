// gfx950 kernels of the MeshBlock finite-volume update.
//
// One RK stage of one block is a stream of independent cells: each thread
// owns a cell, reads the stage-input conserved state of the 13 cells of its
// PLM stencil (own block or a neighbour, with LAT time interpolation),
// computes the six face fluxes of its cell (PLM -> EOS -> HLLC), the
// flux divergence, gravity sources, the auxiliary-energy compression, floors
// and resynchronisation, and writes the stage output.  All state is FP64
// structure-of-arrays; no work is done on matrix cores here.
//
// Method references (paper sections / equations):
//   RK2, PLM, Riemann solver, floors ........ Table 1
//   conserved -> primitive, dual switch ..... eqs dual-econs, dual-primitive-switch
//   aux flux, face velocity ................. eqs dual-flux, dual-face-velocity
//   compression source ...................... eqs dual-compression-continuous, dual-divv,
//                                             dual-tabulated-compression
//   resynchronisation ....................... eq dual-sync
//   gravity sources ......................... eqs lat-grav-momentum, lat-grav-energy
//   point mass, excision .................... eq bh-softened-gravity
//   tabulated EOS ........................... eqs eos-table-range, eos-table-fields
//   LAT ghosts, impulses, reflux ............ Sec. LAT method; eqs lat-flux-impulse,
//                                             lat-mass-impulse-mismatch, lat-grav-reflux
// HLLC follows Toro (Riemann Solvers and Numerical Methods for Fluid
// Dynamics, 3rd ed., Sec. 10.4) with Davis wave speeds; the limiter is van
// Leer's harmonic mean; RK2 is Heun's method.
#include "tdh_internal.hpp"

namespace tdh {

// ---------------------------------------------------------------------------
// mesh addressing
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap_axis(int g, int N, int bc) {
  // offsets are at most 2 cells and N >= 2
  if (bc == 0) return g < 0 ? g + N : (g >= N ? g - N : g);
  return g < 0 ? 0 : (g >= N ? N - 1 : g);
}

__device__ __forceinline__ int block_of(const MeshDev &m, int gx, int gy, int gz) {
  return m.lmap[((gz / m.lat) * m.ly + gy / m.lat) * m.lx + gx / m.lat];
}

// Where a reader with factor fb finds block nb's conserved state at its stage time.
struct Src {
  const double *A, *B;
  double w;  // value = (1 - w) A + w B; w in {0, 1/2, 1}
};

__device__ __forceinline__ Src source_of(const StageArgs &a, int fb, int nb) {
  const int fn = a.fac[nb];
  const int pn = a.par[nb];
  const double *Qend = pn ? a.Qb : a.Qa;   // latest computed state
  const double *Qold = pn ? a.Qa : a.Qb;   // state at the start of that step
  const bool act = (a.k % fn) == 0;
  Src s;
  if (a.phase == 1) {
    if (act) { s.A = Qend; s.B = Qend; s.w = 0.0; return s; }
    const int t0 = a.k - a.k % fn;
    s.A = Qold; s.B = Qend; s.w = (double)(a.k - t0) / fn;
    return s;
  }
  if (act) {
    if (fn <= fb) { s.A = a.Qs; s.B = a.Qs; s.w = 0.0; return s; }
    s.A = Qend; s.B = a.Qs; s.w = (double)fb / fn;
    return s;
  }
  const int t0 = a.k - a.k % fn;
  s.A = Qold; s.B = Qend; s.w = (double)(a.k + fb - t0) / fn;
  return s;
}

__device__ __forceinline__ double src_val(const Src &s, long long idx) {
  if (s.w == 0.0) return s.A[idx];
  if (s.w == 1.0) return s.B[idx];
  return (1.0 - s.w) * s.A[idx] + s.w * s.B[idx];
}

// ---------------------------------------------------------------------------
// equation of state
// ---------------------------------------------------------------------------
__device__ __forceinline__ double u_floor(const Phys &p, double rho) {
  return p.eos_kind == 0 ? p.p_floor / (p.gamma - 1.0) : rho * p.e_floor;
}

__device__ __forceinline__ void table_rho(const Table &t, double lr, int &i, double &w) {
  const double lrmax = t.lr0 + (t.nrho - 1) * t.dlr;
  lr = fmin(fmax(lr, t.lr0), lrmax);
  const double x = (lr - t.lr0) * t.inv_dlr;
  int ii = (int)floor(x);
  ii = min(max(ii, 0), t.nrho - 2);
  i = ii;
  w = x - ii;
}

__device__ __forceinline__ double tcol(const double *F, int nT, int i, double w, int j) {
  return (1.0 - w) * F[i * nT + j] + w * F[(i + 1) * nT + j];
}

// Table cell of a target log e on the density-interpolated column: the largest
// node j in [0, nT-2] whose value does not exceed the (clamped) target.
// A seed (>= 0) is tried first with secant steps in index space; the result is
// accepted only if it brackets the target, which defines the same j as the
// bisection fallback.  iters = secant steps used, -1 when bisection ran.
__device__ __forceinline__ void table_invert(const Table &t, int i, double w, double le, int seed, int maxit,
                                             int &jout, double &wT, int &iters) {
  const int nT = t.nT;
  const double lo_v = tcol(t.le, nT, i, w, 0), hi_v = tcol(t.le, nT, i, w, nT - 1);
  le = fmin(fmax(le, lo_v), hi_v);
  int j = -1;
  double a = 0.0, b = 1.0;
  iters = -1;
  if (seed >= 0) {
    int jj = min(max(seed, 0), nT - 2);
    for (int it = 0; it <= maxit; ++it) {
      a = tcol(t.le, nT, i, w, jj);
      b = tcol(t.le, nT, i, w, jj + 1);
      if (a <= le && (le < b || jj == nT - 2)) { j = jj; iters = it; break; }
      if (it == maxit) break;
      double s = floor((le - a) / (b - a));
      s = fmin(fmax(s, -(double)nT), (double)nT);
      jj = min(max(jj + (int)s, 0), nT - 2);
    }
  }
  if (j < 0) {
    int lo = 0, hi = nT - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (tcol(t.le, nT, i, w, mid) <= le) lo = mid; else hi = mid;
    }
    j = lo;
    a = tcol(t.le, nT, i, w, j);
    b = tcol(t.le, nT, i, w, j + 1);
  }
  jout = j;
  wT = (le - a) / (b - a);
}

__device__ __forceinline__ double tbil(const double *F, int nT, int i, double w, int j, double wT) {
  return (1.0 - wT) * tcol(F, nT, i, w, j) + wT * tcol(F, nT, i, w, j + 1);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Learned seed: log T from (log rho, log e) by the 2-64-64-1 network, bf16
// operands, fp32 accumulation; returns a table cell index.
__device__ __forceinline__ int seed_cell(const Seed &s, const Table &t, double lr, double le) {
  const float x0 = (float)(2.0 * (lr - s.lr_lo) / (s.lr_hi - s.lr_lo) - 1.0);
  const float x1 = (float)(2.0 * (le - s.le_lo) / (s.le_hi - s.le_lo) - 1.0);
  const float xb0 = bf16_to_f32(f32_to_bf16(x0)), xb1 = bf16_to_f32(f32_to_bf16(x1));
  float h1[64];
#pragma unroll
  for (int o = 0; o < 64; ++o) {
    float z = s.b1[o];
    z += bf16_to_f32(s.w1[2 * o]) * xb0;
    z += bf16_to_f32(s.w1[2 * o + 1]) * xb1;
    h1[o] = bf16_to_f32(f32_to_bf16(fmaxf(z, 0.0f)));
  }
  float y = s.b3[0];
  for (int o = 0; o < 64; ++o) {
    float z = s.b2[o];
#pragma unroll
    for (int q = 0; q < 64; ++q) z += bf16_to_f32(s.w2[o * 64 + q]) * h1[q];
    y += bf16_to_f32(s.w3[o]) * bf16_to_f32(f32_to_bf16(fmaxf(z, 0.0f)));
  }
  const double lT = s.lt_lo + 0.5 * ((double)y + 1.0) * (s.lt_hi - s.lt_lo);
  const double x = (lT - t.lT0) / t.dlT;
  if (!(x > 0.0)) return 0;
  if (x > (double)(t.nT - 2)) return t.nT - 2;
  return (int)x;
}

// (rho, U) -> P, c_s.  jseed: table cell to start from (-1: bisection).
__device__ __forceinline__ void eos_pc(const Phys &p, const Table &t, double rho, double U, int jseed, double &P,
                                       double &cs, int *jout = nullptr) {
  if (p.eos_kind == 0) {
    const double Ue = fmax(U, u_floor(p, rho));
    P = (p.gamma - 1.0) * Ue;
    cs = sqrt(p.gamma * P / rho);
    return;
  }
  const double Ue = fmax(U, rho * p.e_floor);
  int i, j, it;
  double w, wT;
  table_rho(t, log10(rho), i, w);
  table_invert(t, i, w, log10(Ue / rho), jseed, p.newton_max_iter, j, wT, it);
  P = exp10(tbil(t.lP, t.nT, i, w, j, wT));
  cs = exp10(0.5 * tbil(t.lc2, t.nT, i, w, j, wT));
  if (jout) *jout = j;
}

// table cell of the cell-centre state, used to seed the face and compression queries
__device__ __forceinline__ int centre_cell(const Phys &p, const Table &t, const Seed &s, double rho, double U) {
  const double Ue = fmax(U, rho * p.e_floor);
  const double lr = log10(rho), le = log10(Ue / rho);
  int i, j, it;
  double w, wT;
  table_rho(t, lr, i, w);
  const int seed = (p.inv_mode == 1 && s.enabled) ? seed_cell(s, t, lr, le) : -1;
  table_invert(t, i, w, le, seed, p.newton_max_iter, j, wT, it);
  return j;
}

// ---------------------------------------------------------------------------
// cell primitives and the Riemann problem
// ---------------------------------------------------------------------------
__device__ __forceinline__ void c2p(const Phys &p, const double *q, double *w) {
  const double rho = q[IDN];
  const double inv = 1.0 / rho;
  const double K = 0.5 * (q[IM1] * q[IM1] + q[IM2] * q[IM2] + q[IM3] * q[IM3]) * inv;
  const double Uc = q[IEN] - K;
  double Ueos = Uc;
  if (p.dual) {
    if (!(Uc > 0.0 && Uc > p.eta1 * q[IEN])) Ueos = q[IAX];
    w[5] = q[IAX];
  }
  w[0] = rho;
  w[1] = q[IM1] * inv;
  w[2] = q[IM2] * inv;
  w[3] = q[IM3] * inv;
  w[4] = Ueos;
}

__device__ __forceinline__ double vanleer(double dm, double dp) {
  const double pr = dm * dp;
  return pr > 0.0 ? 2.0 * pr / (dm + dp) : 0.0;
}

// rotated states (rho, un, ut1, ut2, U[, A]) -> HLLC flux (rho, mn, mt1, mt2, E)
__device__ __forceinline__ void hllc(const double *wl, double pl, double cl, const double *wr, double pr, double cr,
                                     double *f) {
  const double rl = wl[0], ul = wl[1], vl = wl[2], zl = wl[3];
  const double rr = wr[0], ur = wr[1], vr = wr[2], zr = wr[3];
  const double El = wl[4] + 0.5 * rl * (ul * ul + vl * vl + zl * zl);
  const double Er = wr[4] + 0.5 * rr * (ur * ur + vr * vr + zr * zr);
  const double sl = fmin(ul - cl, ur - cr);
  const double sr = fmax(ul + cl, ur + cr);
  if (sl >= 0.0) {
    f[0] = rl * ul; f[1] = rl * ul * ul + pl; f[2] = rl * ul * vl; f[3] = rl * ul * zl; f[4] = (El + pl) * ul;
    return;
  }
  if (sr <= 0.0) {
    f[0] = rr * ur; f[1] = rr * ur * ur + pr; f[2] = rr * ur * vr; f[3] = rr * ur * zr; f[4] = (Er + pr) * ur;
    return;
  }
  const double sm = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) / (rl * (sl - ul) - rr * (sr - ur));
  // both star states share one code path: pick the side first
  const bool left = sm >= 0.0;
  const double r = left ? rl : rr, u = left ? ul : ur, v = left ? vl : vr, z = left ? zl : zr;
  const double E = left ? El : Er, P = left ? pl : pr, s = left ? sl : sr;
  const double a = r * (s - u) / (s - sm);
  const double us4 = a * (E / r + (sm - u) * (sm + P / (r * (s - u))));
  const double f0 = r * u, f1 = r * u * u + P, f2 = r * u * v, f3 = r * u * z, f4 = (E + P) * u;
  f[0] = f0 + s * (a - r);
  f[1] = f1 + s * (a * sm - r * u);
  f[2] = f2 + s * (a * v - r * v);
  f[3] = f3 + s * (a * z - r * z);
  f[4] = f4 + s * (us4 - E);
}

// ---------------------------------------------------------------------------
// gravity / excision geometry
// ---------------------------------------------------------------------------
__device__ __forceinline__ double cell_x(const MeshDev &m, int d, int g) { return m.x0[d] + (g + 0.5) * m.dx[d]; }

__device__ __forceinline__ double phi_point(const Phys &p, const MeshDev &m, int gx, int gy, int gz, double t) {
  const double dx = cell_x(m, 0, gx) - (p.bh_x0[0] - p.v_frame[0] * t);
  const double dy = cell_x(m, 1, gy) - (p.bh_x0[1] - p.v_frame[1] * t);
  const double dz = cell_x(m, 2, gz) - (p.bh_x0[2] - p.v_frame[2] * t);
  return -p.gm_bh / sqrt(dx * dx + dy * dy + dz * dz + p.r_soft * p.r_soft);
}

__device__ __forceinline__ bool excised(const Phys &p, const MeshDev &m, int gx, int gy, int gz, double t) {
  if (p.grav_kind != 2 || !(p.r_exc > 0.0)) return false;
  const double dx = cell_x(m, 0, gx) - (p.bh_x0[0] - p.v_frame[0] * t);
  const double dy = cell_x(m, 1, gy) - (p.bh_x0[1] - p.v_frame[1] * t);
  const double dz = cell_x(m, 2, gz) - (p.bh_x0[2] - p.v_frame[2] * t);
  return dx * dx + dy * dy + dz * dz < p.r_exc * p.r_exc;
}

// potential at local offset (i,j,k) in [-1, n] of block B
__device__ __forceinline__ double phi_at(const StageArgs &a, const BlockInfo &B, int i, int j, int k, double t) {
  if (a.p.grav_kind == 1) {
    const int np = B.n + 2;
    return a.phi[B.poff + ((long long)(k + 1) * np + (j + 1)) * np + (i + 1)];
  }
  return phi_point(a.p, a.m, B.ox + i, B.oy + j, B.oz + k, t);
}

// ---------------------------------------------------------------------------
// stage kernel
// ---------------------------------------------------------------------------
struct Nbr {
  int blk;       // owning block of the cell across a face (-1: beyond an outflow edge)
  long long idx; // its local cell index
  int u0, u1;    // its face-cell coordinates (transverse, increasing axis order)
};

// load conserved state of global cell g (stage view of the reader), return block info
__device__ __forceinline__ void load_q(const StageArgs &a, int b, const BlockInfo &B, const Src &own, int fb,
                                       int gx, int gy, int gz, double *q, int *nb_out, long long *idx_out) {
  const MeshDev &m = a.m;
  gx = wrap_axis(gx, m.nx, m.bc[0]);
  gy = wrap_axis(gy, m.ny, m.bc[1]);
  gz = wrap_axis(gz, m.nz, m.bc[2]);
  const int lx = gx - B.ox, ly = gy - B.oy, lz = gz - B.oz;
  const int nv = m.nv;
  if ((unsigned)lx < (unsigned)B.n && (unsigned)ly < (unsigned)B.n && (unsigned)lz < (unsigned)B.n) {
    const long long n3 = (long long)B.n * B.n * B.n;
    const long long idx = ((long long)lz * B.n + ly) * B.n + lx;
    for (int v = 0; v < nv; ++v) q[v] = src_val(own, B.off + v * n3 + idx);
    if (nb_out) { *nb_out = b; *idx_out = idx; }
    return;
  }
  const int nb = block_of(m, gx, gy, gz);
  const BlockInfo Bn = m.blocks[nb];
  const Src s = source_of(a, fb, nb);
  const long long n3 = (long long)Bn.n * Bn.n * Bn.n;
  const long long idx = ((long long)(gz - Bn.oz) * Bn.n + (gy - Bn.oy)) * Bn.n + (gx - Bn.ox);
  for (int v = 0; v < nv; ++v) q[v] = src_val(s, Bn.off + v * n3 + idx);
  if (nb_out) { *nb_out = nb; *idx_out = idx; }
}

// flux through the face between stencil cells 1 and 2 of w[0..3] (rotated primitives)
__device__ __forceinline__ void face_flux(const Phys &p, const Table &t, int nv, const double (*w)[6], int jseed,
                                          double *f, double &vf) {
  double wl[6], wr[6];
#pragma unroll
  for (int v = 0; v < 6; ++v) {
    if (v >= nv) break;
    const double q0 = w[0][v], q1 = w[1][v], q2 = w[2][v], q3 = w[3][v];
    wl[v] = q1 + 0.5 * vanleer(q1 - q0, q2 - q1);
    wr[v] = q2 - 0.5 * vanleer(q2 - q1, q3 - q2);
  }
  double pl, cl, pr, cr;
  eos_pc(p, t, wl[0], wl[4], jseed, pl, cl);
  eos_pc(p, t, wr[0], wr[4], jseed, pr, cr);
  hllc(wl, pl, cl, wr, pr, cr, f);
  const double *wu = f[0] >= 0.0 ? wl : wr;
  f[5] = p.dual ? f[0] * (wu[5] / wu[0]) : 0.0;
  vf = f[0] / wu[0];
}

__global__ __launch_bounds__(kChunk) void stage_kernel(StageArgs a) {
  const int a0 = a.cnt_ge[a.Lhi + 1], a1 = a.cnt_ge[a.Llo];
  if (a1 <= a0) return;
  const int i0 = a.item_start[a0], i1 = a.item_start[a1];
  const Phys &p = a.p;
  const MeshDev &m = a.m;
  const int nv = m.nv;
  for (int item = i0 + (int)blockIdx.x; item < i1; item += (int)gridDim.x) {
    int lo = a0, hi = a1;  // item_start[lo] <= item < item_start[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.item_start[mid] <= item) lo = mid; else hi = mid;
    }
    const int b = a.order[lo];
    const BlockInfo B = m.blocks[b];
    const int n = B.n;
    const long long n3 = (long long)n * n * n;
    const long long cell = (long long)(item - a.item_start[lo]) * kChunk + threadIdx.x;
    if (cell >= n3) continue;
    const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
    const int g[3] = {B.ox + ci, B.oy + cj, B.oz + ck};
    const int lc[3] = {ci, cj, ck};
    const int fb = a.fac[b];
    const double dt0 = a.win[1];
    const double tk = a.win[0] + a.k * dt0;
    const double dtb = fb * dt0;
    const double t = a.phase == 1 ? tk : tk + dtb;
    const Src own = source_of(a, fb, b);
    double qc[6], wc[6];
    for (int v = 0; v < nv; ++v) qc[v] = src_val(own, B.off + v * n3 + cell);
    c2p(p, qc, wc);
    const int jseed = (p.eos_kind == 1 && p.inv_mode != 0) ? centre_cell(p, a.t, a.s, wc[0], wc[4]) : -1;
    const bool exc_on = p.grav_kind == 2 && p.r_exc > 0.0;
    const bool exc_c = exc_on && excised(p, m, g[0], g[1], g[2], t);
    double rhs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double divv = 0.0;
    double emax = qc[IEN];
    const int N[3] = {m.nx, m.ny, m.nz};
    for (int d = 0; d < 3; ++d) {
      const int pn = 1 + d, p1 = 1 + (d + 1) % 3, p2 = 1 + (d + 2) % 3;
      double W[5][6];
      int nbk[2] = {b, b};
      long long nidx[2] = {0, 0};
      bool inside[2] = {true, true};
      for (int s = 0; s < 5; ++s) {
        double q[6], w[6];
        if (s == 2) {
          for (int v = 0; v < nv; ++v) w[v] = wc[v];
        } else {
          int gg[3] = {g[0], g[1], g[2]};
          gg[d] += s - 2;
          int nb_;
          long long id_;
          load_q(a, b, B, own, fb, gg[0], gg[1], gg[2], q, &nb_, &id_);
          c2p(p, q, w);
          if (s == 1 || s == 3) {
            const int side = s == 3;
            if (q[IEN] > emax) emax = q[IEN];
            nbk[side] = nb_;
            nidx[side] = id_;
            inside[side] = m.bc[d] == 0 || (gg[d] >= 0 && gg[d] < N[d]);
          }
        }
        W[s][0] = w[0]; W[s][1] = w[pn]; W[s][2] = w[p1]; W[s][3] = w[p2]; W[s][4] = w[4];
        if (nv > 5) W[s][5] = w[5];
      }
      double F[2][6], vf[2];
      face_flux(p, a.t, nv, W, jseed, F[0], vf[0]);
      face_flux(p, a.t, nv, W + 1, jseed, F[1], vf[1]);
      // excision: a face between an active and an excised cell keeps its flux
      // unless the mass flux leaves the sink
      if (exc_on) {
        for (int side = 0; side < 2; ++side) {
          int gg[3] = {g[0], g[1], g[2]};
          gg[d] += side ? 1 : -1;
          const bool eo = excised(p, m, gg[0], gg[1], gg[2], t);
          if (eo != exc_c) {
            const bool right_exc = side ? eo : exc_c;  // is the cell on the + side excised
            const bool into = right_exc ? (F[side][0] >= 0.0) : (F[side][0] <= 0.0);
            if (!into) {
              for (int v = 0; v < 6; ++v) F[side][v] = 0.0;
              vf[side] = 0.0;
            }
          }
        }
      }
      // back to (rho, mx, my, mz, E, A)
      double G[2][6];
      for (int side = 0; side < 2; ++side) {
        G[side][IDN] = F[side][0];
        G[side][pn] = F[side][1];
        G[side][p1] = F[side][2];
        G[side][p2] = F[side][3];
        G[side][IEN] = F[side][4];
        G[side][IAX] = F[side][5];
      }
      const double idx = m.inv_dx[d];
      for (int v = 0; v < nv; ++v) rhs[v] -= (G[1][v] - G[0][v]) * idx;
      divv += (vf[1] - vf[0]) * idx;
      if (p.grav_kind) {
        int im[3] = {ci, cj, ck}, ip[3] = {ci, cj, ck};
        im[d] -= 1;
        ip[d] += 1;
        const double pm = phi_at(a, B, im[0], im[1], im[2], t);
        const double p0 = phi_at(a, B, ci, cj, ck, t);
        const double pp = phi_at(a, B, ip[0], ip[1], ip[2], t);
        rhs[pn] -= qc[IDN] * (pp - pm) / (2.0 * m.dx[d]);
        rhs[IEN] -= (G[1][IDN] * (pp - p0) + G[0][IDN] * (p0 - pm)) / (2.0 * m.dx[d]);
      }
      // boundary faces: stage-1 flux, then the time-integrated impulse
      for (int side = 0; side < 2; ++side) {
        if (lc[d] != (side ? n - 1 : 0)) continue;
        const int u0 = d == 0 ? cj : ci;
        const int u1 = d == 2 ? cj : ck;
        const long long base = B.ioff + (long long)(2 * d + side) * nv * n * n + (long long)u1 * n + u0;
        if (a.phase == 1) {
          for (int v = 0; v < nv; ++v) a.bf1[base + (long long)v * n * n] = G[side][v];
        } else if (inside[side]) {
          const double area = m.dx[(d + 1) % 3] * m.dx[(d + 2) % 3];
          const int fn = a.fac[nbk[side]];
          const int fw = fb > fn ? fb : fn;
          const bool overwrite = (a.k % fw) == 0;
          for (int v = 0; v < nv; ++v) {
            const long long ix = base + (long long)v * n * n;
            const double Is = 0.5 * (a.bf1[ix] + G[side][v]) * area * dtb;
            a.imp[ix] = overwrite ? Is : a.imp[ix] + Is;
          }
        }
      }
    }
    // combine
    const double *Qbase = a.par[b] ? a.Qb : a.Qa;
    double qn[6];
    for (int v = 0; v < nv; ++v) {
      const double qs = qc[v] + dtb * rhs[v];
      qn[v] = a.phase == 1 ? qs : 0.5 * Qbase[B.off + v * n3 + cell] + 0.5 * qs;
    }
    if (p.dual) {
      const double tau = a.phase == 1 ? dtb : 0.5 * dtb;
      if (p.eos_kind == 0) {
        qn[IAX] = qn[IAX] * exp(-(p.gamma - 1.0) * divv * tau);
      } else {
        double Pa, ca;
        eos_pc(p, a.t, qc[IDN], qn[IAX], jseed, Pa, ca);
        qn[IAX] = qn[IAX] - Pa * divv * tau;
      }
      const double uf = u_floor(p, qn[IDN] > p.rho_floor ? qn[IDN] : p.rho_floor);
      if (qn[IAX] < uf) qn[IAX] = uf;
    }
    if (qn[IDN] < p.rho_floor) qn[IDN] = p.rho_floor;
    {
      double w[6];
      c2p(p, qn, w);
      const double uf = u_floor(p, qn[IDN]);
      if (w[4] < uf) {
        qn[IEN] += uf - w[4];
        if (p.dual && qn[IAX] < uf) qn[IAX] = uf;
      }
    }
    if (p.dual) {
      const double K = 0.5 * (qn[IM1] * qn[IM1] + qn[IM2] * qn[IM2] + qn[IM3] * qn[IM3]) / qn[IDN];
      const double Uc = qn[IEN] - K;
      if (Uc > 0.0 && Uc > p.eta2 * emax) qn[IAX] = Uc;
    }
    if (a.phase == 2 && exc_on && excised(p, m, g[0], g[1], g[2], tk + dtb)) {
      const double uf = u_floor(p, p.rho_floor);
      qn[IDN] = p.rho_floor;
      qn[IM1] = qn[IM2] = qn[IM3] = 0.0;
      qn[IEN] = uf;
      if (p.dual) qn[IAX] = uf;
    }
    double *out = a.phase == 1 ? a.Qs : (a.par[b] ? a.Qa : a.Qb);
    for (int v = 0; v < nv; ++v) out[B.off + v * n3 + cell] = qn[v];
  }
}

__global__ void set_window_kernel(double *win, double t, double dt0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    win[0] = t;
    win[1] = dt0;
  }
}

__global__ void commit_kernel(const int *order, const int *cnt_ge, int lmin, int *par) {
  const int na = cnt_ge[lmin];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += gridDim.x * blockDim.x) par[order[i]] ^= 1;
}

// Delayed flux correction for blocks completing now against finer neighbours
// (eqs lat-mass-impulse-mismatch, lat-grav-reflux); one launch per axis so a
// cell touched by several faces is corrected in axis order without races.
__global__ void reflux_kernel(StageArgs a, int lc, int dir, int nmax) {
  const MeshDev &m = a.m;
  const int nv = m.nv;
  const int nc = a.cnt_ge[lc];
  const long long per = 2LL * nmax * nmax;
  const long long total = (long long)nc * per;
  const int N[3] = {m.nx, m.ny, m.nz};
  const double vol = m.dx[0] * m.dx[1] * m.dx[2];
  const double tc = a.win[0] + a.k * a.win[1];  // completion time
  for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (long long)gridDim.x * blockDim.x) {
    const int ai = (int)(it / per);
    const long long rem = it % per;
    const int side = (int)(rem / ((long long)nmax * nmax));
    const int uu = (int)(rem % ((long long)nmax * nmax));
    const int b = a.order[ai];
    const BlockInfo B = m.blocks[b];
    const int n = B.n;
    const int u0 = uu % nmax, u1 = uu / nmax;
    if (u0 >= n || u1 >= n) continue;
    int loc[3];
    if (dir == 0) { loc[1] = u0; loc[2] = u1; }
    if (dir == 1) { loc[0] = u0; loc[2] = u1; }
    if (dir == 2) { loc[0] = u0; loc[1] = u1; }
    loc[dir] = side ? n - 1 : 0;
    int gg[3] = {B.ox + loc[0], B.oy + loc[1], B.oz + loc[2]};
    gg[dir] += side ? 1 : -1;
    if (m.bc[dir] != 0 && (gg[dir] < 0 || gg[dir] >= N[dir])) continue;
    gg[0] = wrap_axis(gg[0], m.nx, m.bc[0]);
    gg[1] = wrap_axis(gg[1], m.ny, m.bc[1]);
    gg[2] = wrap_axis(gg[2], m.nz, m.bc[2]);
    const int nb = block_of(m, gg[0], gg[1], gg[2]);
    if (a.fac[nb] >= a.fac[b]) continue;
    const BlockInfo Bn = m.blocks[nb];
    const int ln[3] = {gg[0] - Bn.ox, gg[1] - Bn.oy, gg[2] - Bn.oz};
    const int v0 = dir == 0 ? ln[1] : ln[0];
    const int v1 = dir == 2 ? ln[1] : ln[2];
    const int nn = Bn.n;
    double dI[6];
    for (int v = 0; v < nv; ++v) {
      const long long ib = B.ioff + ((long long)(2 * dir + side) * nv + v) * n * n + (long long)u1 * n + u0;
      const long long in = Bn.ioff + ((long long)(2 * dir + 1 - side) * nv + v) * nn * nn + (long long)v1 * nn + v0;
      dI[v] = a.imp[ib] - a.imp[in];
    }
    const double sg = side ? 1.0 : -1.0;
    double *q = a.par[b] ? a.Qb : a.Qa;
    const long long n3 = (long long)n * n * n;
    const long long cidx = ((long long)loc[2] * n + loc[1]) * n + loc[0];
    if (a.p.grav_kind) {
      int lnb[3] = {loc[0], loc[1], loc[2]};
      lnb[dir] += side ? 1 : -1;
      const double pn = phi_at(a, B, lnb[0], lnb[1], lnb[2], tc);
      const double pi = phi_at(a, B, loc[0], loc[1], loc[2], tc);
      q[B.off + IEN * n3 + cidx] += sg / (2.0 * vol) * dI[IDN] * (pn - pi);
    }
    for (int v = 0; v < nv; ++v) q[B.off + v * n3 + cidx] += sg * dI[v] / vol;
  }
}

// ---------------------------------------------------------------------------
// CFL step: per-item minimum, then per-block minimum
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ __launch_bounds__(kChunk) void cfl_items_kernel(StageArgs a, double t, const int *item_block,
                                                           const int *block_item_start, int nitems, double *part) {
  __shared__ double red[kChunk / 64];
  const MeshDev &m = a.m;
  const Phys &p = a.p;
  const int nv = m.nv;
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int b = item_block[item];
    const BlockInfo B = m.blocks[b];
    const int n = B.n;
    const long long n3 = (long long)n * n * n;
    const long long cell = (long long)(item - block_item_start[b]) * kChunk + threadIdx.x;
    double best = INFINITY;
    if (cell < n3) {
      const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
      const bool exc = p.grav_kind == 2 && p.r_exc > 0.0 && excised(p, m, B.ox + ci, B.oy + cj, B.oz + ck, t);
      if (!exc) {
        const double *Q = a.par[b] ? a.Qb : a.Qa;
        double q[6], w[6];
        for (int v = 0; v < nv; ++v) q[v] = Q[B.off + v * n3 + cell];
        c2p(p, q, w);
        double P, cs;
        int seed = -1;
        if (p.eos_kind == 1 && p.inv_mode == 1 && a.s.enabled) {
          const double Ue = fmax(w[4], w[0] * p.e_floor);
          seed = seed_cell(a.s, a.t, log10(w[0]), log10(Ue / w[0]));
        }
        eos_pc(p, a.t, w[0], w[4], seed, P, cs);
        for (int d = 0; d < 3; ++d) best = fmin(best, m.dx[d] / (fabs(w[1 + d]) + cs));
      }
    }
    best = wave_min(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = red[0];
      for (int i = 1; i < kChunk / 64; ++i) r = fmin(r, red[i]);
      part[item] = r;
    }
    __syncthreads();
  }
}

__global__ void cfl_blocks_kernel(const double *part, const int *block_item_start, int nblocks, double cfl,
                                  double *dtb) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nblocks; b += gridDim.x * blockDim.x) {
    double r = INFINITY;
    for (int i = block_item_start[b]; i < block_item_start[b + 1]; ++i) r = fmin(r, part[i]);
    dtb[b] = cfl * r;
  }
}

// ---------------------------------------------------------------------------
// batched EOS queries
// ---------------------------------------------------------------------------
__global__ void eos_invert_kernel(Table t, Seed s, int maxit, const double *lr, const double *le, double *lT,
                                  int32_t *jo, int32_t *iters, long long n, int mode) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    int i, j, it;
    double w, wT;
    table_rho(t, lr[q], i, w);
    int seed = -1;
    if (mode == 1 && s.enabled) seed = seed_cell(s, t, lr[q], le[q]);
    if (mode == 2) {
      // bisection result as the seed: the secant loop accepts it at once
      int jj;
      double ww;
      int it2;
      table_invert(t, i, w, le[q], -1, 0, jj, ww, it2);
      seed = jj;
    }
    table_invert(t, i, w, le[q], seed, maxit, j, wT, it);
    if (lT) lT[q] = t.lT0 + (j + wT) * t.dlT;
    if (jo) jo[q] = j;
    if (iters) iters[q] = it;
  }
}

__global__ void eos_eval_kernel(Phys p, Table t, const double *rho, const double *U, double *P, double *cs,
                                long long n) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    double pp, cc;
    eos_pc(p, t, rho[q], U[q], -1, pp, cc);
    P[q] = pp;
    cs[q] = cc;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_stage(const StageArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(stage_kernel, dim3(grid), dim3(kChunk), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_set_window(double *win, double t, double dt0, hipStream_t s) {
  hipLaunchKernelGGL(set_window_kernel, dim3(1), dim3(64), 0, s, win, t, dt0);
  return hipGetLastError();
}

hipError_t launch_commit(const int *order, const int *cnt_ge, int lmin, int *par, hipStream_t s) {
  hipLaunchKernelGGL(commit_kernel, dim3(64), dim3(256), 0, s, order, cnt_ge, lmin, par);
  return hipGetLastError();
}

hipError_t launch_reflux(const StageArgs &a, int lc, int dir, int nmax, int grid, hipStream_t s) {
  hipLaunchKernelGGL(reflux_kernel, dim3(grid), dim3(256), 0, s, a, lc, dir, nmax);
  return hipGetLastError();
}

hipError_t launch_cfl(const StageArgs &a, double cfl, double t, const int *item_block, int nitems, double *part,
                      int nblocks, const int *block_item_start, double *dtb, hipStream_t s) {
  const int grid = nitems < 4096 ? nitems : 4096;
  hipLaunchKernelGGL(cfl_items_kernel, dim3(grid), dim3(kChunk), 0, s, a, t, item_block, block_item_start, nitems,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cfl_blocks_kernel, dim3((nblocks + 255) / 256), dim3(256), 0, s, part, block_item_start,
                     nblocks, cfl, dtb);
  return hipGetLastError();
}

hipError_t launch_eos_invert(const Table &t, const Seed &sd, int maxit, const double *lr, const double *le,
                             double *lT, int32_t *j, int32_t *iters, int64_t n, int mode, hipStream_t st) {
  const long long blocks = (n + 255) / 256;
  const int grid = blocks < 16384 ? (int)blocks : 16384;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(eos_invert_kernel, dim3(grid), dim3(256), 0, st, t, sd, maxit, lr, le, lT, j, iters,
                     (long long)n, mode);
  return hipGetLastError();
}

hipError_t launch_eos_eval(const Phys &p, const Table &t, const double *rho, const double *U, double *P, double *cs,
                           int64_t n, hipStream_t st) {
  const long long blocks = (n + 255) / 256;
  const int grid = blocks < 16384 ? (int)blocks : 16384;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(eos_eval_kernel, dim3(grid), dim3(256), 0, st, p, t, rho, U, P, cs, (long long)n);
  return hipGetLastError();
}

}  // namespace tdh
