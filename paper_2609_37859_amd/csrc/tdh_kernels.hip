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
#include "tdh_mlp_dev.hpp"

#include <mutex>
#include <unordered_map>

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
  return m.lmap[((gz >> m.lat_shift) * m.ly + (gy >> m.lat_shift)) * m.lx + (gx >> m.lat_shift)];
}

// block covering global cell (gx, gy, gz) of refinement level r (inside the
// level's extents); its own level may be r, r + 1 or r - 1
__device__ __forceinline__ int block_of(const MeshDev &m, int r, int gx, int gy, int gz) {
  const int sh = m.lat_shift + r;
  return m.lmap[((gz >> sh) * m.ly + (gy >> sh)) * m.lx + (gx >> sh)];
}

// Physics switches of the stage path.  PK = 0 reads them from Phys at run time;
// PK = kPkAmr reads them at run time too and adds ghosts across refinement
// levels (the only kernels that take meshes with a refined block); otherwise
// they are fixed at compile time, PK = physics_code(p), so the compiler drops
// the other paths and the registers they would hold.  multi = 0 marks a window
// without levels: every neighbour is on the reader's schedule, so ghosts need
// no time interpolation and faces no impulses.
__host__ __device__ constexpr int physics_code(int eos, int dual, int grav, int riemann, int dense, int multi,
                                               int amr = 0) {
  return 1 + eos + 2 * dual + 4 * grav + 16 * riemann + 32 * dense + 64 * multi + 128 * amr;
}
constexpr int kPkAmr = -1;
template <int PK> __device__ __forceinline__ int k_eos(const Phys &p) { return PK > 0 ? (PK - 1) & 1 : p.eos_kind; }
template <int PK> __device__ __forceinline__ int k_dual(const Phys &p) { return PK > 0 ? ((PK - 1) >> 1) & 1 : p.dual; }
template <int PK> __device__ __forceinline__ int k_grav(const Phys &p) { return PK > 0 ? ((PK - 1) >> 2) & 3 : p.grav_kind; }
template <int PK> __device__ __forceinline__ int k_riemann(const Phys &p) { return PK > 0 ? ((PK - 1) >> 4) & 1 : p.riemann; }
template <int PK> __device__ __forceinline__ int k_dense(const Phys &p) { return PK > 0 ? ((PK - 1) >> 5) & 1 : p.ghost_dense; }
template <int PK> __host__ __device__ constexpr bool k_multi() { return PK > 0 ? ((PK - 1) >> 6) & 1 : true; }
// ghosts across refinement levels (kPkAmr and the compiled kinds with the amr
// bit; every other kind assumes one level)
template <int PK> __host__ __device__ constexpr bool k_amr() { return PK == kPkAmr || (PK > 0 && (((PK - 1) >> 7) & 1)); }
template <int PK> __device__ __forceinline__ int lev_of(const BlockInfo &B) { return k_amr<PK>() ? B.lev : 0; }
// cell width and its inverse along d on refinement level r (exact: powers of two)
__device__ __forceinline__ double dx_lev(const MeshDev &m, int d, int r) { return r ? 0.5 * m.dx[d] : m.dx[d]; }
__device__ __forceinline__ double inv_dx_lev(const MeshDev &m, int d, int r) { return r ? 2.0 * m.inv_dx[d] : m.inv_dx[d]; }
// compiled point-mass kinds keep each staged cell's potential and excision
// flag in LDS: every cell's value serves its own and its neighbours' terms
// (a stored potential is one cached load, not worth the LDS)
template <int PK> __host__ __device__ constexpr bool k_gcache() { return PK > 0 && (((PK - 1) >> 2) & 3) == 2; }

// The stage kernel's arguments read again from the kernel-argument segment
// (scalar loads) at the start of each work item: the pointer passes through an
// empty volatile asm, so loads through it can neither be hoisted above that
// point nor merged with earlier ones.  It bounds the live ranges of the many
// uniform fields, which the scalar register file cannot hold for the whole
// kernel (the compiler would park them in vector-register lanes and restore
// them a lane at a time: on the point-mass kind 1176 such restores in the
// code, 55 with the re-read).  Valid in kernels whose one argument is the
// StageArgs, passed by value, first.
__device__ __forceinline__ const StageArgs &kargs() {
  auto p = (const __attribute__((address_space(4))) StageArgs *)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *(const StageArgs *)p;
}

// Where a reader with factor fb finds block nb's conserved state at its stage time.
struct Src {
  const double *A, *B;
  const double *C;  // stage-1 state of a neighbour mid-step (dense output), else null
  double w;         // value = (1 - w) A + w B, w in [0, 1]; with C the RK2 dense output at w
};

template <int PK = 0>
__device__ __forceinline__ Src source_of(const StageArgs &a, int fb, int nb) {
  if constexpr (!k_multi<PK>()) {  // one schedule: the neighbour's stage input, as the reader's own
    Src s;
    s.A = a.phase == 1 ? (a.par[nb] ? a.Qb : a.Qa) : a.Qs;
    s.B = s.A;
    s.C = nullptr;
    s.w = 0.0;
    return s;
  }
  const int fn = a.fac[nb];
  const int pn = a.par[nb];
  const double *Qend = pn ? a.Qb : a.Qa;   // latest computed state
  const double *Qold = pn ? a.Qa : a.Qb;   // state at the start of that step
  const bool act = (a.k & (fn - 1)) == 0;  // factors are powers of two
  Src s;
  s.C = nullptr;
  if (a.phase == 1) {
    if (act) { s.A = Qend; s.B = Qend; s.w = 0.0; return s; }
    // mid-step: start, stage-1 and end states of its step are stored
    const int t0 = a.k & ~(fn - 1);
    s.A = Qold; s.B = Qend; s.w = (double)(a.k - t0) / fn;
    if (k_dense<PK>(a.p)) s.C = a.Qs;
    return s;
  }
  if (act) {
    if (fn <= fb) { s.A = a.Qs; s.B = a.Qs; s.w = 0.0; return s; }
    s.A = Qend; s.B = a.Qs; s.w = (double)fb / fn;
    return s;
  }
  const int t0 = a.k & ~(fn - 1);
  s.A = Qold; s.B = Qend; s.w = (double)(a.k + fb - t0) / fn;
  if (k_dense<PK>(a.p)) s.C = a.Qs;
  return s;
}

// The stage-input state of a block that is active in this sub-cycle (its own
// cells): source_of's active case, with no interpolation.
__device__ __forceinline__ Src own_source(const StageArgs &a, int par) {
  Src s;
  s.A = a.phase == 1 ? (par ? a.Qb : a.Qa) : a.Qs;
  s.B = s.A;
  s.C = nullptr;
  s.w = 0.0;
  return s;
}

// With C: Heun's dense output (weights th - th^2/2 and th^2/2 on the stage
// slopes) in stored states, (1 - w) Qn + w (1 - w) Q1 + w^2 Q_{n+1}: second
// order in time, and a convex combination, so admissible states stay admissible.
__device__ __forceinline__ double src_val(const Src &s, long long idx) {
  if (s.w == 0.0) return s.A[idx];
  if (s.C) {
#pragma clang fp contract(off)
    return (1.0 - s.w) * s.A[idx] + s.w * (1.0 - s.w) * s.C[idx] + s.w * s.w * s.B[idx];
  }
  if (s.w == 1.0) return s.B[idx];
  return (1.0 - s.w) * s.A[idx] + s.w * s.B[idx];
}

// ---------------------------------------------------------------------------
// equation of state
// ---------------------------------------------------------------------------
template <int PK = 0>
__device__ __forceinline__ double u_floor(const Phys &p, double rho) {
  return k_eos<PK>(p) == 0 ? p.p_floor / (p.gamma - 1.0) : rho * p.e_floor;
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

// (1 - w) x + w y with both products and the sum rounded separately (no fused
// multiply-add): one rounding pattern for every table interpolation, so the
// record and node paths agree bit for bit, and the same pattern as the plain
// definition.  Some low-density cells near a point mass amplify the rounding
// of the EOS; a fused form moves them by ~1e-11 relative.
__device__ __forceinline__ double tlerp(double w, double x, double y) {
#pragma clang fp contract(off)
  return (1.0 - w) * x + w * y;
}

// log e of column j interpolated between density rows i and i+1 (one 16-byte load)
__device__ __forceinline__ double tcol_le(const Table &t, int i, double w, int j) {
  const double2 v = t.le2[i * t.nT + j];
  return tlerp(w, v.x, v.y);
}

// Table cell of a target log e on the density-interpolated column: the largest
// node j in [0, nT-2] whose value does not exceed the (clamped) target.
// A seed (>= 0) is tried first with secant steps in index space; the result is
// accepted only if it brackets the target, which defines the same j as the
// bisection fallback.  iters = secant steps used, -1 when bisection ran.
__device__ __forceinline__ void table_invert(const Table &t, int i, double w, double le, int seed, int maxit,
                                             int &jout, double &wT, int &iters) {
  const int nT = t.nT;
  const double lo_v = tcol_le(t, i, w, 0), hi_v = tcol_le(t, i, w, nT - 1);
  le = fmin(fmax(le, lo_v), hi_v);
  int j = -1;
  double a = 0.0, b = 1.0;
  iters = -1;
  if (seed >= 0) {
    int jj = min(max(seed, 0), nT - 2);
    for (int it = 0; it <= maxit; ++it) {
      a = tcol_le(t, i, w, jj);
      b = tcol_le(t, i, w, jj + 1);
      if (a <= le && (le < b || jj == nT - 2)) { j = jj; iters = it; break; }
      if (it == maxit) break;
      double s = floor((le - a) / (b - a));
      s = fmin(fmax(s, -(double)nT), (double)nT);
      jj = min(max(jj + (int)s, 0), nT - 2);
    }
  }
  if (j < 0) {
    int lo = 0, hi = nT - 1;
    double vlo = lo_v, vhi = hi_v;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      const double vm = tcol_le(t, i, w, mid);
      if (vm <= le) { lo = mid; vlo = vm; } else { hi = mid; vhi = vm; }
    }
    j = lo;
    a = vlo;
    b = hi == lo + 1 ? vhi : tcol_le(t, i, w, j + 1);
  }
  jout = j;
  wT = (le - a) / (b - a);
}

// log P and log c_s^2 at (w, wT) in cell (i, j): two 32-byte loads, each
// holding both density rows of both fields at one T node
__device__ __forceinline__ void tbil_pc(const Table &t, int i, double w, int j, double wT, double &lP, double &lc2) {
  const double4 v0 = t.pc[i * t.nT + j], v1 = t.pc[i * t.nT + j + 1];
  lP = tlerp(wT, tlerp(w, v0.x, v0.y), tlerp(w, v1.x, v1.y));
  lc2 = tlerp(wT, tlerp(w, v0.z, v0.w), tlerp(w, v1.z, v1.w));
}

// Seeded query from the seed cell's record alone: true (and j, wT, lP, lc2)
// when cell jj brackets the target exactly as table_invert would accept it
// (the clamp of an out-of-range target only matters in the edge cells).
__device__ __forceinline__ bool table_record(const Table &t, int i, double w, double le, int jj, double &wT,
                                             double &lP, double &lc2) {
  const double4 *R = (const double4 *)(t.rec + 16 * ((long long)i * (t.nT - 1) + jj));
  const double4 r0 = R[0], r1 = R[1], r2 = R[2];
  const double a = tlerp(w, r0.x, r0.y), b = tlerp(w, r0.z, r0.w);
  if (!(a <= le && le < b)) {
    if (jj == 0 && le < a) le = a;                       // below the table: clamped to its first node
    else if (jj == t.nT - 2 && le >= b) le = b;          // above: clamped to its last node
    else return false;
  }
  wT = (le - a) / (b - a);
  lP = tlerp(wT, tlerp(w, r1.x, r1.y), tlerp(w, r2.x, r2.y));
  lc2 = tlerp(wT, tlerp(w, r1.z, r1.w), tlerp(w, r2.z, r2.w));
  return true;
}

// Table cell seed from the learned network for this lane's (log rho, log e);
// every lane of the wave must call it (the hidden layer runs on the matrix cores).
// lane: the lane index if the caller has an opaque one (see tdh_mlp_dev.hpp)
template <bool HOISTED = false>
__device__ __forceinline__ int seed_cell_wave(const Seed &s, const Table &t, double lr, double le, int lane = -1) {
  const float x0 = norm01(lr, s.lr_lo, s.lr_hi), x1 = norm01(le, s.le_lo, s.le_hi);
  const int l = lane >= 0 ? lane : (int)(threadIdx.x & 63);
  const float y = HOISTED ? mlp_wave_forward_hoisted(s.w, x0, x1, l) : mlp_wave_forward_fast(s.w, x0, x1, l);
  const double lT = s.lt_lo + 0.5 * ((double)y + 1.0) * (s.lt_hi - s.lt_lo);
  const double x = (lT - t.lT0) / t.dlT;
  if (!(x > 0.0)) return 0;
  if (x > (double)(t.nT - 2)) return t.nT - 2;
  return (int)x;
}

// ---------------------------------------------------------------------------
// base-10 logarithm and power of ten for the table lookups (the table path
// takes two of each per EOS evaluation; these cost ~20 vector instructions and
// one cached load each, against ~105 and ~45 for the general-purpose forms)
// ---------------------------------------------------------------------------
// log10 x, x > 0 normal.  x = u 2^(e-1), u = 2m in [1, 2); with c the tabled
// reciprocal of the centre of u's 1/128 interval, r = u c - 1 (one fused
// multiply-add, |r| <= 2^-8) and log10 x = (e-1) log10 2 - log10 c +
// log10(1 + r), the last by its Taylor series through r^7 (truncation below
// 3e-21); log10 2 is split into a part whose product with the exponent is
// exact and a remainder.
__device__ __forceinline__ double log10_tab(const double2 *lg, double x) {
  int e;
  const double m = frexp(x, &e);                     // [1/2, 1)
  const int i = (__double2hiint(m) >> 13) & 127;     // leading 7 fraction bits
  const double2 g = lg[i];                           // {2 c_i, -log10 c_i}
  const double r = fma(m, g.x, -1.0);
  constexpr double A = 0x1.bcb7b1526e50ep-2;         // log10(e)
  double p = A / 7.0;
  p = fma(p, r, -A / 6.0);
  p = fma(p, r, A / 5.0);
  p = fma(p, r, -A / 4.0);
  p = fma(p, r, A / 3.0);
  p = fma(p, r, -A / 2.0);
  p = fma(p, r, A);
  const double l = fma(p, r, g.y);
  const double de = (double)(e - 1);
  constexpr double L2H = 0x1.3441350800000p-2;       // log10(2), leading 32 bits
  constexpr double L2L = 0x1.f79fef311f12bp-34;      // log10(2) - L2H
  return fma(de, L2H, fma(de, L2L, l));
}

// 10^x, |x| < 300.  k = nearest integer to 64 x log2(10); r = x - k log10(2)/64
// (two-part reduction), 10^x = 2^(k>>6) 2^((k&63)/64) e^(r ln 10) with
// |r ln 10| <= ln(2)/128 and e^s - 1 by its Taylor series through s^6
// (truncation below 3e-20).
__device__ __forceinline__ double exp10_tab(const double *ex, double x) {
  constexpr double K64 = 0x1.a934f0979a371p+7;       // 64 log2(10)
  constexpr double L2H = 0x1.3441350800000p-8;       // log10(2)/64, leading 32 bits
  constexpr double L2L = 0x1.f79fef311f12bp-40;
  constexpr double LN10 = 0x1.26bb1bbb55516p+1;
  const double kd = rint(x * K64);
  const int k = (int)kd;
  const double s = fma(-kd, L2L, fma(-kd, L2H, x)) * LN10;
  double p = 1.0 / 720.0;
  p = fma(p, s, 1.0 / 120.0);
  p = fma(p, s, 1.0 / 24.0);
  p = fma(p, s, 1.0 / 6.0);
  p = fma(p, s, 0.5);
  p = fma(p, s, 1.0);
  const double t = ex[k & 63];
  return ldexp(fma(t, p * s, t), k >> 6);
}

// (rho, U) -> P, c_s.  jseed: table cell to start from (-1: bisection).
template <int PK = 0>
__device__ __forceinline__ void eos_pc(const Phys &p, const Table &t, double rho, double U, int jseed, double &P,
                                       double &cs, int *jout = nullptr) {
  if (k_eos<PK>(p) == 0) {
    const double Ue = fmax(U, u_floor(p, rho));
    P = (p.gamma - 1.0) * Ue;
    cs = sqrt(p.gamma * P / rho);
    return;
  }
  const double Ue = fmax(U, rho * p.e_floor);
  int i, j, it;
  double w, wT, lP, lc2;
  table_rho(t, log10_tab(t.lg, rho), i, w);
  const double le = log10_tab(t.lg, Ue / rho);
  const int jj = min(jseed, t.nT - 2);
  if (jseed >= 0 && table_record(t, i, w, le, jj, wT, lP, lc2)) {
    j = jj;
  } else {
    table_invert(t, i, w, le, jseed, p.newton_max_iter, j, wT, it);
    tbil_pc(t, i, w, j, wT, lP, lc2);
  }
  P = exp10_tab(t.ex, lP);
  cs = exp10_tab(t.ex, 0.5 * lc2);
  if (jout) *jout = j;
}

// ---------------------------------------------------------------------------
// cell primitives and the Riemann problem
// ---------------------------------------------------------------------------
template <int PK = 0>
__device__ __forceinline__ void c2p(const Phys &p, const double *q, double *w) {
  const double rho = q[IDN];
  const double inv = 1.0 / rho;
  const double K = 0.5 * (q[IM1] * q[IM1] + q[IM2] * q[IM2] + q[IM3] * q[IM3]) * inv;
  const double Uc = q[IEN] - K;
  double Ueos = Uc;
  if (k_dual<PK>(p)) {
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

// HLLE: the HLL flux (Toro Sec. 10.3) with the Davis wave-speed bounds of the
// HLLC solver above; the solver of the paper's production runs (Table 1)
__device__ __forceinline__ void hlle(const double *wl, double pl, double cl, const double *wr, double pr, double cr,
                                     double *f) {
  const double rl = wl[0], ul = wl[1], vl = wl[2], zl = wl[3];
  const double rr = wr[0], ur = wr[1], vr = wr[2], zr = wr[3];
  const double El = wl[4] + 0.5 * rl * (ul * ul + vl * vl + zl * zl);
  const double Er = wr[4] + 0.5 * rr * (ur * ur + vr * vr + zr * zr);
  const double sl = fmin(ul - cl, ur - cr);
  const double sr = fmax(ul + cl, ur + cr);
  const double fl[5] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, rl * ul * zl, (El + pl) * ul};
  const double fr[5] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, rr * ur * zr, (Er + pr) * ur};
  if (sl >= 0.0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) f[v] = fl[v];
    return;
  }
  if (sr <= 0.0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) f[v] = fr[v];
    return;
  }
  const double ql[5] = {rl, rl * ul, rl * vl, rl * zl, El};
  const double qr[5] = {rr, rr * ur, rr * vr, rr * zr, Er};
  const double ss = sl * sr, den = sr - sl;
#pragma unroll
  for (int v = 0; v < 5; ++v) f[v] = (sr * fl[v] - sl * fr[v] + ss * (qr[v] - ql[v])) / den;
}

// ---------------------------------------------------------------------------
// gravity / excision geometry
// ---------------------------------------------------------------------------
// centre of global cell g (refinement level r) along d
__device__ __forceinline__ double cell_x(const MeshDev &m, int d, int g, int r = 0) {
  return m.x0[d] + (g + 0.5) * dx_lev(m, d, r);
}

__device__ __forceinline__ double phi_point(const Phys &p, const MeshDev &m, int gx, int gy, int gz, double t,
                                            int r = 0) {
  const double dx = cell_x(m, 0, gx, r) - (p.bh_x0[0] - p.v_frame[0] * t);
  const double dy = cell_x(m, 1, gy, r) - (p.bh_x0[1] - p.v_frame[1] * t);
  const double dz = cell_x(m, 2, gz, r) - (p.bh_x0[2] - p.v_frame[2] * t);
  return -p.gm_bh / sqrt(dx * dx + dy * dy + dz * dz + p.r_soft * p.r_soft);
}

template <int PK = 0>
__device__ __forceinline__ bool excised(const Phys &p, const MeshDev &m, int gx, int gy, int gz, double t,
                                        int r = 0) {
  if (k_grav<PK>(p) != 2 || !(p.r_exc > 0.0)) return false;
  const double dx = cell_x(m, 0, gx, r) - (p.bh_x0[0] - p.v_frame[0] * t);
  const double dy = cell_x(m, 1, gy, r) - (p.bh_x0[1] - p.v_frame[1] * t);
  const double dz = cell_x(m, 2, gz, r) - (p.bh_x0[2] - p.v_frame[2] * t);
  return dx * dx + dy * dy + dz * dz < p.r_exc * p.r_exc;
}

// potential at local offset (i,j,k) in [-1, n] of block B
template <int PK = 0>
__device__ __forceinline__ double phi_at(const StageArgs &a, const BlockInfo &B, int i, int j, int k, double t) {
  if (k_grav<PK>(a.p) == 1) {
    const int np = B.n + 2;
    return a.phi[B.poff + ((long long)(k + 1) * np + (j + 1)) * np + (i + 1)];
  }
  return phi_point(a.p, a.m, B.ox + i, B.oy + j, B.oz + k, t, lev_of<PK>(B));
}

// phi_at for the kernels that serve every mesh (CFL reduction, flux
// correction): the block's own refinement level, whatever the kind
__device__ __forceinline__ double phi_at_block(const StageArgs &a, const BlockInfo &B, int i, int j, int k, double t) {
  if (a.p.grav_kind == 1) return phi_at<0>(a, B, i, j, k, t);
  return phi_point(a.p, a.m, B.ox + i, B.oy + j, B.oz + k, t, B.lev);
}

// ---------------------------------------------------------------------------
// stage kernel
// ---------------------------------------------------------------------------
struct Nbr {
  int blk;       // owning block of the cell across a face (-1: beyond an outflow edge)
  long long idx; // its local cell index
  int u0, u1;    // its face-cell coordinates (transverse, increasing axis order)
};

// Src's combination of three stored values (start or latest A, end or stage-1
// B, stage-1 C of a dense output), as src_val takes it from the buffers.
__device__ __forceinline__ double src_combine(const Src &s, double A, double B, double C) {
  if (s.w == 0.0) return A;
  if (s.C) return (1.0 - s.w) * A + s.w * (1.0 - s.w) * C + s.w * s.w * B;
  if (s.w == 1.0) return B;
  return (1.0 - s.w) * A + s.w * B;
}

// Conserved state of a cell of a finer block Bn (source s) as the reader sees
// it: each stored history of the 2x2x2 children from local cell (i0, j0, k0)
// is restricted to their mean (summed in k, j, i order), then interpolated in
// time (Sec. LAT method, coarse-fine interfaces).
template <int NV>
__device__ __forceinline__ void restricted(const BlockInfo &Bn, const Src &s, int i0, int j0, int k0, double *q) {
  const long long n = Bn.n, n3 = n * n * n;
  const long long c0 = Bn.off + (k0 * n + j0) * n + i0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double hA = 0.0, hB = 0.0, hC = 0.0;
    for (int kz = 0; kz < 2; ++kz)
      for (int jy = 0; jy < 2; ++jy)
        for (int ix = 0; ix < 2; ++ix) {
          const long long o = c0 + v * n3 + (kz * n + jy) * n + ix;
          hA += s.A[o];
          hB += s.B[o];
          if (s.C) hC += s.C[o];
        }
    q[v] = src_combine(s, 0.125 * hA, 0.125 * hB, 0.125 * hC);
  }
}

// Conserved state of global cell g of level r (any index: wrapped here) when
// the block covering it is on level r or r + 1.
template <int NV, int PK>
__device__ __forceinline__ void level_state(const StageArgs &a, int fb, int r, int gx, int gy, int gz, double *q) {
  const MeshDev &m = a.m;
  gx = wrap_axis(gx, m.nx << r, m.bc[0]);
  gy = wrap_axis(gy, m.ny << r, m.bc[1]);
  gz = wrap_axis(gz, m.nz << r, m.bc[2]);
  const int nb = block_of(m, r, gx, gy, gz);
  const BlockInfo Bn = m.blocks[nb];
  const Src s = source_of<PK>(a, fb, nb);
  if (Bn.lev != r) {
    restricted<NV>(Bn, s, 2 * gx - Bn.ox, 2 * gy - Bn.oy, 2 * gz - Bn.oz, q);
    return;
  }
  const long long n = Bn.n, n3 = n * n * n;
  const long long idx = ((long long)(gz - Bn.oz) * n + (gy - Bn.oy)) * n + (gx - Bn.ox);
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = src_val(s, Bn.off + v * n3 + idx);
}

// Ghost state of fine cell g (level r = 1, inside the extents) covered by a
// coarser block: prolongation of the coarse cell containing it from coarse
// values at the reader's stage time, q_c + sum_d s_d minmod(q_c - q_-d,
// q_+d - q_c) / 4 in x, y, z order, s_d = +1 for the upper child, -1 for the
// lower (coarse neighbours covered by fine blocks enter restricted).
template <int NV, int PK>
__device__ __forceinline__ void prolonged(const StageArgs &a, int fb, int r, int gx, int gy, int gz, double *q) {
  const int c[3] = {gx >> 1, gy >> 1, gz >> 1};
  const int g[3] = {gx, gy, gz};
  double qc[6];
  level_state<NV, PK>(a, fb, r - 1, c[0], c[1], c[2], qc);
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = qc[v];
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    int cm[3] = {c[0], c[1], c[2]}, cp[3] = {c[0], c[1], c[2]};
    cm[d] -= 1;
    cp[d] += 1;
    double qm[6], qp[6];
    level_state<NV, PK>(a, fb, r - 1, cm[0], cm[1], cm[2], qm);
    level_state<NV, PK>(a, fb, r - 1, cp[0], cp[1], cp[2], qp);
    const double sgn = (g[d] & 1) ? 0.25 : -0.25;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double dl = qc[v] - qm[v], dr = qp[v] - qc[v];
      const double mm = dl * dr <= 0.0 ? 0.0 : (fabs(dl) < fabs(dr) ? dl : dr);
      q[v] += sgn * mm;
    }
  }
}

// load conserved state of global cell g (stage view of the reader), return block info
template <int NV, int PK = 0>
__device__ __forceinline__ void load_q(const StageArgs &a, int b, const BlockInfo &B, const Src &own, int fb,
                                       int gx, int gy, int gz, double *q, int *nb_out, long long *idx_out) {
  const MeshDev &m = a.m;
  const int r = lev_of<PK>(B);
  gx = wrap_axis(gx, m.nx << r, m.bc[0]);
  gy = wrap_axis(gy, m.ny << r, m.bc[1]);
  gz = wrap_axis(gz, m.nz << r, m.bc[2]);
  const int lx = gx - B.ox, ly = gy - B.oy, lz = gz - B.oz;
  if ((unsigned)lx < (unsigned)B.n && (unsigned)ly < (unsigned)B.n && (unsigned)lz < (unsigned)B.n) {
    const long long n3 = (long long)B.n * B.n * B.n;
    const long long idx = ((long long)lz * B.n + ly) * B.n + lx;
    _Pragma("unroll") for (int v = 0; v < NV; ++v) q[v] = src_val(own, B.off + v * n3 + idx);
    if (nb_out) { *nb_out = b; *idx_out = idx; }
    return;
  }
  const int nb = k_amr<PK>() ? block_of(m, r, gx, gy, gz) : block_of(m, gx, gy, gz);
  const BlockInfo Bn = m.blocks[nb];
  if (k_amr<PK>() && Bn.lev != r) {  // a block on the other refinement level
    if (Bn.lev > r) {
      const Src s = source_of<PK>(a, fb, nb);
      restricted<NV>(Bn, s, 2 * gx - Bn.ox, 2 * gy - Bn.oy, 2 * gz - Bn.oz, q);
    } else {
      prolonged<NV, PK>(a, fb, r, gx, gy, gz, q);
    }
    if (nb_out) { *nb_out = nb; *idx_out = -1; }
    return;
  }
  const Src s = source_of<PK>(a, fb, nb);
  const long long n3 = (long long)Bn.n * Bn.n * Bn.n;
  const long long idx = ((long long)(gz - Bn.oz) * Bn.n + (gy - Bn.oy)) * Bn.n + (gx - Bn.ox);
  _Pragma("unroll") for (int v = 0; v < NV; ++v) q[v] = src_val(s, Bn.off + v * n3 + idx);
  if (nb_out) { *nb_out = nb; *idx_out = idx; }
}

// ---------------------------------------------------------------------------
// tiled stage kernel
//
// A workgroup advances one tile of TX x TY x TZ cells (256 cells, one per
// thread).  For each axis it stages the tile extended by two cells along
// that axis in LDS as primitives (C2P done once per staged cell), computes
// every face flux of the tile once (PLM -> EOS -> HLLC), and each thread
// accumulates the divergence, gravity sources and neighbour energies of its
// own cell.  Tile shapes are template parameters so the runtime can pick
// the fastest; every shape gives the same result bit for bit.
// ---------------------------------------------------------------------------
template <int TX, int TY, int TZ>
struct TileGeom {
  static constexpr int TV = TX * TY * TZ;
  static constexpr int A0 = TY * TZ, A1 = TX * TZ, A2 = TX * TY;  // face areas normal to x, y, z
  static constexpr int AMAX = A0 > A1 ? (A0 > A2 ? A0 : A2) : (A1 > A2 ? A1 : A2);
  static constexpr int HALO = 4 * AMAX;  // two layers on each side along one axis
  static constexpr int F0 = (TX + 1) * TY * TZ, F1 = TX * (TY + 1) * TZ, F2 = TX * TY * (TZ + 1);
  static constexpr int NF = F0 > F1 ? (F0 > F2 ? F0 : F2) : (F1 > F2 ? F1 : F2);
};

// LDS slot of the staged cell at tile coordinates (c0, c1, c2), only the D-th of
// which may lie outside the tile: the tile's own cells first (x fastest), then
// the halo of axis D as [layer][transverse] with layers -2, -1, T_D, T_D + 1.
template <int TX, int TY, int TZ, int D>
__device__ __forceinline__ int cell_slot(int c0, int c1, int c2) {
  using G = TileGeom<TX, TY, TZ>;
  constexpr int TD = D == 0 ? TX : (D == 1 ? TY : TZ);
  constexpr int A = D == 0 ? G::A0 : (D == 1 ? G::A1 : G::A2);
  const int cd = D == 0 ? c0 : (D == 1 ? c1 : c2);
  const int u = D == 0 ? c1 + TY * c2 : (D == 1 ? c0 + TX * c2 : c0 + TX * c1);
  const int layer = cd < 0 ? cd + 2 : cd - TD + 2;
  return (cd >= 0 && cd < TD) ? c0 + TX * (c1 + TY * c2) : G::TV + layer * A + u;
}

// The thread index as a value the compiler cannot hoist out of the item loop:
// every per-thread index below is then recomputed per item (a few integer
// operations) instead of being held in registers for the kernel's lifetime.
__device__ __forceinline__ int item_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
  return t;
}

// Per-item values that are the same in every lane, moved to scalar registers
// (the loads that produce them are vector loads from writable memory).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long uni(long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ BlockInfo uni(const BlockInfo &b) {
  BlockInfo r;
  r.n = uni(b.n); r.ox = uni(b.ox); r.oy = uni(b.oy); r.oz = uni(b.oz);
  r.lev = uni(b.lev); r.pad_ = 0;
  r.off = uni(b.off); r.poff = uni(b.poff); r.ioff = uni(b.ioff); r.foff = uni(b.foff);
  return r;
}

// Segment of the seed cells that belongs to a block's stage input / output
// buffer (0: Qa, 1: Qb, 2: Qs) given the block's parity.
__device__ __forceinline__ int jseg_in(const StageArgs &a, int par) { return a.phase == 1 ? par : 2; }
__device__ __forceinline__ int jseg_out(const StageArgs &a, int par) { return a.phase == 1 ? 2 : 1 - par; }

// Work items of a persistent launch, XCD-aware.  Workgroups are dispatched to
// the eight XCDs round robin (workgroup w on XCD w % 8), so each XCD takes a
// contiguous share of the items: neighbouring tiles, whose halos overlap,
// then run under one L2.
struct ItemRange {
  int first, end, step;
};
__device__ __forceinline__ ItemRange xcd_items(int i0, int i1) {
  constexpr int kXcd = 8;
  const int w = (int)blockIdx.x, G = (int)gridDim.x;
  ItemRange r;
  if (G < kXcd) {  // too few workgroups to give every XCD some: plain striding
    r.first = i0 + w;
    r.end = i1;
    r.step = G;
    return r;
  }
  const int x = w % kXcd;
  const int total = i1 - i0, per = (total + kXcd - 1) / kXcd;
  r.first = i0 + min(total, x * per) + w / kXcd;
  r.end = i0 + min(total, (x + 1) * per);
  r.step = G / kXcd + (x < G % kXcd ? 1 : 0);  // workgroups on this XCD
  return r;
}

// Work items of a launch over levels Llo..Lhi (blocks sorted finest level
// first, item prefix `start` over that order), level by level from the finest,
// each level's items shared among the XCDs as by xcd_items: every XCD gets its
// share of every level, so a launch that mixes levels is balanced across the
// XCDs as separate per-level launches would be.
struct LevelItems {
  const int *cnt_ge, *start;
  int L, Llo, item;
  ItemRange R;
  __device__ __forceinline__ LevelItems(const StageArgs &a, const int *st) : cnt_ge(a.cnt_ge), start(st) {
    Llo = a.Llo;
    L = min(a.Lhi, a.lmax) + 1;
    item = 0;
    R.first = R.end = R.step = 0;
    advance_level();
  }
  __device__ __forceinline__ void advance_level() {
    while (--L >= Llo) {
      const int b0 = cnt_ge[L + 1], b1 = cnt_ge[L];
      if (b1 <= b0) continue;
      R = xcd_items(start[b0], start[b1]);
      item = R.first;
      if (item < R.end) return;
    }
  }
  __device__ __forceinline__ bool valid() const { return L >= Llo; }
  __device__ __forceinline__ void next() {
    item += R.step;
    if (item >= R.end) advance_level();
  }
};

struct TileCtx {
  int b;
  BlockInfo B;
  int to[3];      // tile origin in the block
  int fb;         // block factor
  double dtb, t;  // block step, stage time
  Src own;
};

// ---------------------------------------------------------------------------
// pieces shared by the two stage-kernel forms (so that they agree bit for bit)
// ---------------------------------------------------------------------------
// PLM states either side of a face from four cells along the axis (q1 | q2 are
// the cells left | right of the face)
__device__ __forceinline__ void plm_face(double q0, double q1, double q2, double q3, double &l, double &r) {
  l = q1 + 0.5 * vanleer(q1 - q0, q2 - q1);
  r = q2 - 0.5 * vanleer(q2 - q1, q3 - q2);
}

// Flux through one face along D from its reconstructed states (rotated:
// normal velocity first): EOS of both states, HLLC, auxiliary-energy flux and
// face velocity, the excision rule, and for block-boundary faces the stage-1
// flux or the time-integrated impulse.  Gf receives the fluxes in conserved
// order (slots 0..NV-1) and the face velocity (slot 6).
//   fr: local coordinates of the cell right of the face; nbo: block owning the
//   cell across a block face (-1 beyond an outflow edge); seedl, seedr: seed
//   cells of the left and right states (-1: none).  The two seeds come from
//   the cells' centre states, so the two EOS evaluations do not wait on each
//   other.
template <int NV, int D, int PK = 0>
__device__ __forceinline__ void face_flux(const StageArgs &a, const BlockInfo &B, int fb, double t, double dtb,
                                          const int *fr, const double *wl, const double *wr, int seedl, int seedr,
                                          int nbo, double *Gf, int excl = -1, int excr = -1) {
  constexpr int PN = 1 + D, P1 = 1 + (D + 1) % 3, P2 = 1 + (D + 2) % 3;
  const Phys &p = a.p;
  const MeshDev &m = a.m;
  const int n = B.n;
  double pl, cl, pr, cr;
  eos_pc<PK>(p, a.t, wl[0], wl[4], seedl, pl, cl);
  eos_pc<PK>(p, a.t, wr[0], wr[4], seedr, pr, cr);
  double F[5];
  if (k_riemann<PK>(p) == 1) hlle(wl, pl, cl, wr, pr, cr, F);
  else hllc(wl, pl, cl, wr, pr, cr, F);
  double FA = 0.0, vf;
  {
    const bool up_left = F[0] >= 0.0;
    const double ru = up_left ? wl[0] : wr[0];
    if (NV > 5) FA = F[0] * ((up_left ? wl[5] : wr[5]) / ru);
    vf = F[0] / ru;
  }
  if (k_grav<PK>(p) == 2 && p.r_exc > 0.0) {
    bool eR, eL;
    if constexpr (k_gcache<PK>()) {  // the flags staged in LDS
      eR = excr != 0;
      eL = excl != 0;
    } else {
      int gl[3] = {B.ox + fr[0], B.oy + fr[1], B.oz + fr[2]};
      eR = excr >= 0 ? excr != 0 : excised<PK>(p, m, gl[0], gl[1], gl[2], t, lev_of<PK>(B));
      gl[D] -= 1;
      eL = excl >= 0 ? excl != 0 : excised<PK>(p, m, gl[0], gl[1], gl[2], t, lev_of<PK>(B));
    }
    if (eL != eR) {
      const bool into = eR ? (F[0] >= 0.0) : (F[0] <= 0.0);
      if (!into) {
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = 0.0;
        FA = 0.0;
        vf = 0.0;
      }
    }
  }
  Gf[IDN] = F[0];
  Gf[PN] = F[1];
  Gf[P1] = F[2];
  Gf[P2] = F[3];
  Gf[IEN] = F[4];
  Gf[5] = FA;
  Gf[6] = vf;
  // block-boundary faces: stage-1 flux, then the time-integrated impulse
  const int bd = fr[D];
  if (k_multi<PK>() && (bd == 0 || bd == n)) {
    const int side = bd == n;
    const int u0 = D == 0 ? fr[1] : fr[0];
    const int u1 = D == 2 ? fr[1] : fr[2];
    const long long nn2 = (long long)n * n;
    const long long base = B.ioff + (long long)(2 * D + side) * NV * nn2 + (long long)u1 * n + u0;
    // only faces towards a block on another schedule, or on another
    // refinement level, take part in the reflux
    const int fn = nbo >= 0 ? a.fac[nbo] : fb;
    const bool other_level = k_amr<PK>() && nbo >= 0 && m.blocks[nbo].lev != B.lev;
    if (fn == fb && !other_level) {
    } else if (a.phase == 1) {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.bf1[base + v * nn2] = Gf[v];
    } else {
      const int r = lev_of<PK>(B);
      const double area = dx_lev(m, (D + 1) % 3, r) * dx_lev(m, (D + 2) % 3, r);
      const int fw = fb > fn ? fb : fn;
      const bool overwrite = (a.k & (fw - 1)) == 0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const long long ix = base + v * nn2;
        const double Is = 0.5 * (a.bf1[ix] + Gf[v]) * area * dtb;
        a.imp[ix] = overwrite ? Is : a.imp[ix] + Is;
      }
    }
  }
}

// One axis's contribution to a cell's right-hand side (divergence, face-
// velocity divergence, gravity) and the neighbour energies of the resync.
// Flo / Fhi: the cell's low / high face along D (slots as face_flux); Em, Ep:
// stage-input E of the neighbours along D; rho: the cell's stage-input density.
template <int NV, int D, int PK = 0>
__device__ __forceinline__ void axis_update(const StageArgs &a, const BlockInfo &B, double t, const int *lc,
                                            const double *Flo, const double *Fhi, double rho, double Em, double Ep,
                                            double *rhs, double &divv, double &emax, const double *phis = nullptr) {
  constexpr int PN = 1 + D;
  const Phys &p = a.p;
  const MeshDev &m = a.m;
  const double idx = inv_dx_lev(m, D, lev_of<PK>(B));
  const double hd = dx_lev(m, D, lev_of<PK>(B));
#pragma unroll
  for (int v = 0; v < NV; ++v) rhs[v] -= (Fhi[v] - Flo[v]) * idx;
  divv += (Fhi[6] - Flo[6]) * idx;
  emax = fmax(emax, fmax(Em, Ep));
  if (k_grav<PK>(p)) {
    int im[3] = {lc[0], lc[1], lc[2]}, ip[3] = {lc[0], lc[1], lc[2]};
    im[D] -= 1;
    ip[D] += 1;
    const double pm = phis ? phis[0] : phi_at<PK>(a, B, im[0], im[1], im[2], t);
    const double p0 = phis ? phis[1] : phi_at<PK>(a, B, lc[0], lc[1], lc[2], t);
    const double pp = phis ? phis[2] : phi_at<PK>(a, B, ip[0], ip[1], ip[2], t);
    rhs[PN] -= rho * (pp - pm) / (2.0 * hd);
    rhs[IEN] -= (Fhi[IDN] * (pp - p0) + Flo[IDN] * (p0 - pm)) / (2.0 * hd);
  }
  // Pin the sums here: otherwise the compiler may sink this axis's arithmetic
  // to the final use and keep its inputs live through the remaining axes.
#pragma unroll
  for (int v = 0; v < NV; ++v) asm volatile("" : "+v"(rhs[v]));
  asm volatile("" : "+v"(divv), "+v"(emax));
}

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// RK combine of one cell and everything after it: compression of U_aux,
// floors, resynchronisation, excision reset, the store, and (modes 1 and 3)
// the table cell of the output state for the next stage.
//   cflv (stage 2 of the fused form, a.cfl_part set): receives the cell's CFL
//   limit of its output state, computed as the CFL reduction does; in modes 2
//   and 4 that state's table cell is recorded as the next stage's seed.
template <int NV, bool NET, int PK = 0>
__device__ __forceinline__ void finish_cell(const StageArgs &a, const BlockInfo &B, const Src &own, int parb, double dtb,
                                            double tk, const int *lc, long long cell, int jcell, const double *rhs,
                                            double divv, double emax, double *cflv = nullptr) {
  const Phys &p = a.p;
  const MeshDev &m = a.m;
  const long long n3 = (long long)B.n * B.n * B.n;
  double qc[6];
#pragma unroll
  for (int v = 0; v < NV; ++v) qc[v] = src_val(own, B.off + v * n3 + cell);
  const double *Qbase = parb ? a.Qb : a.Qa;
  double qn[6];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double qs = qc[v] + dtb * rhs[v];
    qn[v] = a.phase == 1 ? qs : 0.5 * Qbase[B.off + v * n3 + cell] + 0.5 * qs;
  }
  if (NV > 5) {
    const double tau = a.phase == 1 ? dtb : 0.5 * dtb;
    if (k_eos<PK>(p) == 0) {
      qn[IAX] = qn[IAX] * exp(-(p.gamma - 1.0) * divv * tau);
    } else {
      double Pa, ca;
      eos_pc<PK>(p, a.t, qc[IDN], qn[IAX], p.inv_mode == 0 ? -1 : jcell, Pa, ca);
      qn[IAX] = qn[IAX] - Pa * divv * tau;
    }
    const double uf = u_floor<PK>(p, qn[IDN] > p.rho_floor ? qn[IDN] : p.rho_floor);
    if (qn[IAX] < uf) qn[IAX] = uf;
  }
  if (qn[IDN] < p.rho_floor) qn[IDN] = p.rho_floor;
  {
    double w[6];
    c2p<PK>(p, qn, w);
    const double uf = u_floor<PK>(p, qn[IDN]);
    if (w[4] < uf) {
      qn[IEN] += uf - w[4];
      if (NV > 5 && qn[IAX] < uf) qn[IAX] = uf;
    }
  }
  if (NV > 5) {
    const double K = 0.5 * (qn[IM1] * qn[IM1] + qn[IM2] * qn[IM2] + qn[IM3] * qn[IM3]) / qn[IDN];
    const double Uc = qn[IEN] - K;
    if (Uc > 0.0 && Uc > p.eta2 * emax) qn[IAX] = Uc;
  }
  if (a.phase == 2 && k_grav<PK>(p) == 2 && p.r_exc > 0.0) {
    if (excised<PK>(p, m, B.ox + lc[0], B.oy + lc[1], B.oz + lc[2], tk + dtb, lev_of<PK>(B))) {
      const double uf = u_floor<PK>(p, p.rho_floor);
      qn[IDN] = p.rho_floor;
      qn[IM1] = qn[IM2] = qn[IM3] = 0.0;
      qn[IEN] = uf;
      if (NV > 5) qn[IAX] = uf;
    }
  }
  double *out = a.phase == 1 ? a.Qs : (parb ? a.Qa : a.Qb);
#pragma unroll
  for (int v = 0; v < NV; ++v) out[B.off + v * n3 + cell] = qn[v];
  if (k_eos<PK>(p) == 1 && (p.inv_mode == 1 || p.inv_mode == 3)) {
    // The table cell of the output state seeds the next stage's queries of
    // this cell.  Its search starts from the learned network's prediction
    // (mode 1; the whole wave takes part, every thread owns a cell) or from
    // the input state's cell (mode 3).
    double w[6];
    c2p<PK>(p, qn, w);
    const double Ue = fmax(w[4], w[0] * p.e_floor);
    const double lr = log10_tab(a.t.lg, w[0]), le = log10_tab(a.t.lg, Ue / w[0]);
    int start = jcell;
    if constexpr (NET) start = seed_cell_wave<true>(a.s, a.t, lr, le, item_tid() & 63);
    int i, j, it;
    double wr, wT;
    table_rho(a.t, lr, i, wr);
    table_invert(a.t, i, wr, le, start, p.newton_max_iter, j, wT, it);
    a.jc[jseg_out(a, parb) * a.jn + B.off / NV + cell] = j;
  }
  if (cflv && a.cfl_part && a.phase == 2) {
    double w[6];
    c2p<PK>(p, qn, w);
    double P, cs;
    int jo = -1;
    eos_pc<PK>(p, a.t, w[0], w[4], (k_eos<PK>(p) == 1 && p.inv_mode != 0) ? jcell : -1, P, cs, &jo);
    double best = INFINITY;
    const int r = lev_of<PK>(B);
    for (int d = 0; d < 3; ++d) best = fmin(best, dx_lev(m, d, r) / (fabs(w[1 + d]) + cs));
    if (k_grav<PK>(p)) {
      const double t = tk + dtb;
      double g2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        int ip[3] = {lc[0], lc[1], lc[2]}, im[3] = {lc[0], lc[1], lc[2]};
        ip[d] += 1;
        im[d] -= 1;
        const double gd = (phi_at<PK>(a, B, ip[0], ip[1], ip[2], t) - phi_at<PK>(a, B, im[0], im[1], im[2], t)) /
                          (2.0 * dx_lev(m, d, r));
        g2 += gd * gd;
      }
      const double dmin = fmin(dx_lev(m, 0, r), fmin(dx_lev(m, 1, r), dx_lev(m, 2, r)));
      if (g2 > 0.0) best = fmin(best, sqrt(dmin / sqrt(g2)));
    }
    *cflv = best;
    if (k_eos<PK>(p) == 1 && (p.inv_mode == 2 || p.inv_mode == 4))
      a.jc[jseg_out(a, parb) * a.jn + B.off / NV + cell] = jo;
  }
}

// ---------------------------------------------------------------------------
// fused form: one workgroup per tile, faces through LDS
// ---------------------------------------------------------------------------
template <int TX, int TY, int TZ, int NV, int D, int NT, int PK>
__device__ __forceinline__ void tile_axis(const StageArgs &a, const TileCtx &T, double *sW, double *sF, int *sB,
                                          const int *sJc, double *rhs, double &divv, double &emax, double *sPhi,
                                          unsigned char *sExc) {
  using G = TileGeom<TX, TY, TZ>;
  constexpr int SW = G::TV + G::HALO;  // stride of one variable in sW
  constexpr int TD = D == 0 ? TX : (D == 1 ? TY : TZ);
  constexpr int A = D == 0 ? G::A0 : (D == 1 ? G::A1 : G::A2);
  constexpr int F0 = TX + (D == 0), F1 = TY + (D == 1), F2 = TZ + (D == 2);
  constexpr int NFD = F0 * F1 * F2;
  constexpr int FSTR = D == 0 ? 1 : (D == 1 ? F0 : F0 * F1);
  constexpr int PN = 1 + D, P1 = 1 + (D + 1) % 3, P2 = 1 + (D + 2) % 3;
  static_assert(4 * A <= kChunk, "one halo cell per thread");
  const Phys &p = a.p;
  const MeshDev &m = a.m;
  const int tid = item_tid();
  const int cc[3] = {tid % TX, (tid / TX) % TY, tid / (TX * TY)};  // own cell in the tile
  const int Nd = (D == 0 ? m.nx : (D == 1 ? m.ny : m.nz)) << lev_of<PK>(T.B);
  // stage the halo along D (the tile's own cells were staged at the item start)
  if (tid < 4 * A) {
    const int layer = tid / A, u = tid % A;
    int c[3];
    const int cd = layer < 2 ? layer - 2 : TD + layer - 2;
    if (D == 0) { c[0] = cd; c[1] = u % TY; c[2] = u / TY; }
    if (D == 1) { c[0] = u % TX; c[1] = cd; c[2] = u / TX; }
    if (D == 2) { c[0] = u % TX; c[1] = u / TX; c[2] = cd; }
    const int g[3] = {T.B.ox + T.to[0] + c[0], T.B.oy + T.to[1] + c[1], T.B.oz + T.to[2] + c[2]};
    double q[6], w[6];
    int nb_;
    long long id_;
    load_q<NV, PK>(a, T.b, T.B, T.own, T.fb, g[0], g[1], g[2], q, &nb_, &id_);
    c2p<PK>(p, q, w);
    const int slot = G::TV + tid;
#pragma unroll
    for (int v = 0; v < NV; ++v) sW[v * SW + slot] = w[v];
    sW[6 * SW + slot] = q[IEN];
    sB[tid] = (m.bc[D] == 0 || (g[D] >= 0 && g[D] < Nd)) ? nb_ : -1;
    if constexpr (k_gcache<PK>()) {
      if (layer == 1 || layer == 2) {  // the cells next to the tile: the only halo the terms need
        const int l0 = T.to[0] + c[0], l1 = T.to[1] + c[1], l2 = T.to[2] + c[2];
        sPhi[slot] = phi_at<PK>(a, T.B, l0, l1, l2, T.t);
        sExc[slot] = excised<PK>(p, m, g[0], g[1], g[2], T.t, lev_of<PK>(T.B)) ? 1 : 0;
      }
    }
  }
  __syncthreads();
  // every face of the tile along D, once
#pragma unroll 1
  for (int f = tid; f < NFD; f += NT) {
    const int fc[3] = {f % F0, (f / F0) % F1, f / (F0 * F1)};
    int sl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int c[3] = {fc[0], fc[1], fc[2]};
      c[D] += k - 2;
      sl[k] = cell_slot<TX, TY, TZ, D>(c[0], c[1], c[2]);
    }
    double wl[6], wr[6];
    constexpr int perm[6] = {0, PN, P1, P2, 4, 5};
#pragma unroll
    for (int vv = 0; vv < NV; ++vv) {
      const double *col = sW + perm[vv] * SW;
      plm_face(col[sl[0]], col[sl[1]], col[sl[2]], col[sl[3]], wl[vv], wr[vv]);
    }
    int seedl = -1, seedr = -1;
    if (k_eos<PK>(p) == 1 && p.inv_mode != 0) {
      // seed each state from the table cell of its cell's centre (the nearest
      // tile cell where its cell is a halo cell)
      int tl[3] = {fc[0], fc[1], fc[2]}, tr[3] = {fc[0], fc[1], fc[2]};
      if (tl[D] > 0) tl[D] -= 1;
      if (tr[D] >= TD) tr[D] = TD - 1;
      seedl = sJc[tl[0] + TX * (tl[1] + TY * tl[2])];
      seedr = sJc[tr[0] + TX * (tr[1] + TY * tr[2])];
    }
    const int fr[3] = {T.to[0] + fc[0], T.to[1] + fc[1], T.to[2] + fc[2]};  // cell right of the face
    const int side = fr[D] == T.B.n;
    // block across a block face: a halo cell (layer -1 below, T_D above)
    const int nbo = (fr[D] == 0 || side) ? sB[(side ? sl[2] : sl[1]) - G::TV] : T.b;
    double Gf[7];
    if constexpr (k_gcache<PK>())
      face_flux<NV, D, PK>(a, T.B, T.fb, T.t, T.dtb, fr, wl, wr, seedl, seedr, nbo, Gf, sExc[sl[1]], sExc[sl[2]]);
    else
      face_flux<NV, D, PK>(a, T.B, T.fb, T.t, T.dtb, fr, wl, wr, seedl, seedr, nbo, Gf);
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[v * G::NF + f] = Gf[v];
    sF[6 * G::NF + f] = Gf[6];
  }
  __syncthreads();
  // own cell: divergence, gravity, neighbour energies (threads past the tile's
  // cells only stage and compute faces)
  if (tid < G::TV) {
    const int flo = cc[0] + F0 * (cc[1] + F1 * cc[2]);
    const int fhi = flo + FSTR;
    double Flo[7], Fhi[7];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Flo[v] = sF[v * G::NF + flo];
      Fhi[v] = sF[v * G::NF + fhi];
    }
    Flo[6] = sF[6 * G::NF + flo];
    Fhi[6] = sF[6 * G::NF + fhi];
    int cm[3] = {cc[0], cc[1], cc[2]}, cp[3] = {cc[0], cc[1], cc[2]};
    cm[D] -= 1;
    cp[D] += 1;
    if (D == 0) emax = fmax(emax, sW[6 * SW + tid]);  // own stage-input E
    const int lc[3] = {T.to[0] + cc[0], T.to[1] + cc[1], T.to[2] + cc[2]};
    const int sm = cell_slot<TX, TY, TZ, D>(cm[0], cm[1], cm[2]), sp = cell_slot<TX, TY, TZ, D>(cp[0], cp[1], cp[2]);
    if constexpr (k_gcache<PK>()) {
      const double phis[3] = {sPhi[sm], sPhi[tid], sPhi[sp]};
      axis_update<NV, D, PK>(a, T.B, T.t, lc, Flo, Fhi, sW[tid], sW[6 * SW + sm], sW[6 * SW + sp], rhs, divv, emax,
                             phis);
    } else {
      axis_update<NV, D, PK>(a, T.B, T.t, lc, Flo, Fhi, sW[tid], sW[6 * SW + sm], sW[6 * SW + sp], rhs, divv, emax);
    }
  }
  __syncthreads();
}

// NET: the learned network starts the output states' table-cell searches (a
// separate instantiation, so its matrix-core registers burden no other form)
// PK: physics switches (read at run time, or fixed: see k_eos)
// NT: threads per workgroup, 256 (one per cell) or 320 (every axis's faces in
// one round; the last wave only stages and computes faces).
template <int TX, int TY, int TZ, int NV, int OCC, bool NET, int NT, int PK>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(OCC, OCC))) void stage_tiled(StageArgs a_in) {
  using G = TileGeom<TX, TY, TZ>;
  static_assert(G::TV == kChunk, "one cell per thread");
  static_assert(NT == kChunk || NT >= G::NF, "a wide workgroup covers every axis's faces in one round");
  constexpr int SW = G::TV + G::HALO;
  __shared__ double sW[7 * SW];        // primitives (rho, vx, vy, vz, U_EOS, A) + stage-input E: own cells, halo
  __shared__ double sF[7 * G::NF];     // fluxes (rho, mx, my, mz, E, A) + face velocity
  __shared__ int sB[G::HALO];          // owning block of a halo cell, -1 beyond an outflow edge
  __shared__ int sJc[kChunk];          // table cell of each tile cell's centre state (seeds)
  __shared__ double sRed[NT / 64];     // per-wave CFL minima
  constexpr int GC = k_gcache<PK>() ? SW : 1;
  __shared__ double sPhi[GC];          // potential of the staged cells (compiled gravity kinds)
  __shared__ unsigned char sExc[GC];   // their excision flags
  const double dt0 = a_in.win[1];
  const double tk = a_in.win[0] + a_in.k * dt0;
  for (LevelItems it(a_in, a_in.item_start); it.valid(); it.next()) {
    // re-read per item on the kinds whose uniform values overflow the scalar
    // registers (the table EOS and the run-time kinds; measured: the
    // point-mass kind's stage 2.21 -> 2.16 ms, the ideal-gas kind 2.7 % slower)
    const StageArgs &a = (PK <= 0 || k_eos<PK>(a_in.p) == 1) ? kargs() : a_in;
    const Phys &p = a.p;
    const MeshDev &m = a.m;
    const int item = it.item;
    const int tid = item_tid();
    const int2 bt = a.item_bt[item];
    TileCtx T;
    T.b = uni(bt.x);
    T.B = uni(m.blocks[T.b]);
    const int n = T.B.n;
    const long long n3 = (long long)n * n * n;
    const int tile = uni(bt.y);
    const int ntx = n / TX, nty = n / TY;
    T.to[0] = (tile % ntx) * TX;
    T.to[1] = ((tile / ntx) % nty) * TY;
    T.to[2] = (tile / (ntx * nty)) * TZ;
    T.fb = uni(a.fac[T.b]);
    T.dtb = T.fb * dt0;
    T.t = a.phase == 1 ? tk : tk + T.dtb;
    T.own = own_source(a, uni(a.par[T.b]));
    const int cc[3] = {tid % TX, (tid / TX) % TY, tid / (TX * TY)};
    const int lc[3] = {T.to[0] + cc[0], T.to[1] + cc[1], T.to[2] + cc[2]};
    const long long cell = ((long long)lc[2] * n + lc[1]) * n + lc[0];
    // the tile's own cells, staged once for all three axes
    const bool has_cell = tid < G::TV;  // uniform per wave
    if (has_cell) {
      double q[6], w[6];
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = src_val(T.own, T.B.off + v * n3 + cell);
      c2p<PK>(p, q, w);
#pragma unroll
      for (int v = 0; v < NV; ++v) sW[v * SW + tid] = w[v];
      sW[6 * SW + tid] = q[IEN];
      if constexpr (k_gcache<PK>()) {
        sPhi[tid] = phi_at<PK>(a, T.B, lc[0], lc[1], lc[2], T.t);
        sExc[tid] = excised<PK>(p, m, T.B.ox + lc[0], T.B.oy + lc[1], T.B.oz + lc[2], T.t, lev_of<PK>(T.B)) ? 1 : 0;
      }
    }
    double rhs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double divv = 0.0, emax = -INFINITY;
    // seeded inversion: the table cell of each tile cell's stage-input state
    // starts the face and compression queries
    int jcell = -1;
    const int parb = uni(a.par[T.b]);
    if (has_cell && k_eos<PK>(p) == 1 && p.inv_mode != 0) {
      jcell = a.jc[jseg_in(a, parb) * a.jn + T.B.off / NV + cell];
      sJc[tid] = jcell;
    }
    tile_axis<TX, TY, TZ, NV, 0, NT, PK>(a, T, sW, sF, sB, sJc, rhs, divv, emax, sPhi, sExc);
    tile_axis<TX, TY, TZ, NV, 1, NT, PK>(a, T, sW, sF, sB, sJc, rhs, divv, emax, sPhi, sExc);
    tile_axis<TX, TY, TZ, NV, 2, NT, PK>(a, T, sW, sF, sB, sJc, rhs, divv, emax, sPhi, sExc);
    double cflv = INFINITY;
    if (has_cell) finish_cell<NV, NET, PK>(a, T.B, T.own, parb, T.dtb, tk, lc, cell, jcell, rhs, divv, emax, &cflv);
    if (a.cfl_part && a.phase == 2) {  // the tile's CFL minimum for the next reduction
      cflv = wave_min(cflv);
      if ((tid & 63) == 0) sRed[tid >> 6] = cflv;
      __syncthreads();
      if (tid == 0) {
        double r = sRed[0];
        for (int w = 1; w < NT / 64; ++w) r = fmin(r, sRed[w]);
        a.cfl_part[a.cfl_start[T.b] + tile] = r;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// split form: a kernel per axis computes every face flux of the active blocks
// into the flux arrays (one face per thread, no LDS, no barriers), then one
// kernel per cell sums them.  Same arithmetic as the fused form, bit for bit.
// Single-level meshes only (refined meshes run the fused form's kPkAmr kind).
// ---------------------------------------------------------------------------
// face (fi, fj, fk) of axis D: the D-th coordinate in [0, n], the others in
// [0, n), x fastest
template <int D>
__device__ __forceinline__ long long face_index(int n, int i, int j, int k) {
  const int ex = n + (D == 0), ey = n + (D == 1);
  return (long long)i + (long long)ex * (j + (long long)ey * k);
}

template <int NV, int D, int OCC>
__global__ __launch_bounds__(kChunk) __attribute__((amdgpu_waves_per_eu(OCC, OCC))) void face_kernel(StageArgs a_in) {
  constexpr int PN = 1 + D, P1 = 1 + (D + 1) % 3, P2 = 1 + (D + 2) % 3;
      const int a0 = a_in.cnt_ge[a_in.Lhi + 1], a1 = a_in.cnt_ge[a_in.Llo];
  if (a1 <= a0) return;
  const int i0 = a_in.fitem_start[a0], i1 = a_in.fitem_start[a1];
  const double dt0 = a_in.win[1];
  const double tk = a_in.win[0] + a_in.k * dt0;
  const int Nd = D == 0 ? a_in.m.nx : (D == 1 ? a_in.m.ny : a_in.m.nz);
  const ItemRange R = xcd_items(i0, i1);
  for (int item = R.first; item < R.end; item += R.step) {
    const StageArgs &a = kargs();  // re-read per item (as in stage_tiled)
    const Phys &p = a.p;
    const MeshDev &m = a.m;
    const int2 bt = a.fitem_bt[item];
    const int b = uni(bt.x);
    const BlockInfo B = uni(m.blocks[b]);
    const int n = B.n;
    const long long nf = (long long)(n + 1) * n * n;
    const long long f = (long long)uni(bt.y) * kChunk + item_tid();
    if (f >= nf) continue;
    const int fb = uni(a.fac[b]);
    const double dtb = fb * dt0;
    const double t = a.phase == 1 ? tk : tk + dtb;
    const Src own = own_source(a, uni(a.par[b]));
    const int ex = n + (D == 0), ey = n + (D == 1);
    const int fr[3] = {(int)(f % ex), (int)((f / ex) % ey), (int)(f / ((long long)ex * ey))};  // cell right of the face
    // the four cells of the stencil along D: primitives, and the block across a block face
    double W[4][6], wl[6], wr[6];
    int nbo = b;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int g[3] = {B.ox + fr[0], B.oy + fr[1], B.oz + fr[2]};
      g[D] += s - 2;
      double q[6];
      int nb_;
      long long id_;
      load_q<NV>(a, b, B, own, fb, g[0], g[1], g[2], q, &nb_, &id_);
      c2p(p, q, W[s]);
      if ((s == 1 && fr[D] == 0) || (s == 2 && fr[D] == n))
        nbo = (m.bc[D] == 0 || (g[D] >= 0 && g[D] < Nd)) ? nb_ : -1;
    }
    constexpr int perm[6] = {0, PN, P1, P2, 4, 5};
#pragma unroll
    for (int vv = 0; vv < NV; ++vv)
      plm_face(W[0][perm[vv]], W[1][perm[vv]], W[2][perm[vv]], W[3][perm[vv]], wl[vv], wr[vv]);
    int seedl = -1, seedr = -1;
    if (p.eos_kind == 1 && p.inv_mode != 0) {
      // seed each state from the table cell of the nearest own cell on its side of the face
      int tl[3] = {fr[0], fr[1], fr[2]}, tr[3] = {fr[0], fr[1], fr[2]};
      if (tl[D] > 0) tl[D] -= 1;
      if (tr[D] >= n) tr[D] = n - 1;
      const int parb = uni(a.par[b]);
      const long long base = jseg_in(a, parb) * a.jn + B.off / NV;
      seedl = a.jc[base + ((long long)tl[2] * n + tl[1]) * n + tl[0]];
      seedr = a.jc[base + ((long long)tr[2] * n + tr[1]) * n + tr[0]];
    }
    double Gf[7];
    face_flux<NV, D>(a, B, fb, t, dtb, fr, wl, wr, seedl, seedr, nbo, Gf);
    double *F = a.flx + D * a.fstride + (NV + 1) * B.foff;
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v * nf + f] = Gf[v];
    F[NV * nf + f] = Gf[6];
  }
}

// stage-input E of global cell g as the reader sees it
__device__ __forceinline__ double load_E(const StageArgs &a, int b, const BlockInfo &B, const Src &own, int fb, int gx,
                                         int gy, int gz) {
  const MeshDev &m = a.m;
  gx = wrap_axis(gx, m.nx, m.bc[0]);
  gy = wrap_axis(gy, m.ny, m.bc[1]);
  gz = wrap_axis(gz, m.nz, m.bc[2]);
  const int lx = gx - B.ox, ly = gy - B.oy, lz = gz - B.oz;
  if ((unsigned)lx < (unsigned)B.n && (unsigned)ly < (unsigned)B.n && (unsigned)lz < (unsigned)B.n) {
    const long long n3 = (long long)B.n * B.n * B.n;
    return src_val(own, B.off + IEN * n3 + ((long long)lz * B.n + ly) * B.n + lx);
  }
  const int nb = block_of(m, gx, gy, gz);
  const BlockInfo Bn = m.blocks[nb];
  const Src s = source_of(a, fb, nb);
  const long long n3 = (long long)Bn.n * Bn.n * Bn.n;
  return src_val(s, Bn.off + IEN * n3 + ((long long)(gz - Bn.oz) * Bn.n + (gy - Bn.oy)) * Bn.n + (gx - Bn.ox));
}

template <int NV, bool NET, int OCC>
__global__ __launch_bounds__(kChunk) __attribute__((amdgpu_waves_per_eu(OCC, OCC))) void update_kernel(StageArgs a_in) {
      const int a0 = a_in.cnt_ge[a_in.Lhi + 1], a1 = a_in.cnt_ge[a_in.Llo];
  if (a1 <= a0) return;
  const int i0 = a_in.item_start[a0], i1 = a_in.item_start[a1];
  const double dt0 = a_in.win[1];
  const double tk = a_in.win[0] + a_in.k * dt0;
  const ItemRange R = xcd_items(i0, i1);
  for (int item = R.first; item < R.end; item += R.step) {
    const StageArgs &a = kargs();  // re-read per item (as in stage_tiled)
    const Phys &p = a.p;
    const MeshDev &m = a.m;
    const int2 bt = a.item_bt[item];
    const int b = uni(bt.x);
    const BlockInfo B = uni(m.blocks[b]);
    const int n = B.n;
    const long long n3 = (long long)n * n * n;
    const long long cell = (long long)uni(bt.y) * kChunk + item_tid();
    const int fb = uni(a.fac[b]);
    const double dtb = fb * dt0;
    const double t = a.phase == 1 ? tk : tk + dtb;
    const Src own = own_source(a, uni(a.par[b]));
    const int parb = uni(a.par[b]);
    const int lc[3] = {(int)(cell % n), (int)((cell / n) % n), (int)(cell / ((long long)n * n))};
    const int g[3] = {B.ox + lc[0], B.oy + lc[1], B.oz + lc[2]};
    int jcell = -1;
    if (p.eos_kind == 1 && p.inv_mode != 0) jcell = a.jc[jseg_in(a, parb) * a.jn + B.off / NV + cell];
    const double rho = src_val(own, B.off + IDN * n3 + cell);
    double rhs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double divv = 0.0;
    double emax = src_val(own, B.off + IEN * n3 + cell);  // own stage-input E
    const long long nf = (long long)(n + 1) * n * n;
#define TDH_AXIS(D)                                                                                         \
    {                                                                                                       \
      const double *F = a.flx + D * a.fstride + (NV + 1) * B.foff;                                          \
      const long long flo = face_index<D>(n, lc[0], lc[1], lc[2]);                                          \
      const long long fhi = flo + (D == 0 ? 1 : (D == 1 ? (long long)n : (long long)n * n));                \
      double Flo[7], Fhi[7];                                                                                \
      _Pragma("unroll") for (int v = 0; v <= NV; ++v) {                                                     \
        Flo[v == NV ? 6 : v] = F[v * nf + flo];                                                             \
        Fhi[v == NV ? 6 : v] = F[v * nf + fhi];                                                             \
      }                                                                                                     \
      int gm[3] = {g[0], g[1], g[2]}, gp[3] = {g[0], g[1], g[2]};                                           \
      gm[D] -= 1;                                                                                           \
      gp[D] += 1;                                                                                           \
      const double Em = load_E(a, b, B, own, fb, gm[0], gm[1], gm[2]);                                      \
      const double Ep = load_E(a, b, B, own, fb, gp[0], gp[1], gp[2]);                                      \
      axis_update<NV, D>(a, B, t, lc, Flo, Fhi, rho, Em, Ep, rhs, divv, emax);                              \
    }
    TDH_AXIS(0)
    TDH_AXIS(1)
    TDH_AXIS(2)
#undef TDH_AXIS
    finish_cell<NV, NET>(a, B, own, parb, dtb, tk, lc, cell, jcell, rhs, divv, emax);
  }
}

// Table cell of every active cell's stage-input centre state, which seeds the
// stage kernel's face and compression queries; every start ends at the same,
// exact cell.  Modes 1 and 3 run it once after a state upload (afterwards each
// stage leaves the cells of its output for the next): mode 1 starts every
// search from the learned network's prediction (all three layers on the matrix
// cores), mode 3 bisects.  Modes 2 and 4 run it before every stage except a
// window's first when the CFL pass has recorded the cells of its state: a cell
// first tries the cell held for its previous state (for a second stage the
// stage input's, for a first stage the last stage-1 state's) and keeps it if it
// brackets; where it does not, or none is held, mode 2 bisects and mode 4
// searches from the network's prediction, which a wave evaluates when any of
// its cells needs it.  Blocks hold a multiple of 256 cells, so every wave is
// full when it calls the network.
template <int NV>
__global__ __launch_bounds__(kChunk) void seed_kernel(StageArgs a_in) {
  if (a_in.cnt_ge[a_in.Llo] <= a_in.cnt_ge[a_in.Lhi + 1]) return;
  const int nv = NV;
  const bool net = (a_in.p.inv_mode == 1 || a_in.p.inv_mode == 4) && a_in.s.enabled;
  // the network's weights, staged once per workgroup for all its items
  __shared__ __align__(16) short s_w2[64 * 64];
  __shared__ __align__(16) short s_w13[128 + 64];
  __shared__ __align__(16) float s_b[128 + 4];
  Seed sd = a_in.s;
  sd.w.w2b = s_w2;
  sd.w.w1b = s_w13;
  sd.w.w3b = s_w13 + 128;
  sd.w.b1 = s_b;
  sd.w.b2 = s_b + 64;
  sd.w.b3 = s_b + 128;
  if (net) {
    const int t = threadIdx.x;
    const uint4 *w2 = (const uint4 *)a_in.s.w.w2b;
    for (int k = t; k < 512; k += kChunk) ((uint4 *)s_w2)[k] = w2[k];
    if (t < 16) ((uint4 *)s_w13)[t] = ((const uint4 *)a_in.s.w.w1b)[t];
    else if (t < 24) ((uint4 *)s_w13)[t] = ((const uint4 *)a_in.s.w.w3b)[t - 16];
    else if (t < 40) ((uint4 *)s_b)[t - 24] = ((const uint4 *)a_in.s.w.b1)[t - 24];
    else if (t < 56) ((uint4 *)s_b)[t - 24] = ((const uint4 *)a_in.s.w.b2)[t - 40];
    else if (t == 56) s_b[128] = a_in.s.w.b3[0];
    __syncthreads();
  }
  for (LevelItems li(a_in, a_in.item_start); li.valid(); li.next()) {
    const StageArgs &a = kargs();  // re-read per item (as in stage_tiled)
    const Phys &p = a.p;
    const int2 bt = a.item_bt[li.item];
    const int b = uni(bt.x);
    const BlockInfo B = uni(a.m.blocks[b]);
    const long long n3 = (long long)B.n * B.n * B.n;
    const long long cell = (long long)uni(bt.y) * kChunk + threadIdx.x;
    const int parb = uni(a.par[b]);
    const Src own = own_source(a, parb);
    double q[6], w[6];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = src_val(own, B.off + v * n3 + cell);
    c2p(p, q, w);
    const double Ue = fmax(w[4], w[0] * p.e_floor);
    const double lr = log10_tab(a.t.lg, w[0]), le = log10_tab(a.t.lg, Ue / w[0]);
    int i, j = -1, it;
    double wr, wT;
    table_rho(a.t, lr, i, wr);
    if (p.inv_mode == 2 || p.inv_mode == 4) {
      // the cell held for the previous state: a second stage's input follows
      // the stage input's (segment of the block's current state), a first
      // stage's the last stage-1 state's (segment 2)
      const int prev = a.jc[(a.phase == 2 ? (long long)parb : 2LL) * a.jn + B.off / nv + cell];
      if (prev >= 0) {
        const int jj = min(prev, a.t.nT - 2);
        double lP, lc2;
        if (table_record(a.t, i, wr, le, jj, wT, lP, lc2)) j = jj;
      }
    }
    if (!net || (p.inv_mode == 4 && __ballot(j < 0) == 0)) {
      if (j < 0) table_invert(a.t, i, wr, le, -1, p.newton_max_iter, j, wT, it);
    } else {
      const int seed = seed_cell_wave<true>(sd, a.t, lr, le);  // the whole wave
      if (j < 0) table_invert(a.t, i, wr, le, seed, p.newton_max_iter, j, wT, it);
    }
    a.jc[jseg_in(a, parb) * a.jn + B.off / nv + cell] = j;
  }
}

// stage-kernel variants offered to the runtime: tile shape (x fastest; all
// divide blocks of edge >= 8), waves per SIMD the register budget targets,
// threads per workgroup
// (320-thread workgroups, every axis's faces in one round, measured 1.6x slower:
// at 168 registers only two such workgroups fit a CU)
#define TDH_TILES(X) X(8, 8, 4, 3, 256) X(16, 4, 4, 3, 256) X(4, 8, 8, 3, 256) X(8, 4, 8, 3, 256) \
                     X(16, 4, 4, 2, 256) X(8, 8, 4, 2, 256)

__global__ void set_window_kernel(double *win, double t, double dt0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    win[0] = t;
    win[1] = dt0;
  }
}

// (block, index of the item within the block) of every work item of a
// level-sorted block list: position i of the list owns the items
// start[i] .. start[i+1]-1
__global__ void expand_items_kernel(const int *order, const int *start, int nb, int2 *bt) {
  for (int i = blockIdx.x; i < nb; i += gridDim.x) {
    const int b = order[i], s0 = start[i], s1 = start[i + 1];
    for (int t = s0 + (int)threadIdx.x; t < s1; t += (int)blockDim.x) bt[t] = make_int2(b, t - s0);
  }
}

__global__ void commit_kernel(const int *order, const int *cnt_ge, int lmin, int *par) {
  const int na = cnt_ge[lmin];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += gridDim.x * blockDim.x) par[order[i]] ^= 1;
}

// Delayed flux correction for blocks completing now (eqs lat-flux-impulse,
// lat-mass-impulse-mismatch, lat-grav-reflux): against neighbours on the same
// refinement level that update more often, and against every finer neighbour,
// whose 2x2 face impulses (summed in u1, u0 order) replace the coarse face's
// own; never against a coarser neighbour.  One launch per axis so a cell
// touched by several faces is corrected in axis order without races.
__global__ void reflux_kernel(StageArgs a, int lc, int dir, int nmax) {
  const MeshDev &m = a.m;
  const int nv = m.nv;
  const int nc = a.cnt_ge[lc];
  const long long per = 2LL * nmax * nmax;
  const long long total = (long long)nc * per;
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
    const int r = B.lev;
    const int N[3] = {m.nx << r, m.ny << r, m.nz << r};
    int gg[3] = {B.ox + loc[0], B.oy + loc[1], B.oz + loc[2]};
    gg[dir] += side ? 1 : -1;
    if (m.bc[dir] != 0 && (gg[dir] < 0 || gg[dir] >= N[dir])) continue;
    for (int d = 0; d < 3; ++d) gg[d] = wrap_axis(gg[d], N[d], m.bc[d]);
    const int nb = block_of(m, r, gg[0], gg[1], gg[2]);
    const BlockInfo Bn = m.blocks[nb];
    if (Bn.lev < r || (Bn.lev == r && a.fac[nb] >= a.fac[b])) continue;
    const int w = Bn.lev > r ? 2 : 1;
    int h[3];  // the cell across (the first of the 2x2 fine face cells for a finer neighbour)
    for (int d = 0; d < 3; ++d) h[d] = w == 1 ? gg[d] : (d == dir ? 2 * gg[d] + (side ? 0 : 1) : 2 * gg[d]);
    const int ln[3] = {h[0] - Bn.ox, h[1] - Bn.oy, h[2] - Bn.oz};
    const int v0 = dir == 0 ? ln[1] : ln[0];
    const int v1 = dir == 2 ? ln[1] : ln[2];
    const int nn = Bn.n;
    double dI[6];
    for (int v = 0; v < nv; ++v) {
      const long long ib = B.ioff + ((long long)(2 * dir + side) * nv + v) * n * n + (long long)u1 * n + u0;
      const long long in = Bn.ioff + ((long long)(2 * dir + 1 - side) * nv + v) * nn * nn;
      double In = 0.0;
      for (int e1 = 0; e1 < w; ++e1)
        for (int e0 = 0; e0 < w; ++e0) In += a.imp[in + (long long)(v1 + e1) * nn + (v0 + e0)];
      dI[v] = a.imp[ib] - In;
    }
    const double vol = dx_lev(m, 0, r) * dx_lev(m, 1, r) * dx_lev(m, 2, r);
    const double sg = side ? 1.0 : -1.0;
    double *q = a.par[b] ? a.Qb : a.Qa;
    const long long n3 = (long long)n * n * n;
    const long long cidx = ((long long)loc[2] * n + loc[1]) * n + loc[0];
    if (a.p.grav_kind) {
      int lnb[3] = {loc[0], loc[1], loc[2]};
      lnb[dir] += side ? 1 : -1;
      const double pn = phi_at_block(a, B, lnb[0], lnb[1], lnb[2], tc);
      const double pi = phi_at_block(a, B, loc[0], loc[1], loc[2], tc);
      q[B.off + IEN * n3 + cidx] += sg / (2.0 * vol) * dI[IDN] * (pn - pi);
    }
    for (int v = 0; v < nv; ++v) q[B.off + v * n3 + cidx] += sg * dI[v] / vol;
  }
}

// ---------------------------------------------------------------------------
// CFL step: per-item minimum, then per-block minimum
// ---------------------------------------------------------------------------

// In modes 2 and 4 (table EOS) the pass also records each cell's table cell in
// its block's current segment: the seeds of the window's first stage, so no
// seed pass runs before it.
template <int NV>
__global__ __launch_bounds__(kChunk) void cfl_items_kernel(StageArgs a_in, double t, const int *item_block,
                                                           const int *block_item_start, int nitems, double *part) {
  __shared__ double red[kChunk / 64];
  const int nv = NV;
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const StageArgs &a = kargs();  // re-read per item (as in stage_tiled; the StageArgs is the first argument)
    const MeshDev &m = a.m;
    const Phys &p = a.p;
    const bool rec = p.eos_kind == 1 && (p.inv_mode == 2 || p.inv_mode == 4) && a.jc != nullptr;
    const int b = uni(item_block[item]);
    const BlockInfo B = uni(m.blocks[b]);
    const int n = B.n;
    const long long n3 = (long long)n * n * n;
    const long long cell = (long long)uni(item - block_item_start[b]) * kChunk + threadIdx.x;
    const bool inside = cell < n3;
    const long long cq = inside ? cell : n3 - 1;
    const int parb = uni(a.par[b]);
    const double *Q = parb ? a.Qb : a.Qa;
    double q[6], w[6];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = Q[B.off + v * n3 + cq];
    c2p(p, q, w);
    // the search starts from the cell the state's segment holds (carried, or
    // left by an earlier state of the block; -1 where none: bisection)
    const long long js = (long long)parb * a.jn + B.off / nv + cq;
    const int start = (p.eos_kind == 1 && p.inv_mode != 0 && a.jc) ? a.jc[js] : -1;
    double P, cs;
    int j = -1;
    eos_pc(p, a.t, w[0], w[4], start, P, cs, &j);
    if (rec && inside) a.jc[js] = j;
    double best = INFINITY;
    const int ci = (int)(cq % n), cj = (int)((cq / n) % n), ck = (int)(cq / ((long long)n * n));
    const int r = B.lev;
    const bool exc = p.grav_kind == 2 && p.r_exc > 0.0 && excised(p, m, B.ox + ci, B.oy + cj, B.oz + ck, t, r);
    if (inside && !exc) {
      for (int d = 0; d < 3; ++d) best = fmin(best, dx_lev(m, d, r) / (fabs(w[1 + d]) + cs));
      // source-term limit: sqrt(dx_min / |g|) with g the centred potential gradient
      if (p.grav_kind) {
        double g2 = 0.0;
        const int lc[3] = {ci, cj, ck};
        for (int d = 0; d < 3; ++d) {
          int ip[3] = {lc[0], lc[1], lc[2]}, im[3] = {lc[0], lc[1], lc[2]};
          ip[d] += 1;
          im[d] -= 1;
          const double gd = (phi_at_block(a, B, ip[0], ip[1], ip[2], t) - phi_at_block(a, B, im[0], im[1], im[2], t)) /
                            (2.0 * dx_lev(m, d, r));
          g2 += gd * gd;
        }
        const double dmin = fmin(dx_lev(m, 0, r), fmin(dx_lev(m, 1, r), dx_lev(m, 2, r)));
        if (g2 > 0.0) best = fmin(best, sqrt(dmin / sqrt(g2)));
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

// one wave per block: its lanes stride the block's item minima (a min is exact
// in any order)
__global__ void cfl_blocks_kernel(const double *part, const int *block_item_start, int nblocks, double cfl,
                                  double *dtb) {
  const int lane = threadIdx.x & 63, wpb = blockDim.x >> 6;
  for (int b = blockIdx.x * wpb + (threadIdx.x >> 6); b < nblocks; b += gridDim.x * wpb) {
    double r = INFINITY;
    for (int i = block_item_start[b] + lane; i < block_item_start[b + 1]; i += 64) r = fmin(r, part[i]);
    r = wave_min(r);
    if (lane == 0) dtb[b] = cfl * r;
  }
}

// ---------------------------------------------------------------------------
// batched EOS queries
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void eos_invert_kernel(Table t, Seed s, int maxit, const double *lr,
                                                         const double *le, double *lT, int32_t *jo, int32_t *iters,
                                                         long long n, int mode) {
  const long long nw = (n + 63) / 64;
  const long long wstride = ((long long)gridDim.x * blockDim.x) / 64;
  const int l = threadIdx.x & 63;
  for (long long wv = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / 64; wv < nw; wv += wstride) {
    const long long q = wv * 64 + l;  // the loop is uniform across the wave
    const bool ok = q < n;
    const double qlr = ok ? lr[q] : t.lr0, qle = ok ? le[q] : t.le2[0].x;
    int i, j, it;
    double w, wT;
    table_rho(t, qlr, i, w);
    int seed = -1;
    if (mode == 1) seed = seed_cell_wave(s, t, qlr, qle);
    if (mode == 2) {
      // the bisection result as the seed: the secant loop accepts it at once
      int jj, it2;
      double ww;
      table_invert(t, i, w, qle, -1, 0, jj, ww, it2);
      seed = jj;
    }
    table_invert(t, i, w, qle, seed, maxit, j, wT, it);
    if (ok) {
      if (lT) lT[q] = t.lT0 + (j + wT) * t.dlT;
      if (jo) jo[q] = j;
      if (iters) iters[q] = it;
    }
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
// split-form variants: waves per SIMD the face and the update kernels' registers target
#define TDH_SPLITS(X) X(4, 3) X(3, 3) X(5, 4)

// Variant ids: the fused tile shapes of TDH_TILES in order, then the split
// forms of TDH_SPLITS.
int num_tiles() {
  int n = 0;
#define TDH_COUNT(x, y, z, o, t) ++n;
  TDH_TILES(TDH_COUNT)
#undef TDH_COUNT
#define TDH_COUNT2(f, u) ++n;
  TDH_SPLITS(TDH_COUNT2)
#undef TDH_COUNT2
  return n;
}

void tile_shape(int id, int *dims) {
  int i = 0;
#define TDH_SHAPE(x, y, z, o, t)                           \
  if (i++ == id) {                                         \
    dims[0] = x; dims[1] = y; dims[2] = z; dims[3] = o;                      \
    return;                                                \
  }
  TDH_TILES(TDH_SHAPE)
#undef TDH_SHAPE
#define TDH_SHAPE2(f, u)                                   \
  if (i++ == id) {                                         \
    dims[0] = 0; dims[1] = f; dims[2] = u; dims[3] = 0;    \
    return;                                                \
  }
  TDH_SPLITS(TDH_SHAPE2)
#undef TDH_SHAPE2
  dims[0] = dims[1] = dims[2] = dims[3] = -1;
}

// Workgroups of a persistent launch: kRounds times as many as the chip holds
// at once (compute units x the workgroups of this kernel that one compute unit
// holds, which its registers and LDS decide).  Each workgroup walks a static
// share of the items; the dispatcher starts a new workgroup wherever one ends,
// so the smaller the shares, the less the shares' differing costs leave
// compute units idle at the end of a launch (measured on the stage kernel,
// rounds 1 .. 24: 2.15 ms at the former 8 workgroups per CU, 2.16 at one
// round, 1.91 at 16 and 1.89 at 24 on the production-shaped LAT run).
constexpr int kRounds = 16;

static int resident_grid(const void *kernel, int threads, int cus, int rounds = kRounds) {
  static std::mutex mu;
  static std::unordered_map<const void *, int> per_cu;
  std::lock_guard<std::mutex> lock(mu);
  const auto it = per_cu.find(kernel);
  if (it != per_cu.end()) return cus * it->second * rounds;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1)
    return cus * rounds;  // one workgroup per CU assumed (not kept: the query is tried again)
  per_cu.emplace(kernel, n);
  return cus * n * rounds;
}

// persistent launch of a kernel whose one argument is the StageArgs
template <typename K>
static hipError_t launch_persistent(K kernel, int threads, int cus, hipStream_t s, const StageArgs &a,
                                    int rounds = kRounds) {
  const void *k = reinterpret_cast<const void *>(kernel);
  StageArgs arg = a;
  void *argv[] = {&arg};
  return hipLaunchKernel(k, dim3(resident_grid(k, threads, cus, rounds)), dim3(threads), argv, 0, s);
}

template <int NV, int OF, int OU>
static hipError_t launch_split(const StageArgs &a, bool net, int cus, hipStream_t s) {
  hipError_t e;
  if ((e = launch_persistent(face_kernel<NV, 0, OF>, kChunk, cus, s, a)) != hipSuccess) return e;
  if ((e = launch_persistent(face_kernel<NV, 1, OF>, kChunk, cus, s, a)) != hipSuccess) return e;
  if ((e = launch_persistent(face_kernel<NV, 2, OF>, kChunk, cus, s, a)) != hipSuccess) return e;
  if (net) return launch_persistent(update_kernel<NV, true, OU>, kChunk, cus, s, a);
  return launch_persistent(update_kernel<NV, false, OU>, kChunk, cus, s, a);
}

// The seed pass takes 4 rounds: each of its workgroups first stages the
// network's weights (9 KB) in LDS, which more rounds repeat (measured on the
// production-shaped run: 2.29 ms of seed passes per window at 4 rounds, 2.51
// at 16).
constexpr int kSeedRounds = 4;

hipError_t launch_seed(const StageArgs &a, int cus, hipStream_t s) {
  if (a.m.nv == 6) return launch_persistent(seed_kernel<6>, kChunk, cus, s, a, kSeedRounds);
  return launch_persistent(seed_kernel<5>, kChunk, cus, s, a, kSeedRounds);
}

// Configurations with a stage kernel of their own (physics_code): the table
// EOS with dual energy and no gravity (HLLC, HLLE) in windows without levels,
// the same about a point mass under LAT (linear and dense-output ghosts), and
// the ideal gas in a fixed potential under LAT; the rest run the kernel that
// reads the switches.
#define TDH_KINDS(X) X(physics_code(1, 1, 0, 0, 0, 0), 6) X(physics_code(1, 1, 0, 1, 0, 0), 6) \
                     X(physics_code(1, 1, 2, 0, 0, 1), 6) X(physics_code(1, 1, 2, 0, 1, 1), 6) \
                     X(physics_code(0, 0, 1, 0, 0, 1), 5)

hipError_t launch_stage(const StageArgs &a, int tile, int cus, hipStream_t s) {
  int i = 0;
  // the network variant when it starts the searches (table EOS, mode 1, network on)
  const bool net = a.p.eos_kind == 1 && a.p.inv_mode == 1 && a.s.enabled;
  if (a.m.amr) {
    // Meshes with a refined block: one variant (8 x 8 x 4 cells), whatever the
    // tile; the production physics (table EOS, dual energy, point mass, levels,
    // linear ghosts) has a kind of its own, the rest read the switches (two
    // waves per SIMD: the cross-level ghost path needs the registers).
    constexpr int kAmrProd = physics_code(1, 1, 2, 0, 0, 1, 1);  // 3 waves per SIMD, as the single-level kind
    const int acode = a.m.nv != 5 + (a.p.dual ? 1 : 0)
                          ? 0
                          : physics_code(a.p.eos_kind, a.p.dual ? 1 : 0, a.p.grav_kind, a.p.riemann, a.p.ghost_dense,
                                         1, 1);
    if (!net && acode == kAmrProd) {
      return launch_persistent(stage_tiled<8, 8, 4, 6, 3, false, 256, kAmrProd>, 256, cus, s, a);
    }
    if (a.m.nv == 6) {
      if (net) return launch_persistent(stage_tiled<8, 8, 4, 6, 2, true, 256, kPkAmr>, 256, cus, s, a);
      else return launch_persistent(stage_tiled<8, 8, 4, 6, 2, false, 256, kPkAmr>, 256, cus, s, a);
    } else {
      if (net) return launch_persistent(stage_tiled<8, 8, 4, 5, 2, true, 256, kPkAmr>, 256, cus, s, a);
      else return launch_persistent(stage_tiled<8, 8, 4, 5, 2, false, 256, kPkAmr>, 256, cus, s, a);
    }
  }
  const int code = a.m.nv != 5 + (a.p.dual ? 1 : 0)
                       ? 0
                       : physics_code(a.p.eos_kind, a.p.dual ? 1 : 0, a.p.grav_kind, a.p.riemann, a.p.ghost_dense,
                                      a.lmax > 0 ? 1 : 0);
  // the network variant has a kernel of its own for the table EOS without gravity (HLLC)
  if (net && code == physics_code(1, 1, 0, 0, 0, 0)) {
#define TDH_NET_LAUNCH(x, y, z, o, t) \
    if (i++ == tile) return launch_persistent(stage_tiled<x, y, z, 6, o, true, t, physics_code(1, 1, 0, 0, 0, 0)>, t, cus, s, a);
    TDH_TILES(TDH_NET_LAUNCH)
#undef TDH_NET_LAUNCH
    i = 0;
  }
#define TDH_KIND_LAUNCH(c, nv) \
  if (!net && code == (c)) return launch_persistent(stage_tiled<X_, Y_, Z_, nv, O_, false, T_, (c)>, T_, cus, s, a);
#define TDH_LAUNCH(x, y, z, o, t)                                                                   \
  if (i++ == tile) {                                                                                \
    constexpr int X_ = x, Y_ = y, Z_ = z, O_ = o, T_ = t;                                           \
    TDH_KINDS(TDH_KIND_LAUNCH)                                                                      \
    if (net) {                                                                                      \
      if (a.m.nv == 6) return launch_persistent(stage_tiled<x, y, z, 6, o, true, t, 0>, t, cus, s, a);  \
      return launch_persistent(stage_tiled<x, y, z, 5, o, true, t, 0>, t, cus, s, a);                   \
    }                                                                                               \
    if (a.m.nv == 6) return launch_persistent(stage_tiled<x, y, z, 6, o, false, t, 0>, t, cus, s, a);   \
    return launch_persistent(stage_tiled<x, y, z, 5, o, false, t, 0>, t, cus, s, a);                    \
  }
  TDH_TILES(TDH_LAUNCH)
#undef TDH_LAUNCH
#undef TDH_KIND_LAUNCH
#define TDH_LAUNCH2(f, u)                                                                        \
  if (i++ == tile) return a.m.nv == 6 ? launch_split<6, f, u>(a, net, cus, s) : launch_split<5, f, u>(a, net, cus, s);
  TDH_SPLITS(TDH_LAUNCH2)
#undef TDH_LAUNCH2
  return hipErrorInvalidValue;
}

hipError_t launch_cfl_blocks(const double *part, int nblocks, const int *block_item_start, double cfl, double *dtb,
                             hipStream_t s) {
  const int bgrid = (nblocks + 3) / 4 < 1024 ? (nblocks + 3) / 4 : 1024;
  hipLaunchKernelGGL(cfl_blocks_kernel, dim3(bgrid), dim3(256), 0, s, part, block_item_start, nblocks, cfl, dtb);
  return hipGetLastError();
}

bool tile_is_fused(int id) {
  int n = 0;
#define TDH_COUNT(x, y, z, o, t) ++n;
  TDH_TILES(TDH_COUNT)
#undef TDH_COUNT
  return id >= 0 && id < n;
}

hipError_t launch_set_window(double *win, double t, double dt0, hipStream_t s) {
  hipLaunchKernelGGL(set_window_kernel, dim3(1), dim3(64), 0, s, win, t, dt0);
  return hipGetLastError();
}

hipError_t launch_expand_items(const int *order, const int *start, int nb, int2 *bt, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(expand_items_kernel, dim3(nb < 4096 ? nb : 4096), dim3(256), 0, s, order, start, nb, bt);
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
                      int nblocks, const int *block_item_start, double *dtb, int cus, hipStream_t s) {
  const int rg = resident_grid(a.m.nv == 6 ? reinterpret_cast<const void *>(cfl_items_kernel<6>)
                                           : reinterpret_cast<const void *>(cfl_items_kernel<5>),
                               kChunk, cus);
  const int grid = nitems < rg ? nitems : rg;
  if (a.m.nv == 6)
    hipLaunchKernelGGL(cfl_items_kernel<6>, dim3(grid), dim3(kChunk), 0, s, a, t, item_block, block_item_start,
                       nitems, part);
  else
    hipLaunchKernelGGL(cfl_items_kernel<5>, dim3(grid), dim3(kChunk), 0, s, a, t, item_block, block_item_start,
                       nitems, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int bgrid = (nblocks + 3) / 4 < 1024 ? (nblocks + 3) / 4 : 1024;
  hipLaunchKernelGGL(cfl_blocks_kernel, dim3(bgrid), dim3(256), 0, s, part, block_item_start, nblocks, cfl, dtb);
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
