// Restart remap, Galilean boost and frame-acceleration estimate
// (Sec. Domain remapping and frame conversion, eqs remap-state-vector,
// remap-cell-average, galilean-boost; Sec. Moving-frame dynamics and BH
// treatment, eq frame-acceleration).
//
// Remap: one thread per target cell.  A target cell inside the excision
// sphere takes the sink state and one whose centre lies outside the source
// domain along a non-periodic axis the floor state; within kBand source cells
// inside a source face beyond which the target domain extends, the remapped
// density, momentum and thermal energy density are blended toward the floor
// state (at rest) with the weight s = 3u^2 - 2u^3 of the distance u to the
// nearest such face in band widths, so density and pressure reach the floor
// smoothly at the old domain's edge; on a target grid that
// coincides with the source grid (same spacing, origin a whole number of
// cells away) the source cell's conserved values are copied; otherwise the
// cell averages the trilinear interpolant of the source density, momentum and
// thermal energy density (the auxiliary energy with dual energy on,
// E - |m|^2/2rho otherwise) over its eight sub-cell midpoints, and rebuilds
// E = U + |m|^2/2rho (and U_aux = U).  Source neighbours are found through the
// source mesh's lattice map and read in place from its current buffers;
// stencils clamp at non-periodic source edges and wrap across periodic ones.
// HBM-bound: a target cell writes nv doubles and its samples read about one
// source cell's worth of new data (neighbouring targets share their stencils
// through the caches).
#include "tdh_internal.hpp"

namespace tdh {

namespace {
constexpr int kRmThreads = 256;

struct SrcView {
  MeshDev m;
  const int *par;
  const double *Qa, *Qb;
};

__device__ __forceinline__ int src_axis(int i, int n, int periodic) {
  if (periodic) return i < 0 ? i + n * ((-i + n - 1) / n) : i % n;
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// conserved values (nv) of global source cell (i, j, k), in-range indices
template <int NV>
__device__ __forceinline__ void src_cell(const SrcView &S, int i, int j, int k, double *q) {
  const MeshDev &m = S.m;
  const int b = m.lmap[((k >> m.lat_shift) * m.ly + (j >> m.lat_shift)) * m.lx + (i >> m.lat_shift)];
  const BlockInfo B = m.blocks[b];
  const double *Q = S.par[b] ? S.Qb : S.Qa;
  const long long n3 = (long long)B.n * B.n * B.n;
  const long long l = ((long long)(k - B.oz) * B.n + (j - B.oy)) * B.n + (i - B.ox);
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = Q[B.off + v * n3 + l];
}

// rho, mx, my, mz, U_th of a source cell
template <int NV>
__device__ __forceinline__ void src_fields(const SrcView &S, int i, int j, int k, double *f) {
#pragma clang fp contract(off)
  double q[6];
  src_cell<NV>(S, i, j, k, q);
  f[0] = q[0];
  f[1] = q[1];
  f[2] = q[2];
  f[3] = q[3];
  if (NV > 5) {
    f[4] = q[5];
  } else {
    const double K = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
    f[4] = q[4] - K;
  }
}

// trilinear interpolant of the five fields at point r (x, then y, then z)
template <int NV>
__device__ __forceinline__ void trilinear5(const SrcView &S, const double *r, double *out) {
#pragma clang fp contract(off)
  const int N[3] = {S.m.nx, S.m.ny, S.m.nz};
  int i0[3], i1[3];
  double w[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double xi = (r[d] - S.m.x0[d]) / S.m.dx[d] - 0.5;
    const double fl = floor(xi);
    w[d] = xi - fl;
    const int il = (int)fmin(fmax(fl, -1e9), 1e9);  // far-off points stay in int range (and NaN too)
    i0[d] = src_axis(il, N[d], S.m.bc[d] == 0);
    i1[d] = src_axis(il + 1, N[d], S.m.bc[d] == 0);
  }
  double c000[5], c100[5], c010[5], c110[5], c001[5], c101[5], c011[5], c111[5];
  src_fields<NV>(S, i0[0], i0[1], i0[2], c000);
  src_fields<NV>(S, i1[0], i0[1], i0[2], c100);
  src_fields<NV>(S, i0[0], i1[1], i0[2], c010);
  src_fields<NV>(S, i1[0], i1[1], i0[2], c110);
  src_fields<NV>(S, i0[0], i0[1], i1[2], c001);
  src_fields<NV>(S, i1[0], i0[1], i1[2], c101);
  src_fields<NV>(S, i0[0], i1[1], i1[2], c011);
  src_fields<NV>(S, i1[0], i1[1], i1[2], c111);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double a00 = (1.0 - w[0]) * c000[v] + w[0] * c100[v];
    const double a10 = (1.0 - w[0]) * c010[v] + w[0] * c110[v];
    const double a01 = (1.0 - w[0]) * c001[v] + w[0] * c101[v];
    const double a11 = (1.0 - w[0]) * c011[v] + w[0] * c111[v];
    const double b0 = (1.0 - w[1]) * a00 + w[1] * a10;
    const double b1 = (1.0 - w[1]) * a01 + w[1] * a11;
    out[v] = (1.0 - w[2]) * b0 + w[2] * b1;
  }
}

__device__ __forceinline__ bool excised_at(const Phys &p, const double *r, double t) {
  if (p.grav_kind != 2 || !(p.r_exc > 0.0)) return false;
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double q = r[d] - (p.bh_x0[d] - p.v_frame[d] * t);
    s += q * q;
  }
  return s < p.r_exc * p.r_exc;
}

__device__ __forceinline__ double u_floor_of(const Phys &p, double rho) {
  return p.eos_kind == 0 ? p.p_floor / (p.gamma - 1.0) : rho * p.e_floor;
}

constexpr double kBand = 2.0;  // width of the blending band in source cells

// blending weight of target centre c (inside the source domain): 1 away from the
// source faces the target domain extends beyond, falling smoothly to 0 at them
__device__ __forceinline__ double band_weight(const MeshDev &S, const MeshDev &D, const double *c) {
#pragma clang fp contract(off)
  const int NS[3] = {S.nx, S.ny, S.nz}, ND[3] = {D.nx, D.ny, D.nz};
  double u = 1.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (S.bc[a] == 0) continue;
    const double lo = S.x0[a], hi = S.x0[a] + NS[a] * S.dx[a];
    const double dlo = D.x0[a], dhi = D.x0[a] + ND[a] * D.dx[a];
    const double w = kBand * S.dx[a];
    if (dlo < lo) u = fmin(u, (c[a] - lo) / w);
    if (dhi > hi) u = fmin(u, (hi - c[a]) / w);
  }
  if (u <= 0.0) return 0.0;
  if (u >= 1.0) return 1.0;
  return u * u * (3.0 - 2.0 * u);
}
}  // namespace

template <int NV>
__global__ __launch_bounds__(kRmThreads) void remap_kernel(SrcView S, MeshDev D, double *Qd, Phys p, double t,
                                                            int coincident, int sx, int sy, int sz) {
  const long long n = (long long)D.nx * D.ny * D.nz;
  for (long long g = blockIdx.x * (long long)kRmThreads + threadIdx.x; g < n; g += (long long)gridDim.x * kRmThreads) {
    const int gi[3] = {(int)(g % D.nx), (int)((g / D.nx) % D.ny), (int)(g / ((long long)D.nx * D.ny))};
    double c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = D.x0[d] + (gi[d] + 0.5) * D.dx[d];
    const int NS[3] = {S.m.nx, S.m.ny, S.m.nz};
    bool outside = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double lo = S.m.x0[d], hi = S.m.x0[d] + NS[d] * S.m.dx[d];
      if (S.m.bc[d] != 0 && (c[d] < lo || c[d] >= hi)) outside = true;
    }
    double q[6], uth0 = 0.0;  // conserved state; its thermal energy density
    const bool sink = excised_at(p, c, t);
    if (sink || outside) {
      const double uf = u_floor_of(p, p.rho_floor);
      q[0] = p.rho_floor;
      q[1] = q[2] = q[3] = 0.0;
      q[4] = uf;
      q[5] = uf;
    } else if (coincident) {
      const int sh[3] = {sx, sy, sz};
      int si[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) si[d] = src_axis(gi[d] + sh[d], NS[d], S.m.bc[d] == 0);
      src_cell<NV>(S, si[0], si[1], si[2], q);
      uth0 = NV > 5 ? q[5] : q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
    } else {
#pragma clang fp contract(off)
      double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
      for (int s = 0; s < 8; ++s) {
        const int ox = s & 1, oy = (s >> 1) & 1, oz = s >> 2;  // z outer, x inner
        const double r[3] = {c[0] + (ox ? 0.25 : -0.25) * D.dx[0], c[1] + (oy ? 0.25 : -0.25) * D.dx[1],
                             c[2] + (oz ? 0.25 : -0.25) * D.dx[2]};
        double f[5];
        trilinear5<NV>(S, r, f);
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += f[v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] *= 0.125;
      q[0] = acc[0];
      q[1] = acc[1];
      q[2] = acc[2];
      q[3] = acc[3];
      q[4] = acc[4] + 0.5 * (acc[1] * acc[1] + acc[2] * acc[2] + acc[3] * acc[3]) / acc[0];
      q[5] = acc[4];
      uth0 = acc[4];
    }
    if (!sink && !outside) {
#pragma clang fp contract(off)
      const double w = band_weight(S.m, D, c);
      if (w < 1.0) {
        const double uf = u_floor_of(p, p.rho_floor);
        const double rho = w * q[0] + (1.0 - w) * p.rho_floor;
        const double m0 = w * q[1], m1 = w * q[2], m2 = w * q[3];
        const double uth = w * uth0 + (1.0 - w) * uf;
        q[0] = rho;
        q[1] = m0;
        q[2] = m1;
        q[3] = m2;
        q[4] = uth + 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho;
        q[5] = uth;
      }
    }
    const int b = D.lmap[((gi[2] >> D.lat_shift) * D.ly + (gi[1] >> D.lat_shift)) * D.lx + (gi[0] >> D.lat_shift)];
    const BlockInfo B = D.blocks[b];
    const long long n3 = (long long)B.n * B.n * B.n;
    const long long l = ((long long)(gi[2] - B.oz) * B.n + (gi[1] - B.oy)) * B.n + (gi[0] - B.ox);
#pragma unroll
    for (int v = 0; v < NV; ++v) Qd[B.off + v * n3 + l] = q[v];
  }
}

// Galilean boost of the current state, in place (floor-density cells skipped)
template <int NV>
__global__ __launch_bounds__(kRmThreads) void boost_kernel(MeshDev m, const int *par, double *Qa, double *Qb,
                                                           double V0, double V1, double V2, double rho_skip) {
  const long long n = (long long)m.nx * m.ny * m.nz;
  for (long long g = blockIdx.x * (long long)kRmThreads + threadIdx.x; g < n; g += (long long)gridDim.x * kRmThreads) {
    const int i = (int)(g % m.nx), j = (int)((g / m.nx) % m.ny), k = (int)(g / ((long long)m.nx * m.ny));
    const int b = m.lmap[((k >> m.lat_shift) * m.ly + (j >> m.lat_shift)) * m.lx + (i >> m.lat_shift)];
    const BlockInfo B = m.blocks[b];
    double *Q = (par[b] ? Qb : Qa) + B.off;
    const long long n3 = (long long)B.n * B.n * B.n;
    const long long l = ((long long)(k - B.oz) * B.n + (j - B.oy)) * B.n + (i - B.ox);
    const double rho = Q[l];
    if (!(rho > rho_skip)) continue;
    const double mx = Q[n3 + l], my = Q[2 * n3 + l], mz = Q[3 * n3 + l];
    const double mv = (mx * V0 + my * V1) + mz * V2;
    const double v2 = (V0 * V0 + V1 * V1) + V2 * V2;
    Q[4 * n3 + l] = (Q[4 * n3 + l] + mv) + 0.5 * rho * v2;
    Q[n3 + l] = mx + rho * V0;
    Q[2 * n3 + l] = my + rho * V1;
    Q[3 * n3 + l] = mz + rho * V2;
  }
}

// partial sums of rho, rho g (x, y, z) over dense non-excised cells; a fixed
// grid of kRmParts workgroups, then one workgroup sums the partials
constexpr int kRmParts = 1024;
__global__ __launch_bounds__(kRmThreads) void frame_acc_partial_kernel(MeshDev m, const int *par, const double *Qa,
                                                                       const double *Qb, Phys p, double t,
                                                                       double rho_min, double *part) {
  __shared__ double red[4][kRmThreads];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  const long long n = (long long)m.nx * m.ny * m.nz;
  for (long long g = blockIdx.x * (long long)kRmThreads + threadIdx.x; g < n; g += (long long)gridDim.x * kRmThreads) {
    const int i = (int)(g % m.nx), j = (int)((g / m.nx) % m.ny), k = (int)(g / ((long long)m.nx * m.ny));
    const int b = m.lmap[((k >> m.lat_shift) * m.ly + (j >> m.lat_shift)) * m.lx + (i >> m.lat_shift)];
    const BlockInfo B = m.blocks[b];
    const double *Q = (par[b] ? Qb : Qa) + B.off;
    const double rho = Q[((long long)(k - B.oz) * B.n + (j - B.oy)) * B.n + (i - B.ox)];
    const double c[3] = {m.x0[0] + (i + 0.5) * m.dx[0], m.x0[1] + (j + 0.5) * m.dx[1], m.x0[2] + (k + 0.5) * m.dx[2]};
    if (!(rho > rho_min) || excised_at(p, c, t)) continue;
    double dr[3], r2 = p.r_soft * p.r_soft;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      dr[d] = c[d] - (p.bh_x0[d] - p.v_frame[d] * t);
      r2 += dr[d] * dr[d];
    }
    const double f = -p.gm_bh / (r2 * sqrt(r2));
    s[0] += rho;
#pragma unroll
    for (int d = 0; d < 3; ++d) s[1 + d] += rho * (f * dr[d]);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[v][threadIdx.x] = s[v];
  __syncthreads();
  for (int w = kRmThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[threadIdx.x * kRmParts + blockIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kRmThreads) void frame_acc_final_kernel(const double *part, double *out) {
  __shared__ double red[4][kRmThreads];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < kRmParts; q += kRmThreads)
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] += part[v * kRmParts + q];
#pragma unroll
  for (int v = 0; v < 4; ++v) red[v][threadIdx.x] = s[v];
  __syncthreads();
  for (int w = kRmThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[0][0] > 0.0 ? red[1 + threadIdx.x][0] / red[0][0] : 0.0;
}

static int rm_grid(long long n) {
  const long long g = (n + kRmThreads - 1) / kRmThreads;
  return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t launch_remap(const MeshDev &src, const int *src_par, const double *sQa, const double *sQb,
                        const MeshDev &dst, double *Qd, const Phys &p, double t, int nv, int coincident,
                        const int *shift, hipStream_t s) {
  SrcView S{src, src_par, sQa, sQb};
  const long long n = (long long)dst.nx * dst.ny * dst.nz;
  if (nv == 6)
    hipLaunchKernelGGL((remap_kernel<6>), dim3(rm_grid(n)), dim3(kRmThreads), 0, s, S, dst, Qd, p, t, coincident,
                       shift[0], shift[1], shift[2]);
  else
    hipLaunchKernelGGL((remap_kernel<5>), dim3(rm_grid(n)), dim3(kRmThreads), 0, s, S, dst, Qd, p, t, coincident,
                       shift[0], shift[1], shift[2]);
  return hipGetLastError();
}

hipError_t launch_boost(const MeshDev &m, const int *par, double *Qa, double *Qb, int nv, const double *V,
                        double rho_skip, hipStream_t s) {
  const long long n = (long long)m.nx * m.ny * m.nz;
  if (nv == 6)
    hipLaunchKernelGGL((boost_kernel<6>), dim3(rm_grid(n)), dim3(kRmThreads), 0, s, m, par, Qa, Qb, V[0], V[1], V[2],
                       rho_skip);
  else
    hipLaunchKernelGGL((boost_kernel<5>), dim3(rm_grid(n)), dim3(kRmThreads), 0, s, m, par, Qa, Qb, V[0], V[1], V[2],
                       rho_skip);
  return hipGetLastError();
}

hipError_t launch_frame_acceleration(const MeshDev &m, const int *par, const double *Qa, const double *Qb,
                                     const Phys &p, double t, double rho_min, double *part, double *out,
                                     hipStream_t s) {
  hipLaunchKernelGGL(frame_acc_partial_kernel, dim3(kRmParts), dim3(kRmThreads), 0, s, m, par, Qa, Qb, p, t, rho_min,
                     part);
  hipLaunchKernelGGL(frame_acc_final_kernel, dim3(1), dim3(kRmThreads), 0, s, part, out);
  return hipGetLastError();
}

int frame_acceleration_parts() { return kRmParts; }

}  // namespace tdh
