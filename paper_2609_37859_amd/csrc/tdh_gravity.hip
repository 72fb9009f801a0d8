// Self-gravity (Sec. Self-gravity solver): geometric multigrid for the
// periodic Poisson problem A phi = S on the mesh's uniform grid, A = -lap_h the
// seven-point operator with the anisotropic weights the paper states
// (wy = (dx/dy)^2, wz = (dx/dz)^2, centre 2 (1 + wy + wz)) and
// S = -4 pi G (rho - mean rho) (eq selfgrav-poisson; the mean is removed so the
// periodic problem is solvable).
//
// V-cycle (the paper's order): two red-black Gauss-Seidel sweeps with
// over-relaxation 1.15, the defect d = S - A phi (eq selfgrav-defect) averaged
// over the eight children onto the coarser level, full-approximation coarse
// problem (start R phi, source R d + A_c R phi), the correction returned by
// tricubic interpolation, two post-sweeps; the coarsest level takes
// 2 (nx+ny+nz)^2 sweeps in one workgroup's LDS; one extra finest sweep ends
// each cycle.
//
// Every level is a dense [nz][ny][nx] array (x fastest) with periodic
// addressing; no ghost cells, so no ghost-fill launches.  Each level has even
// dimensions, so red (i+j+k even) and black cells are a true 2-colouring and
// a colour's cells update independently: one thread per cell of the colour,
// the same values as a sequential sweep.  Levels are HBM-bound stencils
// (about 24 bytes per cell and sweep at the finest level); coarse levels are
// launch-bound, which the host keeps cheap by capturing a cycle in a graph.
// Sums (mean density, defect norm, mean potential) use a fixed grid and a
// fixed tree, so they are deterministic.
#include "tdh_internal.hpp"

namespace tdh {

namespace {

constexpr double kOmegaGS = 1.15;
constexpr int kMgThreads = 256;

__device__ __forceinline__ int pwrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ long long at(const MgLevel &L, int i, int j, int k) {
  return ((long long)pwrap(k, L.nz) * L.ny + pwrap(j, L.ny)) * L.nx + pwrap(i, L.nx);
}

// ((x- + x+) + wy (y- + y+)) + wz (z- + z+)
__device__ __forceinline__ double nbsum(const MgLevel &L, const double *f, int i, int j, int k) {
#pragma clang fp contract(off)
  const double sx = f[at(L, i - 1, j, k)] + f[at(L, i + 1, j, k)];
  const double sy = f[at(L, i, j - 1, k)] + f[at(L, i, j + 1, k)];
  const double sz = f[at(L, i, j, k - 1)] + f[at(L, i, j, k + 1)];
  return (sx + L.wy * sy) + L.wz * sz;
}

__device__ __forceinline__ double apply_A(const MgLevel &L, const double *f, int i, int j, int k) {
#pragma clang fp contract(off)
  return (L.c0 * f[at(L, i, j, k)] - nbsum(L, f, i, j, k)) / L.hx2;
}

__device__ __forceinline__ double gs_value(const MgLevel &L, const double *phi, double src, int i, int j, int k,
                                           double old) {
#pragma clang fp contract(off)
  const double gs = (nbsum(L, phi, i, j, k) + L.hx2 * src) / L.c0;
  return (1.0 - kOmegaGS) * old + kOmegaGS * gs;
}

__device__ __forceinline__ double child_mean(const MgLevel &F, const double *f, int i, int j, int k) {
#pragma clang fp contract(off)
  const int I = 2 * i, J = 2 * j, K = 2 * k;
  const double a = f[at(F, I, J, K)] + f[at(F, I + 1, J, K)];
  const double b = f[at(F, I, J + 1, K)] + f[at(F, I + 1, J + 1, K)];
  const double c = f[at(F, I, J, K + 1)] + f[at(F, I + 1, J, K + 1)];
  const double d = f[at(F, I, J + 1, K + 1)] + f[at(F, I + 1, J + 1, K + 1)];
  return 0.125 * ((a + b) + (c + d));
}

__device__ __forceinline__ long long ncell(const MgLevel &L) { return (long long)L.nx * L.ny * L.nz; }

// cell (i, j, k) of the t-th cell of colour `color` (nx even)
__device__ __forceinline__ void color_cell(const MgLevel &L, long long t, int color, int &i, int &j, int &k) {
  const int hx = L.nx >> 1;
  const long long row = t / hx;
  j = (int)(row % L.ny);
  k = (int)(row / L.ny);
  i = 2 * (int)(t % hx) + ((j + k + color) & 1);
}

}  // namespace

__global__ __launch_bounds__(kMgThreads) void mg_gather_kernel(MeshDev m, const int *par, const double *Qa,
                                                                  const double *Qb, double *rho) {
  const long long n = (long long)m.nx * m.ny * m.nz;
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads) {
    const int i = (int)(p % m.nx), j = (int)((p / m.nx) % m.ny), k = (int)(p / ((long long)m.nx * m.ny));
    const int b = m.lmap[((k >> m.lat_shift) * m.ly + (j >> m.lat_shift)) * m.lx + (i >> m.lat_shift)];
    const BlockInfo B = m.blocks[b];
    const double *Q = par[b] ? Qb : Qa;
    rho[p] = Q[B.off + ((long long)(k - B.oz) * B.n + (j - B.oy)) * B.n + (i - B.ox)];
  }
}

// per-workgroup partial sums of x (or x^2) over a fixed grid-stride share
__global__ __launch_bounds__(kMgThreads) void mg_partial_sum_kernel(const double *x, long long n, int square,
                                                                       double *part) {
  __shared__ double red[kMgThreads];
  double s = 0.0;
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads) {
    const double v = x[p];
    s += square ? v * v : v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kMgThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = sum(part) * scale (op 0) or sqrt(sum(part) * scale) (op 1); one workgroup
__global__ __launch_bounds__(kMgThreads) void mg_final_sum_kernel(const double *part, int nparts, double scale,
                                                                     int op, double *out) {
  __shared__ double red[kMgThreads];
  double s = 0.0;
  for (int p = threadIdx.x; p < nparts; p += kMgThreads) s += part[p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kMgThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = op == 0 ? red[0] * scale : sqrt(red[0] * scale);
}

// src = -4 pi G (rho - mean); rho arrives in src
__global__ __launch_bounds__(kMgThreads) void mg_source_kernel(double *src, const double *mean, double four_pi_G,
                                                                  long long n) {
  const double mu = mean[0];
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads)
    src[p] = -four_pi_G * (src[p] - mu);
}

__global__ __launch_bounds__(kMgThreads) void mg_affine_kernel(double *x, const double *shift, double zero_fill,
                                                                  long long n) {
  // x -= shift[0] (shift non-null) or x = zero_fill
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads)
    x[p] = shift ? x[p] - shift[0] : zero_fill;
}

__global__ __launch_bounds__(kMgThreads) void mg_rbgs_kernel(MgLevel L, int color) {
  const long long half = ncell(L) >> 1;
  for (long long t = blockIdx.x * (long long)kMgThreads + threadIdx.x; t < half; t += (long long)gridDim.x * kMgThreads) {
    int i, j, k;
    color_cell(L, t, color, i, j, k);
    const long long p = at(L, i, j, k);
    L.phi[p] = gs_value(L, L.phi, L.src[p], i, j, k, L.phi[p]);
  }
}

__global__ __launch_bounds__(kMgThreads) void mg_defect_kernel(MgLevel L) {
  const long long n = ncell(L);
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads) {
    const int i = (int)(p % L.nx), j = (int)((p / L.nx) % L.ny), k = (int)(p / ((long long)L.nx * L.ny));
    L.tmp[p] = L.src[p] - apply_A(L, L.phi, i, j, k);
  }
}

// coarse start R phi (also kept in rphi) and the restricted defect
__global__ __launch_bounds__(kMgThreads) void mg_restrict_kernel(MgLevel F, MgLevel C) {
  const long long n = ncell(C);
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads) {
    const int i = (int)(p % C.nx), j = (int)((p / C.nx) % C.ny), k = (int)(p / ((long long)C.nx * C.ny));
    const double r = child_mean(F, F.phi, i, j, k);
    C.phi[p] = r;
    C.rphi[p] = r;
    C.src[p] = child_mean(F, F.tmp, i, j, k);
  }
}

// coarse source R d + A_c R phi
__global__ __launch_bounds__(kMgThreads) void mg_coarse_source_kernel(MgLevel C) {
  const long long n = ncell(C);
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads) {
    const int i = (int)(p % C.nx), j = (int)((p / C.nx) % C.ny), k = (int)(p / ((long long)C.nx * C.ny));
    C.src[p] = C.src[p] + apply_A(C, C.phi, i, j, k);
  }
}

// the coarsest level: `sweeps` red-black sweeps in one workgroup's LDS
constexpr int kMgCoarseMax = 2048;
__global__ __launch_bounds__(1024) void mg_coarse_solve_kernel(MgLevel C, int sweeps) {
  __shared__ double sphi[kMgCoarseMax], ssrc[kMgCoarseMax];
  const int n = (int)ncell(C);
  for (int p = threadIdx.x; p < n; p += 1024) {
    sphi[p] = C.phi[p];
    ssrc[p] = C.src[p];
  }
  __syncthreads();
  for (int s = 0; s < sweeps; ++s)
    for (int color = 0; color < 2; ++color) {
      for (int t = threadIdx.x; t < (n >> 1); t += 1024) {
        int i, j, k;
        color_cell(C, t, color, i, j, k);
        const int p = (int)at(C, i, j, k);
        sphi[p] = gs_value(C, sphi, ssrc[p], i, j, k, sphi[p]);
      }
      __syncthreads();
    }
  for (int p = threadIdx.x; p < n; p += 1024) C.phi[p] = sphi[p];
}

// correction (coarse result - R phi), in place of rphi
__global__ __launch_bounds__(kMgThreads) void mg_correction_kernel(MgLevel C) {
  const long long n = ncell(C);
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads)
    C.rphi[p] = C.phi[p] - C.rphi[p];
}

// fine phi += tricubic interpolation of the coarse correction: per axis the
// cubic through the four nearest coarse centres, weights (-5, 35, 105, -7)/128
// for the child at -1/4 of its parent (centres parent-2 .. parent+1) and
// (-7, 105, 35, -5)/128 for the child at +1/4 (parent-1 .. parent+2)
__global__ __launch_bounds__(kMgThreads) void mg_prolong_kernel(MgLevel F, MgLevel C) {
  const double wl[4] = {-5.0 / 128.0, 35.0 / 128.0, 105.0 / 128.0, -7.0 / 128.0};
  const double wr[4] = {-7.0 / 128.0, 105.0 / 128.0, 35.0 / 128.0, -5.0 / 128.0};
  const long long n = ncell(F);
  for (long long p = blockIdx.x * (long long)kMgThreads + threadIdx.x; p < n; p += (long long)gridDim.x * kMgThreads) {
    const int I = (int)(p % F.nx), J = (int)((p / F.nx) % F.ny), K = (int)(p / ((long long)F.nx * F.ny));
    const double *wx = (I & 1) ? wr : wl, *wy = (J & 1) ? wr : wl, *wz = (K & 1) ? wr : wl;
    const int i0 = (I >> 1) - ((I & 1) ? 1 : 2), j0 = (J >> 1) - ((J & 1) ? 1 : 2), k0 = (K >> 1) - ((K & 1) ? 1 : 2);
    double sz = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double sy = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        double sx = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) sx += wx[a] * C.rphi[at(C, i0 + a, j0 + b, k0 + c)];
        sy += wy[b] * sx;
      }
      sz += wz[c] * sy;
    }
    F.phi[p] += sz;
  }
}

// the per-block stored potential with one periodic ghost layer; blockIdx.y = block
__global__ __launch_bounds__(kMgThreads) void mg_scatter_kernel(MeshDev m, const double *phi, double *phib) {
  const BlockInfo B = m.blocks[blockIdx.y];
  const int np = B.n + 2;
  const int tot = np * np * np;
  for (int e = blockIdx.x * kMgThreads + threadIdx.x; e < tot; e += gridDim.x * kMgThreads) {
    const int i = e % np - 1, j = (e / np) % np - 1, k = e / (np * np) - 1;
    const int gx = pwrap(B.ox + i, m.nx), gy = pwrap(B.oy + j, m.ny), gz = pwrap(B.oz + k, m.nz);
    phib[B.poff + e] = phi[((long long)gz * m.ny + gy) * m.nx + gx];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int grid_for(long long n) {
  const long long g = (n + kMgThreads - 1) / kMgThreads;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

hipError_t mg_launch_gather(const MeshDev &m, const int *par, const double *Qa, const double *Qb, double *rho,
                            hipStream_t s) {
  hipLaunchKernelGGL(mg_gather_kernel, dim3(grid_for((long long)m.nx * m.ny * m.nz)), dim3(kMgThreads), 0, s, m, par,
                     Qa, Qb, rho);
  return hipGetLastError();
}

hipError_t mg_launch_sum(const double *x, long long n, int square, double scale, int op, double *part, double *out,
                         hipStream_t s) {
  hipLaunchKernelGGL(mg_partial_sum_kernel, dim3(kMgSumParts), dim3(kMgThreads), 0, s, x, n, square, part);
  hipLaunchKernelGGL(mg_final_sum_kernel, dim3(1), dim3(kMgThreads), 0, s, part, kMgSumParts, scale, op, out);
  return hipGetLastError();
}

hipError_t mg_launch_source(double *src, const double *mean, double four_pi_G, long long n, hipStream_t s) {
  hipLaunchKernelGGL(mg_source_kernel, dim3(grid_for(n)), dim3(kMgThreads), 0, s, src, mean, four_pi_G, n);
  return hipGetLastError();
}

hipError_t mg_launch_affine(double *x, const double *shift, double fill, long long n, hipStream_t s) {
  hipLaunchKernelGGL(mg_affine_kernel, dim3(grid_for(n)), dim3(kMgThreads), 0, s, x, shift, fill, n);
  return hipGetLastError();
}

hipError_t mg_launch_sweep(const MgLevel &L, hipStream_t s) {
  const long long half = ((long long)L.nx * L.ny * L.nz) >> 1;
  for (int color = 0; color < 2; ++color)
    hipLaunchKernelGGL(mg_rbgs_kernel, dim3(grid_for(half)), dim3(kMgThreads), 0, s, L, color);
  return hipGetLastError();
}

hipError_t mg_launch_defect(const MgLevel &L, hipStream_t s) {
  hipLaunchKernelGGL(mg_defect_kernel, dim3(grid_for((long long)L.nx * L.ny * L.nz)), dim3(kMgThreads), 0, s, L);
  return hipGetLastError();
}

hipError_t mg_launch_restrict(const MgLevel &F, const MgLevel &C, hipStream_t s) {
  const long long n = (long long)C.nx * C.ny * C.nz;
  hipLaunchKernelGGL(mg_restrict_kernel, dim3(grid_for(n)), dim3(kMgThreads), 0, s, F, C);
  hipLaunchKernelGGL(mg_coarse_source_kernel, dim3(grid_for(n)), dim3(kMgThreads), 0, s, C);
  return hipGetLastError();
}

hipError_t mg_launch_coarse_solve(const MgLevel &C, int sweeps, hipStream_t s) {
  if ((long long)C.nx * C.ny * C.nz > kMgCoarseMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mg_coarse_solve_kernel, dim3(1), dim3(1024), 0, s, C, sweeps);
  return hipGetLastError();
}

hipError_t mg_launch_prolong(const MgLevel &F, const MgLevel &C, hipStream_t s) {
  hipLaunchKernelGGL(mg_correction_kernel, dim3(grid_for((long long)C.nx * C.ny * C.nz)), dim3(kMgThreads), 0, s, C);
  hipLaunchKernelGGL(mg_prolong_kernel, dim3(grid_for((long long)F.nx * F.ny * F.nz)), dim3(kMgThreads), 0, s, F, C);
  return hipGetLastError();
}

hipError_t mg_launch_scatter(const MeshDev &m, int nblocks, int nmax, const double *phi, double *phib, hipStream_t s) {
  const int np = nmax + 2;
  const int gx = (np * np * np + kMgThreads - 1) / kMgThreads;
  hipLaunchKernelGGL(mg_scatter_kernel, dim3(gx, nblocks), dim3(kMgThreads), 0, s, m, phi, phib);
  return hipGetLastError();
}

int mg_coarse_max() { return kMgCoarseMax; }

}  // namespace tdh
