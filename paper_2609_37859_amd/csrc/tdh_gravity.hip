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
// Every level is stored in red-black order: the red cells (i+j+k even) first,
// then the black ones, each colour as [nz][ny][nx/2] with x fastest, and
// addressed periodically (no ghost cells, so no ghost-fill launches).  Each
// level has even dimensions, so the colours are a true 2-colouring and a
// colour's cells update independently: one thread per cell of the colour,
// the same values as a sequential sweep, reading and writing its colour's
// half contiguously and its neighbours from the other half.  Levels are HBM-bound stencils
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

__device__ __forceinline__ long long ncell(const MgLevel &L) { return (long long)L.nx * L.ny * L.nz; }

// storage index of cell (i, j, k), offsets of up to two cells wrapped
__device__ __forceinline__ long long at(const MgLevel &L, int i, int j, int k) {
  i = pwrap(i, L.nx);
  j = pwrap(j, L.ny);
  k = pwrap(k, L.nz);
  const long long nat = ((long long)k * L.ny + j) * L.nx + i;
  return ((i + j + k) & 1) * (ncell(L) >> 1) + (nat >> 1);
}

// cell of storage index q
__device__ __forceinline__ void cell_of(const MgLevel &L, long long q, int &i, int &j, int &k) {
  const long long half = ncell(L) >> 1;
  const int color = q >= half;
  const long long r = q - color * half;
  const int hx = L.nx >> 1;
  const long long row = r / hx;
  j = (int)(row % L.ny);
  k = (int)(row / L.ny);
  i = 2 * (int)(r % hx) + ((j + k + color) & 1);
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


}  // namespace

// the density of every cell into the finest level's source array
__global__ __launch_bounds__(kMgThreads) void mg_gather_kernel(MeshDev m, const int *par, const double *Qa,
                                                                  const double *Qb, MgLevel F) {
  const long long n = ncell(F);
  for (long long q = blockIdx.x * (long long)kMgThreads + threadIdx.x; q < n; q += (long long)gridDim.x * kMgThreads) {
    int i, j, k;
    cell_of(F, q, i, j, k);
    const int b = m.lmap[((k >> m.lat_shift) * m.ly + (j >> m.lat_shift)) * m.lx + (i >> m.lat_shift)];
    const BlockInfo B = m.blocks[b];
    const double *Q = par[b] ? Qb : Qa;
    F.src[q] = Q[B.off + ((long long)(k - B.oz) * B.n + (j - B.oy)) * B.n + (i - B.ox)];
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
    const long long q = color * half + t;
    int i, j, k;
    cell_of(L, q, i, j, k);
    L.phi[q] = gs_value(L, L.phi, L.src[q], i, j, k, L.phi[q]);
  }
}

__device__ __forceinline__ double defect_at(const MgLevel &L, int i, int j, int k) {
  return L.src[at(L, i, j, k)] - apply_A(L, L.phi, i, j, k);
}

// per-workgroup partial sums of the squared defect over the same fixed
// grid-stride shares as mg_partial_sum_kernel (the defect is not stored)
__global__ __launch_bounds__(kMgThreads) void mg_defect_sq_partial_kernel(MgLevel L, double *part) {
  __shared__ double red[kMgThreads];
  const long long n = ncell(L);
  double s = 0.0;
  for (long long q = blockIdx.x * (long long)kMgThreads + threadIdx.x; q < n; q += (long long)gridDim.x * kMgThreads) {
    int i, j, k;
    cell_of(L, q, i, j, k);
    const double d = L.src[q] - apply_A(L, L.phi, i, j, k);
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kMgThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// coarse start R phi (also kept in rphi) and the restricted defect, the
// children's defects computed here (the same values and order of summation
// as a stored defect averaged over the eight children)
__global__ __launch_bounds__(kMgThreads) void mg_restrict_kernel(MgLevel F, MgLevel C) {
  const long long n = ncell(C);
  for (long long q = blockIdx.x * (long long)kMgThreads + threadIdx.x; q < n; q += (long long)gridDim.x * kMgThreads) {
    int i, j, k;
    cell_of(C, q, i, j, k);
    const double r = child_mean(F, F.phi, i, j, k);
    C.phi[q] = r;
    C.rphi[q] = r;
    const int I = 2 * i, J = 2 * j, K = 2 * k;
    double dm;
    {
#pragma clang fp contract(off)
      const double a = defect_at(F, I, J, K) + defect_at(F, I + 1, J, K);
      const double b = defect_at(F, I, J + 1, K) + defect_at(F, I + 1, J + 1, K);
      const double c = defect_at(F, I, J, K + 1) + defect_at(F, I + 1, J, K + 1);
      const double d = defect_at(F, I, J + 1, K + 1) + defect_at(F, I + 1, J + 1, K + 1);
      dm = 0.125 * ((a + b) + (c + d));
    }
    C.src[q] = dm;
  }
}

// coarse source R d + A_c R phi
__global__ __launch_bounds__(kMgThreads) void mg_coarse_source_kernel(MgLevel C) {
  const long long n = ncell(C);
  for (long long q = blockIdx.x * (long long)kMgThreads + threadIdx.x; q < n; q += (long long)gridDim.x * kMgThreads) {
    int i, j, k;
    cell_of(C, q, i, j, k);
    C.src[q] = C.src[q] + apply_A(C, C.phi, i, j, k);
  }
}

// the coarsest level: `sweeps` red-black sweeps in one workgroup's LDS; with at
// most 2048 cells every thread owns at most one cell of each colour, whose
// neighbour slots it finds once
constexpr int kMgCoarseMax = 2048;
__global__ __launch_bounds__(1024) void mg_coarse_solve_kernel(MgLevel C, int sweeps) {
  __shared__ double sphi[kMgCoarseMax], ssrc[kMgCoarseMax];
  const int n = (int)ncell(C), half = n >> 1;
  for (int p = threadIdx.x; p < n; p += 1024) {
    sphi[p] = C.phi[p];
    ssrc[p] = C.src[p];
  }
  const bool own = (int)threadIdx.x < half;
  int q[2] = {0, 0}, nb[2][6];
  if (own) {
#pragma unroll
    for (int color = 0; color < 2; ++color) {
      int i, j, k;
      q[color] = color * half + threadIdx.x;
      cell_of(C, q[color], i, j, k);
      nb[color][0] = (int)at(C, i - 1, j, k);
      nb[color][1] = (int)at(C, i + 1, j, k);
      nb[color][2] = (int)at(C, i, j - 1, k);
      nb[color][3] = (int)at(C, i, j + 1, k);
      nb[color][4] = (int)at(C, i, j, k - 1);
      nb[color][5] = (int)at(C, i, j, k + 1);
    }
  }
  __syncthreads();
  for (int s = 0; s < sweeps; ++s) {
#pragma unroll
    for (int color = 0; color < 2; ++color) {
      if (own) {
#pragma clang fp contract(off)
        const int *g = nb[color];
        const double sx = sphi[g[0]] + sphi[g[1]];
        const double sy = sphi[g[2]] + sphi[g[3]];
        const double sz = sphi[g[4]] + sphi[g[5]];
        const double nbs = (sx + C.wy * sy) + C.wz * sz;
        const double gs = (nbs + C.hx2 * ssrc[q[color]]) / C.c0;
        sphi[q[color]] = (1.0 - kOmegaGS) * sphi[q[color]] + kOmegaGS * gs;
      }
      __syncthreads();
    }
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
// (-7, 105, 35, -5)/128 for the child at +1/4 (parent-1 .. parent+2), summed
// along x, then y, then z.  One thread per coarse cell makes its eight
// children from the 5 x 5 x 5 coarse neighbourhood they share (125 loads
// instead of 512), keeping that order of summation for each child.
__global__ __launch_bounds__(kMgThreads) void mg_prolong_kernel(MgLevel F, MgLevel C) {
  const double w[2][4] = {{-5.0 / 128.0, 35.0 / 128.0, 105.0 / 128.0, -7.0 / 128.0},
                          {-7.0 / 128.0, 105.0 / 128.0, 35.0 / 128.0, -5.0 / 128.0}};
  const long long n = ncell(C);
  for (long long q = blockIdx.x * (long long)kMgThreads + threadIdx.x; q < n; q += (long long)gridDim.x * kMgThreads) {
    int i, j, k;
    cell_of(C, q, i, j, k);
    double Z[2][2][2] = {{{0.0, 0.0}, {0.0, 0.0}}, {{0.0, 0.0}, {0.0, 0.0}}};  // [cz][cy][cx]
    // coarse offsets -2..2 along each axis; child c (0 left, 1 right) uses offsets c-2 .. c+1
#pragma unroll
    for (int oz = 0; oz < 5; ++oz) {
      double Y[2][2] = {{0.0, 0.0}, {0.0, 0.0}};  // [cy][cx] at this z offset
#pragma unroll
      for (int oy = 0; oy < 5; ++oy) {
        double e[5];
#pragma unroll
        for (int ox = 0; ox < 5; ++ox) e[ox] = C.rphi[at(C, i + ox - 2, j + oy - 2, k + oz - 2)];
        double X[2];
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          double sx = 0.0;
#pragma unroll
          for (int a = 0; a < 4; ++a) sx += w[cx][a] * e[cx + a];
          X[cx] = sx;
        }
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const int b = oy - cy;  // this row's place in child cy's stencil
          if (b < 0 || b > 3) continue;
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) Y[cy][cx] += w[cy][b] * X[cx];
        }
      }
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        const int c = oz - cz;
        if (c < 0 || c > 3) continue;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) Z[cz][cy][cx] += w[cz][c] * Y[cy][cx];
      }
    }
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          F.phi[at(F, 2 * i + cx, 2 * j + cy, 2 * k + cz)] += Z[cz][cy][cx];
        }
  }
}

// The same prolongation by tiles: a workgroup takes 8 x 8 x 4 coarse cells
// (natural order, one per thread), stages their restricted potential with a
// two-cell halo in LDS once (12 x 12 x 8 values, against 125 gathers per cell
// with a wrapped red-black index each), then forms each cell's eight children
// from LDS with the same products and sums in the same order as
// mg_prolong_kernel (the same bits).  Levels whose edges are multiples of 8, 8
// and 4.
constexpr int kPtx = 8, kPty = 8, kPtz = 4;
static_assert(kPtx * kPty * kPtz == kMgThreads, "one coarse cell per thread");

__global__ __launch_bounds__(kMgThreads) void mg_prolong_tiled_kernel(MgLevel F, MgLevel C) {
  constexpr int HX = kPtx + 4, HY = kPty + 4, HZ = kPtz + 4;
  __shared__ double sc[HZ][HY][HX];
  const double w[2][4] = {{-5.0 / 128.0, 35.0 / 128.0, 105.0 / 128.0, -7.0 / 128.0},
                          {-7.0 / 128.0, 105.0 / 128.0, 35.0 / 128.0, -5.0 / 128.0}};
  const int tx = C.nx / kPtx, ty = C.ny / kPty, tz = C.nz / kPtz;
  const int li = threadIdx.x % kPtx, lj = (threadIdx.x / kPtx) % kPty, lk = threadIdx.x / (kPtx * kPty);
  for (int tile = blockIdx.x; tile < tx * ty * tz; tile += gridDim.x) {
    const int i0 = (tile % tx) * kPtx, j0 = ((tile / tx) % ty) * kPty, k0 = (tile / (tx * ty)) * kPtz;
    __syncthreads();  // the previous tile's reads are done
    for (int v = threadIdx.x; v < HX * HY * HZ; v += kMgThreads) {
      const int a = v % HX, b = (v / HX) % HY, c = v / (HX * HY);
      sc[c][b][a] = C.rphi[at(C, i0 + a - 2, j0 + b - 2, k0 + c - 2)];
    }
    __syncthreads();
    double Z[2][2][2] = {{{0.0, 0.0}, {0.0, 0.0}}, {{0.0, 0.0}, {0.0, 0.0}}};  // [cz][cy][cx]
#pragma unroll
    for (int oz = 0; oz < 5; ++oz) {
      double Y[2][2] = {{0.0, 0.0}, {0.0, 0.0}};  // [cy][cx] at this z offset
#pragma unroll
      for (int oy = 0; oy < 5; ++oy) {
        double e[5];
#pragma unroll
        for (int ox = 0; ox < 5; ++ox) e[ox] = sc[lk + oz][lj + oy][li + ox];
        double X[2];
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          double sx = 0.0;
#pragma unroll
          for (int a = 0; a < 4; ++a) sx += w[cx][a] * e[cx + a];
          X[cx] = sx;
        }
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const int b = oy - cy;
          if (b < 0 || b > 3) continue;
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) Y[cy][cx] += w[cy][b] * X[cx];
        }
      }
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        const int c = oz - cz;
        if (c < 0 || c > 3) continue;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) Z[cz][cy][cx] += w[cz][c] * Y[cy][cx];
      }
    }
    const int i = i0 + li, j = j0 + lj, k = k0 + lk;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) F.phi[at(F, 2 * i + cx, 2 * j + cy, 2 * k + cz)] += Z[cz][cy][cx];
  }
}

// the per-block stored potential with one periodic ghost layer; blockIdx.y = block
__global__ __launch_bounds__(kMgThreads) void mg_scatter_kernel(MeshDev m, MgLevel F, double *phib) {
  const BlockInfo B = m.blocks[blockIdx.y];
  const int np = B.n + 2;
  const int tot = np * np * np;
  for (int e = blockIdx.x * kMgThreads + threadIdx.x; e < tot; e += gridDim.x * kMgThreads) {
    const int i = e % np - 1, j = (e / np) % np - 1, k = e / (np * np) - 1;
    phib[B.poff + e] = F.phi[at(F, B.ox + i, B.oy + j, B.oz + k)];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int grid_for(long long n) {
  const long long g = (n + kMgThreads - 1) / kMgThreads;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

hipError_t mg_launch_gather(const MeshDev &m, const int *par, const double *Qa, const double *Qb, const MgLevel &F,
                            hipStream_t s) {
  hipLaunchKernelGGL(mg_gather_kernel, dim3(grid_for((long long)m.nx * m.ny * m.nz)), dim3(kMgThreads), 0, s, m, par,
                     Qa, Qb, F);
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

hipError_t mg_launch_defect_norm(const MgLevel &L, double *part, double *out, hipStream_t s) {
  const long long n = (long long)L.nx * L.ny * L.nz;
  hipLaunchKernelGGL(mg_defect_sq_partial_kernel, dim3(kMgSumParts), dim3(kMgThreads), 0, s, L, part);
  hipLaunchKernelGGL(mg_final_sum_kernel, dim3(1), dim3(kMgThreads), 0, s, part, kMgSumParts, 1.0 / (double)n, 1,
                     out);
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
  if (C.nx % kPtx == 0 && C.ny % kPty == 0 && C.nz % kPtz == 0) {
    const int tiles = (C.nx / kPtx) * (C.ny / kPty) * (C.nz / kPtz);
    hipLaunchKernelGGL(mg_prolong_tiled_kernel, dim3(tiles < 4096 ? tiles : 4096), dim3(kMgThreads), 0, s, F, C);
  } else {
    hipLaunchKernelGGL(mg_prolong_kernel, dim3(grid_for((long long)C.nx * C.ny * C.nz)), dim3(kMgThreads), 0, s, F,
                       C);
  }
  return hipGetLastError();
}

hipError_t mg_launch_scatter(const MeshDev &m, int nblocks, int nmax, const MgLevel &F, double *phib, hipStream_t s) {
  const int np = nmax + 2;
  const int gx = (np * np * np + kMgThreads - 1) / kMgThreads;
  hipLaunchKernelGGL(mg_scatter_kernel, dim3(gx, nblocks), dim3(kMgThreads), 0, s, m, F, phib);
  return hipGetLastError();
}

int mg_coarse_max() { return kMgCoarseMax; }

}  // namespace tdh
