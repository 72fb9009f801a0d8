// Internal declarations shared by the gfx950 kernels and the host runtime of
// libtdh.  Not part of the C ABI (include/tdh.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdh {

enum { IDN = 0, IM1 = 1, IM2 = 2, IM3 = 3, IEN = 4, IAX = 5 };

constexpr int kChunk = 256;       // cells per stage work item (one workgroup)
constexpr int kMaxLevel = 30;
constexpr int kCntSlots = 33;     // cnt_ge[0..32]

// One MeshBlock as the kernels see it.
struct BlockInfo {
  int n, ox, oy, oz;  // edge and origin, in cells of the block's refinement level
  int lev, pad_;      // refinement level (0 or 1: cell widths dx / 2^lev)
  long long off;   // offset (doubles) of the block in every state buffer
  long long poff;  // offset of its (n+2)^3 potential
  long long ioff;  // offset of its [6][nv][n^2] face arrays
  long long foff;  // offset (in faces) of its (n+1) n^2 faces of one axis in the flux arrays
};

struct MeshDev {
  int nx, ny, nz;                  // cells of refinement level 0 (level r: 2^r times as many)
  int bc[3];
  double x0[3], dx[3], inv_dx[3];  // level 0's cell widths
  int lat, lat_shift, lx, ly, lz;  // lattice edge in level-0 cells (a power of two) and its log2
  int amr;                         // some block is on refinement level 1
  int nv;
  const int *lmap;          // lattice cell -> block
  const BlockInfo *blocks;
};

struct Phys {
  int eos_kind, dual, grav_kind, inv_mode, newton_max_iter, riemann, ghost_dense;
  double gamma, eta1, eta2, rho_floor, p_floor, e_floor;
  double gm_bh, r_soft, r_exc;
  double bh_x0[3], v_frame[3];
};

// Tabulated EOS on (log10 rho, log10 T) nodes, packed by density-row pairs:
// le2[i][j] = (log e[i][j], log e[i+1][j]);
// pc[i][j] = (log P[i][j], log P[i+1][j], log cs2[i][j], log cs2[i+1][j]).
struct Table {
  int nrho, nT;
  double lr0, dlr, inv_dlr, lT0, dlT;
  const double2 *le2;
  const double4 *pc;
  // Cell records, one 128-byte line per table cell (i, j), i < nrho-1, j < nT-1:
  // le2[i][j], le2[i][j+1], pc[i][j], pc[i][j+1] (12 doubles, 4 unused): a
  // seeded query whose seed cell brackets its target needs this line only.
  const double *rec;
  // Function tables of the lookups' own log10 and 10^x: lg[i] = {2 c_i,
  // -log10 c_i} with c_i = 1 / (1 + (i + 1/2)/128), i < 128; ex[j] = 2^(j/64), j < 64.
  const double2 *lg;
  const double *ex;
};

constexpr int kMlpParams = 4417;  // W1[64][2], b1[64], W2[64][64], b2[64], W3[64], b3

// Learned seed network weights as the kernels read them (bf16 operands).
struct MlpDev {
  const float *b1, *b2, *b3;
  const short *w1b;   // [64][2]
  const short *w2b;   // [64 out][64 in]
  const short *w2tb;  // [64 in][64 out]
  const short *w3b;   // [64]
};

// Seed network and the normalisation ranges of its inputs and output.
struct Seed {
  int enabled;
  MlpDev w;
  double lr_lo, lr_hi, le_lo, le_hi, lt_lo, lt_hi;
};

struct StageArgs {
  MeshDev m;
  Phys p;
  Table t;
  Seed s;
  double *Qa, *Qb, *Qs;     // state ping-pong pair and stage-1 state
  double *imp, *bf1;        // face impulses, stage-1 boundary fluxes
  const double *phi;        // stored potential (grav_kind 1)
  const int *fac;           // factor (in dt0 units) per block
  const int *par;           // 0: latest state in Qa, 1: in Qb
  const int *order;         // block ids sorted by level, finest first
  const int *item_start;    // prefix sum of work items over `order`
  const int *cnt_ge;        // cnt_ge[L] = blocks with level >= L
  int Llo, Lhi;             // levels advanced by this launch
  int k;                    // sub-cycle index in the window (dt0 units)
  int phase;                // 1 or 2
  const double *win;        // device {window start time, finest step dt0}
  int *jc;                  // table cell of each cell's state, one segment per state buffer
                            // (Qa, Qb, Qs; jn cells each), the seeds of the inversion
  long long jn;
  // split stage form: face fluxes of axis d at flx + d * fstride, per block
  // [nv + 1][(n+1) n^2] (fluxes, then the face velocity) from its foff
  double *flx;
  long long fstride;
  const int *fitem_start;   // prefix sum of 256-face work items (one axis) over `order`
  const int2 *item_bt;      // per work item (cells): block id, index of the item within its block
  const int2 *fitem_bt;     // the same for the face items of the split form
  // CFL partial minima the fused form's second stage leaves for every tile of
  // its output state, at cfl_part[cfl_start[b] + tile] (null: not taken)
  double *cfl_part;
  const int *cfl_start;
  int lmax;                 // finest level of the window (0: every block on one schedule)
};

// host-side launchers (tdh_kernels.hip)
// One multigrid level of the self-gravity solve: a periodic nx x ny x nz grid
// stored in red-black order (red cells, i+j+k even, first; each colour
// [nz][ny][nx/2], x fastest) with x spacing hx (hx2 = hx^2), anisotropy weights wy = (hx/hy)^2,
// wz = (hx/hz)^2, centre coefficient c0 = 2 (1 + wy + wz); phi, the source and
// the restricted fine solution (rphi, coarse levels only).  Defects are
// computed where they are used, never stored.
struct MgLevel {
  int nx, ny, nz;
  double hx2, wy, wz, c0;
  double *phi, *src, *rphi;
};
constexpr int kMgMaxLevels = 24;
constexpr int kMgSumParts = 1024;  // workgroups of the deterministic sums

hipError_t mg_launch_gather(const MeshDev &m, const int *par, const double *Qa, const double *Qb, const MgLevel &F,
                            hipStream_t s);
hipError_t mg_launch_sum(const double *x, long long n, int square, double scale, int op, double *part, double *out,
                         hipStream_t s);
hipError_t mg_launch_source(double *src, const double *mean, double four_pi_G, long long n, hipStream_t s);
hipError_t mg_launch_affine(double *x, const double *shift, double fill, long long n, hipStream_t s);
hipError_t mg_launch_sweep(const MgLevel &L, hipStream_t s);
hipError_t mg_launch_defect_norm(const MgLevel &L, double *part, double *out, hipStream_t s);  // RMS defect
hipError_t mg_launch_restrict(const MgLevel &F, const MgLevel &C, hipStream_t s);
hipError_t mg_launch_coarse_solve(const MgLevel &C, int sweeps, hipStream_t s);
hipError_t mg_launch_prolong(const MgLevel &F, const MgLevel &C, hipStream_t s);
hipError_t mg_launch_scatter(const MeshDev &m, int nblocks, int nmax, const MgLevel &F, double *phib, hipStream_t s);
int mg_coarse_max();

hipError_t launch_remap(const MeshDev &src, const int *src_par, const double *sQa, const double *sQb,
                        const MeshDev &dst, double *Qd, const Phys &p, double t, int nv, int coincident,
                        const int *shift, hipStream_t s);
hipError_t launch_boost(const MeshDev &m, const int *par, double *Qa, double *Qb, int nv, const double *V,
                        double rho_skip, hipStream_t s);
hipError_t launch_frame_acceleration(const MeshDev &m, const int *par, const double *Qa, const double *Qb,
                                     const Phys &p, double t, double rho_min, double *part, double *out,
                                     hipStream_t s);
int frame_acceleration_parts();

int num_tiles();
void tile_shape(int id, int *dims);  // x, y, z edges and waves per SIMD of variant id (x = 0: split form)
// persistent launches: cus = compute units of the device (the launchers size the grid)
hipError_t launch_stage(const StageArgs &a, int tile, int cus, hipStream_t s);
hipError_t launch_seed(const StageArgs &a, int cus, hipStream_t s);
hipError_t launch_set_window(double *win, double t, double dt0, hipStream_t s);
hipError_t launch_commit(const int *order, const int *cnt_ge, int lmin, int *par, hipStream_t s);
// per work item (block, item within the block) of the level-sorted list order / start (nb blocks)
hipError_t launch_expand_items(const int *order, const int *start, int nb, int2 *bt, hipStream_t s);
hipError_t launch_reflux(const StageArgs &a, int lc, int dir, int nmax, int grid, hipStream_t s);  // a.k = completing index
hipError_t launch_cfl_blocks(const double *part, int nblocks, const int *block_item_start, double cfl, double *dtb,
                             hipStream_t s);
bool tile_is_fused(int id);
hipError_t launch_cfl(const StageArgs &a, double cfl, double t, const int *item_block, int nitems,
                      double *part, int nblocks, const int *block_item_start, double *dtb, int cus, hipStream_t s);
hipError_t launch_eos_invert(const Table &t, const Seed &s, int newton_max_iter, const double *lr, const double *le,
                             double *lT, int32_t *j, int32_t *iters, int64_t n, int mode, hipStream_t st);
hipError_t launch_eos_eval(const Phys &p, const Table &t, const double *rho, const double *U, double *P,
                           double *cs, int64_t n, hipStream_t st);

hipError_t mlp_launch_forward(const MlpDev &w, const Seed &s, const double *in, double *out, int64_t n,
                              hipStream_t st);
hipError_t mlp_launch_fwd_bwd(const MlpDev &w, const Seed &s, const double *in, const double *tgt, int64_t n,
                              int batch, uint64_t seed, int step, int random_batch, float *part, float *loss_part,
                              float *grad, float *loss, hipStream_t st);
hipError_t mlp_launch_adam(float *wm, float *m, float *v, const float *g, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t st);
hipError_t mlp_launch_pack(const float *wm, short *w1b, short *w2b, short *w2tb, short *w3b, float *b1, float *b2,
                           float *b3, hipStream_t st);

}  // namespace tdh
