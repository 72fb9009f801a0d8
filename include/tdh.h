/*
 * tdh.h - C ABI of the MI355X (gfx950) MeshBlock hydro library.
 *
 * The library advances a mesh of cubic MeshBlocks with the finite-volume
 * Godunov update of "An End-to-End Numerical Framework for Tidal Disruption
 * Events with AthenaK": RK2 + PLM + a Riemann solver (Table 1; the solver here
 * is HLLC), pressure and sound speed from an ideal gas or a tabulated EOS in
 * (log rho, log T) (Sec. Tabulated EOS construction, eqs eos-table-range and
 * eos-table-fields), dual-energy internal-energy evolution (Sec. Dual-energy
 * evolution, eqs dual-econs to dual-sync), fixed-potential gravity with
 * centred momentum and flux-form energy sources (eqs lat-grav-momentum,
 * lat-grav-energy) or a softened point mass with an excised sink
 * (eq bh-softened-gravity), all under localized adaptive time stepping:
 * per-block power-of-two steps, windows, time-interpolated ghosts and
 * delayed flux correction with gravitational work (Sec. LAT method and
 * Coupling with gravity, eqs lat-base-dt, lat-factor, lat-flux-impulse,
 * lat-mass-impulse-mismatch, lat-grav-reflux).
 *
 * Conventions for every entry point
 *   - Every call returns tdh_status (0 = success) and never aborts or throws.
 *     tdh_last_error() gives a message for the last failing call.
 *   - After TDH_EHIP (a HIP runtime error) the context is poisoned: every
 *     later call except tdh_last_error and tdh_destroy returns TDH_ESTATE.
 *   - Pointers named host_* are host memory, read or written synchronously.
 *     Pointers named dev_* are device memory on the context's GPU; the caller
 *     owns them and keeps them alive while the context uses them.
 *   - All device work is enqueued on the stream given to tdh_init; calls that
 *     return host data synchronise that stream first.
 *   - The library allocates no device memory.  Everything a context uses on
 *     the device lives in buffers the caller owns: the arena of
 *     tdh_init_blocks (state, impulses, potential, block and work-item
 *     tables, reduction partials, the learned seed's weights and moments),
 *     the EOS table buffer of tdh_set_eos_table and the workspace of
 *     tdh_gravity_solve; tdh_reduce_dt_static uses a static per-GPU array
 *     of the library.  Captured windows and V-cycles are HIP graph objects,
 *     which the HIP runtime instantiates (tdh_run_window with use_graph,
 *     tdh_gravity_solve); every other call enqueues plain kernel launches
 *     and copies.
 *
 * State layout (host and device): blocks one after another in the order of
 * the block list; block b holds nv arrays of n_b^3 doubles, x fastest, with
 * nv = 5 (rho, m_x, m_y, m_z, E) or 6 (plus the auxiliary internal energy
 * density U_aux when dual energy is on).
 */
#ifndef TDH_H
#define TDH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdh_ctx tdh_ctx;

typedef enum {
  TDH_OK = 0,
  TDH_EINVAL = -1, /* argument outside its documented range */
  TDH_ENOMEM = -2, /* arena too small, or a setup allocation failed */
  TDH_EHIP = -3,   /* HIP runtime error; the context is poisoned */
  TDH_ESTATE = -4, /* call out of order (e.g. stepping before init_blocks) */
  TDH_ERANGE = -5  /* sizes beyond a documented maximum */
} tdh_status;

/* Run parameters. */
typedef struct {
  int eos_kind;   /* 0 ideal gas (gamma), 1 tabulated (tdh_set_eos_table) */
  int dual;       /* 1: evolve U_aux and use the eta1 switch (eq dual-primitive-switch) */
  int grav_kind;  /* 0 none; 1 stored cell-centred potential (tdh_init_blocks host_phi);
                     2 softened point mass at bh_x0 - v_frame * t (eq bh-softened-gravity)
                        with cells closer than r_exc excised */
  int n_lat;      /* N_LAT of eq lat-factor: factors up to 2^n_lat (0 = synchronous) */
  double gamma;   /* ideal-gas adiabatic index */
  double eta1;    /* pressure-recovery switch threshold (eq dual-primitive-switch) */
  double eta2;    /* resynchronisation threshold (eq dual-sync) */
  double cfl;     /* Courant number */
  double rho_floor, p_floor; /* density floor; pressure floor of the ideal gas */
  double e_floor; /* specific internal energy floor of the tabulated EOS */
  double merge_frac; /* top LAT bins holding fewer than merge_frac * nblocks blocks merge down */
  double gm_bh, r_soft, r_exc; /* G M, softening length, excision radius (grav_kind 2) */
  double bh_x0[3], v_frame[3]; /* point-mass position at t = 0 and frame velocity */
  int inv_mode;   /* table inversion (every mode gives the same cell, hence the same result):
                     0 bisection for every query;
                     2 before each stage a pass bisects for the table cell of every
                       cell's stage-input state; that cell seeds the cell's face and
                       compression queries (a face's right state is seeded by its
                       left state's cell);
                     1 as 2, but each stage records the table cells of its output
                       states for the next stage instead of a pass, their searches
                       starting from the learned network's prediction (tdh_mlp_*;
                       from the input state's cell while the network is off);
                     3 as 1 with every search starting from the input state's cell;
                     4 as 2 with the pass's searches starting from the learned
                       network's prediction (bisection while the network is off).
                     In modes 1 and 3 a pass finds the cells once after a state
                     upload (with the network in mode 1).  In modes 2 and 4 the
                     CFL reduction (tdh_reduce_dt) records the cells of the state
                     it reduces over (its search for c_s finds them), and the
                     next window's first stage runs without a pass. */
  int newton_max_iter; /* seeded secant steps before falling back to bisection (>= 0) */
  int riemann;    /* 0 HLLC (Toro Sec. 10.4); 1 HLLE, the solver of the paper's production
                     runs (Table 1): the HLL flux with the same Davis wave-speed bounds */
  int ghost_dense; /* LAT ghosts of a neighbour that is mid-step at the stage time
                     (Sec. LAT method): 0 linear interpolation in time of its start and
                     end states; 1 the dense output of its RK2 step, a convex combination
                     of its start, stage-1 and end states (admissible where they are) */
} tdh_config;

/* Mesh: cubic blocks whose edge n is a power of two in [8, 256], covering the
 * domain exactly once, on up to two refinement levels (Sec. LAT method,
 * coarse-fine interfaces).  A block on level r has cell widths dx / 2^r and
 * its origin counted in level-r cells; every origin lies on the lattice of the
 * smallest block extent measured in level-0 cells.  Ghost states across a
 * coarse-fine interface are the coarse histories restricted (mean of the 2x2x2
 * fine children), interpolated in time and prolonged (minmod-limited linear);
 * the coarse side takes the flux correction at every coarse-fine face.  Runs
 * with a refined block support neither tdh_gravity_solve, tdh_remap nor
 * tdh_frame_acceleration (TDH_EINVAL). */
typedef struct {
  int nx, ny, nz;   /* global cells per axis of level 0 */
  int bc[3];        /* per axis: 0 periodic, 1 outflow (zero gradient) */
  double x0[3];     /* lower domain corner */
  double dx[3];     /* cell widths of level 0 */
  int nblocks;
  const int *blk;   /* host [nblocks][4] = n, ox, oy, oz (origin in cells of the block's level) */
  const int *rlev;  /* host [nblocks] refinement level of each block, 0 or 1 (NULL: all 0) */
} tdh_mesh;

/* Counters since tdh_init_blocks. */
typedef struct {
  int64_t block_updates;  /* RK2 steps taken by blocks */
  int64_t cell_updates;   /* sum over block updates of the block's cells */
  int64_t windows;        /* completed LAT windows */
  int64_t sub_cycles;     /* step_level calls */
  int64_t kernel_launches;
  int64_t graph_captures; /* window graphs captured and instantiated (one per new Lmax and launch form) */
  double capture_ms;      /* host time those captures and instantiations took */
} tdh_stats;

/* Device bytes the arena must hold for this configuration and mesh (two
 * state copies, the stage-1 state, the potential, face impulses, seed cells,
 * split-form fluxes, block and work-item tables, reduction partials, and with
 * the table EOS the learned seed's buffers, about 22 MB).  Returns 0 for an
 * invalid mesh. */
size_t tdh_arena_bytes(const tdh_config *cfg, const tdh_mesh *mesh);

/* Create a context on the current HIP device; hip_stream is a hipStream_t
 * (NULL = default stream).  The configuration is copied. */
tdh_status tdh_init(const tdh_config *cfg, void *hip_stream, tdh_ctx **out);

/* Install the mesh and the initial state.  dev_arena: caller-owned device
 * buffer of at least tdh_arena_bytes() bytes, 256-byte aligned.
 * host_state: initial conserved state (layout above).  host_phi: for
 * grav_kind 1, per block (n+2)^3 cell-centred potential values including one
 * ghost layer, x fastest (else NULL).  Levels start at 0 (synchronous). */
tdh_status tdh_init_blocks(tdh_ctx *ctx, const tdh_mesh *mesh, void *dev_arena, size_t arena_bytes,
                           const double *host_state, const double *host_phi);

/* Device bytes the packed EOS table of nrho x nT nodes needs (0 outside
 * 2 <= nrho, nT <= 4096). */
size_t tdh_table_bytes(int nrho, int nT);

/* Tabulated EOS (Sec. Tabulated EOS construction): node (i, j) at
 * log10 rho = lr0 + i*dlr, log10 T = lT0 + j*dlT; host arrays [nrho][nT],
 * T contiguous, of log10 P, log10 e (specific internal energy, strictly
 * increasing in T on every row) and log10 c_s^2.  2 <= nrho, nT <= 4096.
 * dev_table: caller-owned device buffer of at least tdh_table_bytes(nrho, nT)
 * bytes, 256-byte aligned, that the context reads until the next call of this
 * function or tdh_destroy (TDH_ENOMEM if smaller, TDH_EINVAL if null or
 * misaligned). */
tdh_status tdh_set_eos_table(tdh_ctx *ctx, int nrho, int nT, double lr0, double dlr, double lT0, double dlT,
                             const double *host_logP, const double *host_loge, const double *host_logcs2,
                             void *dev_table, size_t table_bytes);

/* Per-block CFL step dt_b = cfl * min over cells of min over axes of
 * dx/(|v|+c_s) and, with gravity, sqrt(dx_min/|g|) (g the centred potential
 * gradient; excised cells skipped), its minimum dt0 (eq lat-base-dt) and the LAT
 * levels of eq lat-factor after bin merging and the neighbour limits (one
 * level apart on one refinement level, f_fine <= f_coarse <= 2 f_fine across
 * refinement levels); level = Lmax - log2(f_b), level 0 coarsest.  The levels are
 * installed and start a new window.  host_dt_block [nblocks] and
 * host_levels [nblocks] may be NULL.  With the table EOS in inv_mode 2 or 4
 * it also records every cell's table cell as the seeds of the next window's
 * first stage.  On single-level table-EOS runs without the point mass, after a
 * window of a fused stage variant, it reduces the per-tile minima that the
 * window's second stages computed from their output states (the same values;
 * any other change of the state makes it read the state again).
 * Synchronises the stream. */
tdh_status tdh_reduce_dt(tdh_ctx *ctx, double *host_dt_block, double *host_dt0, int8_t *host_levels,
                         int *host_lmax);

/* tdh_reduce_dt for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same results, bit for bit, with the reduction's per-item partial minima
 * and per-block steps in a static device array of the library (4 MiB per
 * GPU, held until the process ends) instead of buffers the library allocated
 * at tdh_init_blocks.  It always reduces over the state itself (never the
 * minima a window's second stages left).  Meshes with more than 2^19 work
 * items plus blocks (one item per 256 cells of a block: about 134 M cells)
 * return TDH_ERANGE.  Every context on a GPU shares that GPU's array: calls
 * that overlap on one GPU (other threads or streams) race.  Allocates
 * nothing; synchronises the stream. */
tdh_status tdh_reduce_dt_static(tdh_ctx *ctx, double *host_dt_block, double *host_dt0, int8_t *host_levels,
                                int *host_lmax);

/* Install host-chosen levels (each 0..30; neighbours on one refinement level
 * at most one apart; across refinement levels f_fine <= f_coarse <= 2 f_fine
 * with f = 2^(Lmax - level)) and start a new window. */
tdh_status tdh_set_levels(tdh_ctx *ctx, const int8_t *host_levels);

/* One LAT sub-cycle: every block whose level is >= level takes one RK2
 * step, a block on level L with dt * 2^(level - L).  Within a window of
 * 2^Lmax sub-cycles the calls must follow the schedule: sub-cycle k
 * (k = 0 .. 2^Lmax - 1) has level 0 for k = 0 and Lmax - ctz(k) otherwise,
 * and dt * 2^level must equal the window's coarse step; the window ends
 * after its last sub-cycle, when every block is synchronised.
 * Returns TDH_ESTATE for a call out of schedule. */
tdh_status tdh_step_level(tdh_ctx *ctx, int level, double dt);

/* A whole window: all 2^Lmax sub-cycles with coarse step dt_coarse.
 * batched = 1 advances every active level in one launch per phase;
 * batched = 0 launches each level separately (same results bit for bit).
 * use_graph = 1 captures the window into a hipGraph and replays it. */
tdh_status tdh_run_window(tdh_ctx *ctx, double dt_coarse, int batched, int use_graph);

/* Simulation time of the synchronised state. */
tdh_status tdh_get_time(tdh_ctx *ctx, double *host_t);
tdh_status tdh_set_time(tdh_ctx *ctx, double t);

/* Copy the current (synchronised) state to / from host memory. */
tdh_status tdh_get_state(tdh_ctx *ctx, double *host_state);
tdh_status tdh_set_state(tdh_ctx *ctx, const double *host_state);

/* Self-gravity at a synchronised state (Sec. Self-gravity solver, eqs
 * selfgrav-poisson, selfgrav-defect): solves A phi = S on the mesh's uniform
 * grid, A = -lap_h the seven-point operator (neighbours in y and z weighted by
 * (dx/dy)^2 and (dx/dz)^2, centre 2 (1 + wy + wz)), S = -4 pi G (rho - mean
 * rho) from the current density (the mean removed in two passes), with
 * periodic boundaries, by geometric
 * multigrid V-cycles (red-black Gauss-Seidel, over-relaxation 1.15, two pre-
 * and two post-sweeps per level, defect restricted by child means, coarse
 * correction in full-approximation form, tricubic prolongation, one extra
 * finest sweep per cycle; the coarsest level gets 2 (nx+ny+nz)^2 sweeps).  The
 * result, shifted to zero mean, is written into the stored potential that the
 * hydro update reads (per block (n+2)^3 with one ghost layer), so grav_kind
 * must be 1.
 * Requirements: every axis periodic; the levels halve every axis while all
 * are at least 4, and every level, the coarsest included, has even
 * dimensions; the coarsest level holds at most 2048 cells (TDH_EINVAL /
 * TDH_ERANGE otherwise).  Only between windows (TDH_ESTATE).
 * dev_work: caller-owned device buffer of at least the bytes
 * tdh_gravity_workspace_bytes returns; its first nx*ny*nz doubles hold the
 * solution on the global grid in red-black order (the cells with i+j+k even
 * first, then the others, each half [nz][ny][nx/2] with x fastest), the start
 * of the next solve when warm != 0 (pass the same buffer again); warm == 0
 * starts from zero.  V-cycles run until the root-mean-square defect is <= tol or
 * max_cycles in [0, 1000] have run (tol 0: exactly max_cycles).
 * host_cycles (nullable): V-cycles run.  host_defects (nullable,
 * max_cycles + 1 doubles): the RMS defect before the first and after each
 * cycle.  Synchronises the stream. */
tdh_status tdh_gravity_workspace_bytes(tdh_ctx *ctx, size_t *host_bytes);
tdh_status tdh_gravity_solve(tdh_ctx *ctx, void *dev_work, size_t bytes, double four_pi_G, int max_cycles,
                             double tol, int warm, int *host_cycles, double *host_defects);
/* Restart remap (Sec. Domain remapping of conserved variables, eqs
 * remap-state-vector, remap-cell-average): dst's state becomes the remap of
 * src's current state onto dst's mesh, and dst's time src's.  Per target cell:
 * inside dst's excision sphere at that time (grav_kind 2), the sink state
 * (rho_floor, 0, U_floor); centre outside src's domain along a non-periodic
 * axis, the floor state; within two source cells inside a source face beyond
 * which dst's domain extends (non-periodic axes), the value below blended
 * toward the floor state, density, momentum and thermal energy density each
 * as s q + (1 - s) q_floor, s = 3u^2 - 2u^3 with u the distance to the
 * nearest such face in units of two source cells (so density and pressure
 * reach the floor smoothly at the old domain's edge); target grid coincident
 * with the source grid (equal
 * spacings, origins a whole number of cells apart), the source cell copied;
 * otherwise the mean over the eight sub-cell midpoints (+-1/4 cell per axis)
 * of the trilinear interpolant of the source density, momentum and thermal
 * energy density (U_aux with dual energy on, E - |m|^2/2rho otherwise), with
 * E rebuilt as U + |m|^2/2rho and U_aux = U (thermal, not total, energy is
 * carried).  Stencils clamp at non-periodic source edges and wrap across
 * periodic ones.  Both contexts on the current device with the same number
 * of variables (TDH_EINVAL), both between windows (TDH_ESTATE); src's stream
 * is synchronised first, dst's on return.  Seed cells of dst are dropped. */
tdh_status tdh_remap(tdh_ctx *dst, tdh_ctx *src);
/* Galilean boost by host_V[3] (eq galilean-boost): m += rho V,
 * E += m.V + rho |V|^2/2 (with the old m), U_aux unchanged, in every cell with
 * rho > rho_skip (floor-density cells keep their state).  Between windows;
 * synchronises the stream. */
tdh_status tdh_galilean_boost(tdh_ctx *ctx, const double *host_V, double rho_skip);
/* Frame acceleration (eq frame-acceleration) at the context's time: the
 * density-weighted mean over cells with rho > rho_min outside the excision
 * sphere of the point mass's field -GM (r - r_bh) / (|r - r_bh|^2 +
 * r_soft^2)^(3/2) at the cell centre (uniform cells: the volume cancels; 0 if
 * no cell counts) into host_A[3].  grav_kind 2 only (TDH_ESTATE).  Sums in a
 * fixed order; synchronises the stream. */
tdh_status tdh_frame_acceleration(tdh_ctx *ctx, double rho_min, double *host_A);
/* Copy of the stored potential (grav_kind 1): per block (n+2)^3 doubles with
 * one ghost layer, blocks in order, x fastest.  Synchronises the stream. */
tdh_status tdh_get_potential(tdh_ctx *ctx, double *host_phi);

/* Seed table cells held for the current state (tdh_config.inv_mode 3; table
 * EOS only): host_cells receives one int32 per cell, blocks in order, cells of
 * a block x fastest; -1 where none is held yet (after a state upload).  The
 * values only start searches; they never change a result.  Synchronises the
 * stream.  TDH_ESTATE without a table EOS or inside a window. */
tdh_status tdh_get_seed_cells(tdh_ctx *ctx, int32_t *host_cells);

/* Batched EOS queries on device arrays of n values (n <= 2^31):
 *   invert: log10 rho, log10 e -> log10 T, table cell j, secant steps taken
 *           (-1 when the bisection fallback ran); mode as tdh_config.inv_mode
 *           with the seed taken from the network (mode 1) or bisection.
 *   eval:   rho, U (internal energy density) -> P, c_s. */
tdh_status tdh_eos_invert_batch(tdh_ctx *ctx, const double *dev_lrho, const double *dev_le, double *dev_lT,
                                int32_t *dev_j, int32_t *dev_iters, int64_t n, int mode);
tdh_status tdh_eos_eval_batch(tdh_ctx *ctx, const double *dev_rho, const double *dev_U, double *dev_P,
                              double *dev_cs, int64_t n);

/* Stage-kernel variants: tdh_num_tiles() of them.  id -> host_dims4[4]:
 *   fused form (one kernel; a workgroup per tile, faces through LDS):
 *     (x, y, z) tile edges (256 cells, one thread per cell) and the waves
 *     per SIMD its register budget targets;
 *     a tile must divide the smallest block;
 *   split form (a face-flux kernel per axis writing the faces of every active
 *     block to HBM, then a per-cell update kernel; fits every mesh):
 *     (0, waves per SIMD of the face kernels, of the update kernel, 0).
 * Every variant gives bit-identical results.  Meshes with a refined block
 * run one fused variant of their own (8 x 8 x 4 cells) whatever is chosen.
 * tdh_autotune times one stage over all blocks reps times per fitting shape
 * (state unchanged), keeps the fastest, returns its id and per-shape
 * milliseconds (host_ms [tdh_num_tiles()], -1 where a shape does not fit;
 * may be NULL).  Call between windows. */
int tdh_num_tiles(void);
tdh_status tdh_tile_shape(int id, int *host_dims4);
tdh_status tdh_set_tile(tdh_ctx *ctx, int id);
tdh_status tdh_get_tile(tdh_ctx *ctx, int *host_id);
tdh_status tdh_autotune(tdh_ctx *ctx, int reps, int *host_best, float *host_ms);

/* Stage-kernel timing: with on = 1 every stage launch outside graph replay
 * is bracketed by HIP events recorded on the context's stream;
 * tdh_get_stage_time returns the summed kernel milliseconds and the number
 * of timed launches since tdh_set_timing (synchronising on the last event). */
tdh_status tdh_set_timing(tdh_ctx *ctx, int on);
tdh_status tdh_get_stage_time(tdh_ctx *ctx, double *host_ms, int64_t *host_launches);

/* Learned seed of the table inversion (not part of the paper's method; the
 * plain bisection stays the fallback and decides the result): a
 * 2 -> 64 -> 64 -> 1 ReLU network mapping normalised (log10 rho, log10 e)
 * to normalised log10 T, bf16 operands and fp32 accumulation, hidden layer
 * on the matrix cores.  Inputs are normalised as 2 (v - lo)/(hi - lo) - 1.
 *   init:      fp32 parameters [4417] = W1[64][2], b1[64], W2[64 out][64 in],
 *              b2[64], W3[64], b3; resets the Adam moments; the seed is off.
 *   train:     steps of Adam (beta 0.9/0.999, eps 1e-8, cosine-decayed lr) on
 *              the mean squared error, each on `batch` samples (multiple of
 *              64, <= 65536) drawn with replacement from dev_in [n][2]
 *              (log10 rho, log10 e) / dev_lT [n] by a counter hash of seed
 *              and step; host_loss [steps] (nullable) receives each step's loss.
 *   loss_grad: loss and gradient [4417] over the first n samples (n a
 *              multiple of 64, <= 65536), no update.
 *   forward:   log10 T predictions for n queries.
 *   enable_seed: use the network for inv_mode 1 (tdh_config) and eos mode 1. */
tdh_status tdh_mlp_init(tdh_ctx *ctx, const float *host_params, double lr_lo, double lr_hi, double le_lo,
                        double le_hi, double lt_lo, double lt_hi);
tdh_status tdh_mlp_train(tdh_ctx *ctx, const double *dev_in, const double *dev_lT, int64_t n, int steps, int batch,
                         float lr, uint64_t seed, float *host_loss);
tdh_status tdh_mlp_loss_grad(tdh_ctx *ctx, const double *dev_in, const double *dev_lT, int64_t n, float *host_loss,
                             float *host_grad);
/* One Adam step (beta 0.9/0.999, eps 1e-8, bias corrections with the step
 * counter, which advances by one; no learning-rate decay) from a caller-given
 * gradient host_grad [4417] (fp32, parameter order of tdh_mlp_init) at
 * learning rate lr > 0, on the fp32 master parameters; the bf16 copies the
 * kernels read are refreshed.  For training loops the caller drives.
 * Synchronises the stream. */
tdh_status tdh_mlp_adam_step(tdh_ctx *ctx, const float *host_grad, float lr);
tdh_status tdh_mlp_forward(tdh_ctx *ctx, const double *dev_in, double *dev_lT, int64_t n);
tdh_status tdh_mlp_get_params(tdh_ctx *ctx, float *host_params);
tdh_status tdh_mlp_enable_seed(tdh_ctx *ctx, int on);

tdh_status tdh_get_stats(tdh_ctx *ctx, tdh_stats *out);
const char *tdh_last_error(const tdh_ctx *ctx);
void tdh_destroy(tdh_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* TDH_H */
