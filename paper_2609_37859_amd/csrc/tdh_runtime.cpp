// Host runtime of libtdh: context, state arena, block registry, LAT level
// assignment and sub-cycle scheduling, hipGraph capture, and the C ABI of
// include/tdh.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tdh.h"
#include "tdh_internal.hpp"

using namespace tdh;

struct tdh_ctx {
  tdh_config cfg{};
  hipStream_t stream = nullptr;
  bool poisoned = false;
  std::string err;

  // mesh (host copy)
  bool have_mesh = false;
  int nx = 0, ny = 0, nz = 0, bc[3] = {0, 0, 0};
  double x0[3] = {0, 0, 0}, dx[3] = {1, 1, 1};
  int nb = 0, nv = 5, lat = 0, lx = 0, ly = 0, lz = 0, nmax = 0;
  std::vector<int> blk;                 // [nb][4]
  std::vector<int> rl;                  // refinement level of each block (0 or 1)
  bool amr = false;                     // some block is on level 1
  std::vector<int> lmap;
  std::vector<BlockInfo> binfo;
  std::vector<std::vector<int>> adj;    // face/edge/corner neighbours
  long long total = 0, ptotal = 0, itotal = 0;
  long long ncells = 0;

  // device memory: all in the caller's arena and buffers (the library allocates none)
  double *Qa = nullptr, *Qb = nullptr, *Qs = nullptr, *imp = nullptr, *bf1 = nullptr, *phi = nullptr;
  int *jc = nullptr;  // seed table cells: a segment of ncells per state buffer (Qa, Qb, Qs)
  double *flx = nullptr;  // face fluxes of the split stage form (3 axes)
  long long ftotal = 0;   // faces of one axis over all blocks
  bool seeds_held = false;  // the current buffers' segments hold the cells of the current state
  bool cfl_seeds = false;   // modes 2, 4: the CFL pass recorded them and no stage has run since
  bool cfl_parts = false;   // the last window's second stages left every tile's CFL minimum of this state
  BlockInfo *d_blocks = nullptr;
  int *d_lmap = nullptr, *d_fac = nullptr, *d_par = nullptr, *d_order = nullptr, *d_item_start = nullptr;
  int *d_cnt_ge = nullptr, *d_cfl_item_block = nullptr, *d_cfl_block_start = nullptr, *d_fitem_start = nullptr;
  int2 *d_item_bt = nullptr, *d_fitem_bt = nullptr;  // per work item: block, item within the block
  double *d_cfl_part = nullptr, *d_dtb = nullptr, *d_win = nullptr;
  int cfl_nitems = 0;
  std::vector<double> h_dtb;  // host copy of the per-block steps

  // EOS table
  bool have_table = false;
  Table tab{};
  double *d_table = nullptr;
  // learned seed network
  Seed seed{};
  bool have_mlp = false;
  float *d_mw = nullptr, *d_mm = nullptr, *d_mv = nullptr, *d_mgrad = nullptr, *d_mpart = nullptr;
  float *d_mloss_part = nullptr, *d_mloss = nullptr, *d_mb = nullptr;
  short *d_mwb = nullptr;
  int mlp_steps_done = 0;

  // LAT window state
  std::vector<int> levels, fac, par, order, item_start, fitem_start, cnt_ge;
  int Lmax = 0;
  int k = 0;                 // next sub-cycle
  double dt_coarse = 0.0, dt0 = 0.0;
  double t = 0.0;            // time of the last synchronised state
  int cus = 256;             // compute units (the persistent launches size their grids from it)
  int tile = 0;              // stage tile shape (launch_stage id)
  tdh_stats stats{};

  // stage-kernel timing (HIP events around each stage launch, non-graph path)
  bool timing = false;
  bool capturing = false;
  std::vector<hipEvent_t> ev;       // pairs
  size_t ev_used = 0;
  double stage_ms = 0.0;
  long long stage_launches = 0;

  // captured windows: key = (Lmax, batched)
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  // captured multigrid cycles (V-cycle, extra sweep, defect norm): key = workspace
  std::map<const void *, hipGraphExec_t> mg_graphs;
  double *d_facc = nullptr;  // frame-acceleration partial sums and result
  double *scratch = nullptr;  // this GPU's copy of the static device scratch
};

// Device scratch of the allocation-free entry point (tdh_reduce_dt_static):
// its per-item partial minima and per-block steps.  One copy per GPU, held
// until the process ends; every call on a GPU shares it.
constexpr long long kScratchDoubles = 1LL << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static std::map<int, double *> g_scratch_ptr;  // device -> address of its copy

// Address of the current device's scratch copy, resolved once per device
// (null if the runtime cannot resolve it).
static double *device_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  double *ptr = nullptr;
  if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess) ptr = nullptr;
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

static thread_local std::string g_err;

static tdh_status fail(tdh_ctx *c, tdh_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  g_err = buf;
  return s;
}

static tdh_status hip_fail(tdh_ctx *c, hipError_t e, const char *what) {
  if (c) c->poisoned = true;
  return fail(c, TDH_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(c, expr)                                   \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail((c), e_, #expr); \
  } while (0)

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static constexpr int kMlpMaxBatch = 65536;
static constexpr int kMlpMaxSteps = 1 << 20;

// ---------------------------------------------------------------------------
// mesh validation and layout
// ---------------------------------------------------------------------------
struct Layout {
  long long total = 0, ptotal = 0, itotal = 0, ncells = 0, ftotal = 0;
  long long nitems = 0;   // 256-cell work items over all blocks
  long long lcells = 0;   // lattice cells
  std::vector<long long> off, poff, ioff, foff;
  int lat = 0, nmax = 0;
};

static const char *mesh_layout(const tdh_config *cfg, const tdh_mesh *m, Layout &L) {
  if (!m || m->nblocks <= 0 || !m->blk) return "empty mesh";
  const int nv = cfg->dual ? 6 : 5;
  int lat = 1 << 30, nmax = 0;
  for (int b = 0; b < m->nblocks; ++b) {
    const int n = m->blk[4 * b];
    const int r = m->rlev ? m->rlev[b] : 0;
    if (!is_pow2(n) || n < 2 || n > 256) return "block edge must be a power of two in [2, 256]";
    if (r < 0 || r > 1) return "refinement level must be 0 or 1";
    lat = std::min(lat, n >> r);  // the lattice counts level-0 cells
    nmax = std::max(nmax, n);
  }
  if (lat < 1) return "a level-1 block must span at least one level-0 cell";
  if (m->nx <= 0 || m->ny <= 0 || m->nz <= 0 || m->nx % lat || m->ny % lat || m->nz % lat)
    return "domain size must be a positive multiple of the smallest block edge";
  for (int d = 0; d < 3; ++d) {
    if (m->bc[d] != 0 && m->bc[d] != 1) return "boundary kind must be 0 or 1";
    if (!(m->dx[d] > 0.0)) return "cell widths must be positive";
  }
  L.off.resize(m->nblocks);
  L.poff.resize(m->nblocks);
  L.ioff.resize(m->nblocks);
  L.foff.resize(m->nblocks);
  for (int b = 0; b < m->nblocks; ++b) {
    const long long n = m->blk[4 * b];
    L.off[b] = L.total;
    L.total += nv * n * n * n;
    L.poff[b] = L.ptotal;
    L.ptotal += (n + 2) * (n + 2) * (n + 2);
    L.ioff[b] = L.itotal;
    L.itotal += 6LL * nv * n * n;
    L.foff[b] = L.ftotal;
    L.ftotal += (n + 1) * n * n;
    L.ncells += n * n * n;
    L.nitems += (n * n * n + kChunk - 1) / kChunk;
  }
  L.lat = lat;
  L.nmax = nmax;
  L.lcells = (long long)(m->nx / lat) * (m->ny / lat) * (m->nz / lat);
  return nullptr;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
static int nv_of(const tdh_config *cfg) { return cfg->dual ? 6 : 5; }

// The arena's regions in order: every device byte a context uses lives in
// the caller's arena (state, impulses, potential, seeds, split-form fluxes,
// the block and work-item tables, the reduction's partials, and with the
// table EOS the learned seed's weights, moments, gradients and partial
// sums), except the EOS table (tdh_set_eos_table) and the self-gravity
// workspace (tdh_gravity_solve), which are the caller's buffers too.  With
// c == nullptr only the total size.
static size_t arena_regions(const tdh_config *cfg, const Layout &L, int nb, char *base, tdh_ctx *c) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *r = base ? base + off : nullptr;
    off += align256(bytes);
    return r;
  };
  const int nv = nv_of(cfg);
  const long long fitems = (L.ftotal + (long long)nb * (kChunk - 1)) / kChunk;
  char *Qa = take(L.total * sizeof(double)), *Qb = take(L.total * sizeof(double));
  char *Qs = take(L.total * sizeof(double));
  char *imp = take(L.itotal * sizeof(double)), *bf1 = take(L.itotal * sizeof(double));
  char *phi = cfg->grav_kind == 1 ? take(L.ptotal * sizeof(double)) : nullptr;
  char *jc = cfg->eos_kind == 1 ? take(3 * L.ncells * sizeof(int)) : nullptr;  // seed cells of Qa, Qb, Qs
  char *flx = take(3 * (nv + 1) * L.ftotal * sizeof(double));
  char *blocks = take(nb * sizeof(BlockInfo)), *lmap = take(L.lcells * sizeof(int));
  char *fac = take(nb * sizeof(int)), *par = take(nb * sizeof(int)), *order = take(nb * sizeof(int));
  char *item_start = take((nb + 1) * sizeof(int)), *fitem_start = take((nb + 1) * sizeof(int));
  char *item_bt = take(L.nitems * sizeof(int2)), *fitem_bt = take(fitems * sizeof(int2));
  char *cnt_ge = take(kCntSlots * sizeof(int)), *dtb = take(nb * sizeof(double)), *win = take(2 * sizeof(double));
  char *cfl_block_start = take((nb + 1) * sizeof(int)), *cfl_item_block = take(L.nitems * sizeof(int));
  char *cfl_part = take(L.nitems * sizeof(double));
  char *facc = take((4 * frame_acceleration_parts() + 4) * sizeof(double));
  char *mw = nullptr, *mm = nullptr, *mv = nullptr, *mgrad = nullptr, *mpart = nullptr, *mloss_part = nullptr;
  char *mloss = nullptr, *mb = nullptr, *mwb = nullptr;
  if (cfg->eos_kind == 1) {  // the learned seed of the table inversion
    mw = take(kMlpParams * sizeof(float));
    mm = take(kMlpParams * sizeof(float));
    mv = take(kMlpParams * sizeof(float));
    mgrad = take(kMlpParams * sizeof(float));
    mpart = take((size_t)(kMlpMaxBatch / 64) * kMlpParams * sizeof(float));
    mloss_part = take((kMlpMaxBatch / 64) * sizeof(float));
    mloss = take(kMlpMaxSteps * sizeof(float));
    mb = take((64 + 64 + 1) * sizeof(float));
    mwb = take((128 + 4096 + 4096 + 64) * sizeof(short));
  }
  if (c) {
    c->Qa = (double *)Qa; c->Qb = (double *)Qb; c->Qs = (double *)Qs;
    c->imp = (double *)imp; c->bf1 = (double *)bf1; c->phi = (double *)phi; c->jc = (int *)jc;
    c->flx = (double *)flx;
    c->d_blocks = (BlockInfo *)blocks; c->d_lmap = (int *)lmap;
    c->d_fac = (int *)fac; c->d_par = (int *)par; c->d_order = (int *)order;
    c->d_item_start = (int *)item_start; c->d_fitem_start = (int *)fitem_start;
    c->d_item_bt = (int2 *)item_bt; c->d_fitem_bt = (int2 *)fitem_bt;
    c->d_cnt_ge = (int *)cnt_ge; c->d_dtb = (double *)dtb; c->d_win = (double *)win;
    c->d_cfl_block_start = (int *)cfl_block_start; c->d_cfl_item_block = (int *)cfl_item_block;
    c->d_cfl_part = (double *)cfl_part; c->d_facc = (double *)facc;
    c->d_mw = (float *)mw; c->d_mm = (float *)mm; c->d_mv = (float *)mv; c->d_mgrad = (float *)mgrad;
    c->d_mpart = (float *)mpart; c->d_mloss_part = (float *)mloss_part; c->d_mloss = (float *)mloss;
    c->d_mb = (float *)mb; c->d_mwb = (short *)mwb;
  }
  return off;
}

static size_t arena_need(const tdh_config *cfg, const Layout &L, int nb) {
  return arena_regions(cfg, L, nb, nullptr, nullptr);
}

extern "C" size_t tdh_arena_bytes(const tdh_config *cfg, const tdh_mesh *mesh) {
  if (!cfg) return 0;
  Layout L;
  if (mesh_layout(cfg, mesh, L)) return 0;
  return arena_need(cfg, L, mesh->nblocks);
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" tdh_status tdh_init(const tdh_config *cfg, void *hip_stream, tdh_ctx **out) {
  if (!cfg || !out) return fail(nullptr, TDH_EINVAL, "tdh_init: null argument");
  if (cfg->eos_kind < 0 || cfg->eos_kind > 1) return fail(nullptr, TDH_EINVAL, "eos_kind must be 0 or 1");
  if (cfg->grav_kind < 0 || cfg->grav_kind > 2) return fail(nullptr, TDH_EINVAL, "grav_kind must be 0, 1 or 2");
  if (cfg->n_lat < 0 || cfg->n_lat > kMaxLevel) return fail(nullptr, TDH_EINVAL, "n_lat must be in [0, 30]");
  if (cfg->inv_mode < 0 || cfg->inv_mode > 4) return fail(nullptr, TDH_EINVAL, "inv_mode must be in [0, 4]");
  if (cfg->newton_max_iter < 0 || cfg->newton_max_iter > 64)
    return fail(nullptr, TDH_EINVAL, "newton_max_iter must be in [0, 64]");
  if (cfg->riemann < 0 || cfg->riemann > 1) return fail(nullptr, TDH_EINVAL, "riemann must be 0 (HLLC) or 1 (HLLE)");
  if (cfg->ghost_dense < 0 || cfg->ghost_dense > 1) return fail(nullptr, TDH_EINVAL, "ghost_dense must be 0 or 1");
  if (cfg->eos_kind == 0 && !(cfg->gamma > 1.0)) return fail(nullptr, TDH_EINVAL, "gamma must exceed 1");
  if (!(cfg->cfl > 0.0)) return fail(nullptr, TDH_EINVAL, "cfl must be positive");
  tdh_ctx *c = new tdh_ctx();
  c->cfg = *cfg;
  c->stream = (hipStream_t)hip_stream;
  c->nv = cfg->dual ? 6 : 5;
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete c;
    return fail(nullptr, TDH_EHIP, "tdh_init: no HIP device");
  }
  c->cus = prop.multiProcessorCount;
  c->scratch = device_scratch(dev);
  *out = c;
  return TDH_OK;
}

extern "C" void tdh_destroy(tdh_ctx *c) {
  if (!c) return;
  for (hipEvent_t e : c->ev) hipEventDestroy(e);
  for (auto &g : c->graphs) hipGraphExecDestroy(g.second);
  for (auto &g : c->mg_graphs) hipGraphExecDestroy(g.second);
  delete c;
}

extern "C" const char *tdh_last_error(const tdh_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

#define CHECK_CTX(c)                                                                   \
  do {                                                                                 \
    if (!(c)) return fail(nullptr, TDH_EINVAL, "null context");                        \
    if ((c)->poisoned) return fail((c), TDH_ESTATE, "context poisoned by a HIP error"); \
  } while (0)


static Phys make_phys(const tdh_config &g) {
  Phys p{};
  p.eos_kind = g.eos_kind;
  p.dual = g.dual;
  p.grav_kind = g.grav_kind;
  p.inv_mode = g.inv_mode;
  p.newton_max_iter = g.newton_max_iter;
  p.riemann = g.riemann;
  p.ghost_dense = g.ghost_dense;
  p.gamma = g.gamma;
  p.eta1 = g.eta1;
  p.eta2 = g.eta2;
  p.rho_floor = g.rho_floor;
  p.p_floor = g.p_floor;
  p.e_floor = g.e_floor;
  p.gm_bh = g.gm_bh;
  p.r_soft = g.r_soft;
  p.r_exc = g.r_exc;
  for (int d = 0; d < 3; ++d) {
    p.bh_x0[d] = g.bh_x0[d];
    p.v_frame[d] = g.v_frame[d];
  }
  return p;
}

// The second stage leaves the CFL minima of its output state on single-level
// runs with the table EOS and no point mass: under LAT (also levels a caller
// installs) the reflux after a sub-cycle still corrects blocks that have
// completed, the ideal gas's separate reduction is cheaper than the stage's
// extra work, and the point mass's term moves with time (the reduction takes
// the host's time).
static bool stage_cfl(const tdh_ctx *c) {
  return c->cfg.eos_kind == 1 && c->cfg.n_lat == 0 && c->Lmax == 0 && c->cfg.grav_kind != 2 && !c->amr;
}

static StageArgs base_args(tdh_ctx *c) {
  StageArgs a{};
  a.m.nx = c->nx;
  a.m.ny = c->ny;
  a.m.nz = c->nz;
  for (int d = 0; d < 3; ++d) {
    a.m.bc[d] = c->bc[d];
    a.m.x0[d] = c->x0[d];
    a.m.dx[d] = c->dx[d];
    a.m.inv_dx[d] = 1.0 / c->dx[d];
  }
  a.m.lat = c->lat;
  a.m.lat_shift = __builtin_ctz((unsigned)c->lat);
  a.m.lx = c->lx;
  a.m.ly = c->ly;
  a.m.lz = c->lz;
  a.m.amr = c->amr ? 1 : 0;
  a.m.nv = c->nv;
  a.m.lmap = c->d_lmap;
  a.m.blocks = c->d_blocks;
  a.p = make_phys(c->cfg);
  a.t = c->tab;
  a.s = c->seed;
  a.Qa = c->Qa;
  a.Qb = c->Qb;
  a.Qs = c->Qs;
  a.imp = c->imp;
  a.bf1 = c->bf1;
  a.phi = c->phi;
  a.fac = c->d_fac;
  a.par = c->d_par;
  a.order = c->d_order;
  a.item_start = c->d_item_start;
  a.cnt_ge = c->d_cnt_ge;
  a.win = c->d_win;
  a.jc = c->jc;
  a.jn = c->ncells;
  a.flx = c->flx;
  a.fstride = (long long)(c->nv + 1) * c->ftotal;
  a.fitem_start = c->d_fitem_start;
  a.item_bt = c->d_item_bt;
  a.fitem_bt = c->d_fitem_bt;
  a.cfl_part = stage_cfl(c) ? c->d_cfl_part : nullptr;
  a.cfl_start = c->d_cfl_block_start;
  a.lmax = c->Lmax;
  return a;
}

// face/edge/corner adjacency through the lattice (periodic wrap, nothing beyond
// outflow edges), whatever the refinement levels: the lattice cells (level-0
// units) around each block's extent
static void build_adjacency(tdh_ctx *c) {
  c->adj.assign(c->nb, {});
  const int L = c->lat;
  const int N[3] = {c->nx, c->ny, c->nz};
  for (int b = 0; b < c->nb; ++b) {
    const int r = c->rl[b];
    const int n = c->blk[4 * b] >> r;
    const int o[3] = {c->blk[4 * b + 1] >> r, c->blk[4 * b + 2] >> r, c->blk[4 * b + 3] >> r};
    std::vector<int> &A = c->adj[b];
    for (int cz = o[2] - L; cz < o[2] + n + L; cz += L)
      for (int cy = o[1] - L; cy < o[1] + n + L; cy += L)
        for (int cx = o[0] - L; cx < o[0] + n + L; cx += L) {
          int g[3] = {cx, cy, cz};
          bool ok = true;
          for (int d = 0; d < 3; ++d) {
            if (c->bc[d] == 0) g[d] = ((g[d] % N[d]) + N[d]) % N[d];
            else if (g[d] < 0 || g[d] >= N[d]) ok = false;
          }
          if (!ok) continue;
          const int nb2 = c->lmap[((g[2] / L) * c->ly + g[1] / L) * c->lx + g[0] / L];
          if (nb2 != b && std::find(A.begin(), A.end(), nb2) == A.end()) A.push_back(nb2);
        }
  }
}

static bool tile_fits(const tdh_ctx *c, int id);

// device copies of the level-dependent tables; starts a new window
static tdh_status install_levels(tdh_ctx *c, const std::vector<int> &lev) {
  if (c->have_mesh && lev == c->levels) {  // same assignment: the device tables are current
    c->k = 0;
    return TDH_OK;
  }
  c->levels = lev;
  c->Lmax = 0;
  for (int l : lev) c->Lmax = std::max(c->Lmax, l);
  c->fac.resize(c->nb);
  for (int b = 0; b < c->nb; ++b) c->fac[b] = 1 << (c->Lmax - lev[b]);
  c->order.resize(c->nb);
  for (int b = 0; b < c->nb; ++b) c->order[b] = b;
  std::stable_sort(c->order.begin(), c->order.end(), [&](int x, int y) { return lev[x] > lev[y]; });
  c->item_start.assign(c->nb + 1, 0);
  c->fitem_start.assign(c->nb + 1, 0);
  for (int i = 0; i < c->nb; ++i) {
    const long long n = c->blk[4 * c->order[i]];
    c->item_start[i + 1] = c->item_start[i] + (int)((n * n * n + kChunk - 1) / kChunk);
    c->fitem_start[i + 1] = c->fitem_start[i] + (int)(((n + 1) * n * n + kChunk - 1) / kChunk);
  }
  c->cnt_ge.assign(kCntSlots, 0);
  for (int L = 0; L < kCntSlots; ++L)
    for (int b = 0; b < c->nb; ++b)
      if (lev[b] >= L) c->cnt_ge[L]++;
  HIPCHK(c, hipMemcpyAsync(c->d_fac, c->fac.data(), c->nb * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_order, c->order.data(), c->nb * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_item_start, c->item_start.data(), (c->nb + 1) * sizeof(int), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_fitem_start, c->fitem_start.data(), (c->nb + 1) * sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
  // the per-item tables (block, item within the block) are expanded on the
  // device from the lists just uploaded
  HIPCHK(c, launch_expand_items(c->d_order, c->d_item_start, c->nb, c->d_item_bt, c->stream));
  HIPCHK(c, launch_expand_items(c->d_order, c->d_fitem_start, c->nb, c->d_fitem_bt, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_cnt_ge, c->cnt_ge.data(), kCntSlots * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->k = 0;
  return TDH_OK;
}

extern "C" tdh_status tdh_init_blocks(tdh_ctx *c, const tdh_mesh *m, void *dev_arena, size_t arena_bytes,
                                      const double *host_state, const double *host_phi) {
  CHECK_CTX(c);
  if (c->have_mesh) return fail(c, TDH_ESTATE, "tdh_init_blocks: mesh already installed");
  Layout L;
  if (const char *why = mesh_layout(&c->cfg, m, L)) return fail(c, TDH_EINVAL, "tdh_init_blocks: %s", why);
  if (!dev_arena || ((uintptr_t)dev_arena & 255)) return fail(c, TDH_EINVAL, "arena must be non-null, 256-byte aligned");
  if (arena_bytes < arena_need(&c->cfg, L, m->nblocks))
    return fail(c, TDH_ENOMEM, "arena holds %zu bytes, %zu needed", arena_bytes, arena_need(&c->cfg, L, m->nblocks));
  if (!host_state) return fail(c, TDH_EINVAL, "host_state is null");
  if (c->cfg.grav_kind == 1 && !host_phi) return fail(c, TDH_EINVAL, "grav_kind 1 needs host_phi");
  c->nx = m->nx; c->ny = m->ny; c->nz = m->nz;
  for (int d = 0; d < 3; ++d) { c->bc[d] = m->bc[d]; c->x0[d] = m->x0[d]; c->dx[d] = m->dx[d]; }
  c->nb = m->nblocks;
  c->blk.assign(m->blk, m->blk + 4 * m->nblocks);
  c->rl.assign(c->nb, 0);
  if (m->rlev) c->rl.assign(m->rlev, m->rlev + c->nb);
  c->amr = std::any_of(c->rl.begin(), c->rl.end(), [](int r) { return r != 0; });
  c->lat = L.lat;
  c->nmax = L.nmax;
  c->lx = c->nx / c->lat; c->ly = c->ny / c->lat; c->lz = c->nz / c->lat;
  c->lmap.assign((size_t)c->lx * c->ly * c->lz, -1);
  for (int b = 0; b < c->nb; ++b) {
    const int n = c->blk[4 * b], ox = c->blk[4 * b + 1], oy = c->blk[4 * b + 2], oz = c->blk[4 * b + 3];
    const int r = c->rl[b], Lr = c->lat << r;  // lattice edge in this block's cells
    if (ox % Lr || oy % Lr || oz % Lr || ox < 0 || oy < 0 || oz < 0 || ox + n > (c->nx << r) ||
        oy + n > (c->ny << r) || oz + n > (c->nz << r))
      return fail(c, TDH_EINVAL, "block %d is not aligned to the lattice or leaves the domain", b);
    for (int z = oz / Lr; z < (oz + n) / Lr; ++z)
      for (int y = oy / Lr; y < (oy + n) / Lr; ++y)
        for (int x = ox / Lr; x < (ox + n) / Lr; ++x) {
          int &slot = c->lmap[((size_t)z * c->ly + y) * c->lx + x];
          if (slot != -1) return fail(c, TDH_EINVAL, "blocks %d and %d overlap", slot, b);
          slot = b;
        }
  }
  for (int v : c->lmap)
    if (v < 0) return fail(c, TDH_EINVAL, "the blocks do not cover the domain");
  c->binfo.resize(c->nb);
  for (int b = 0; b < c->nb; ++b) {
    BlockInfo &B = c->binfo[b];
    B.n = c->blk[4 * b]; B.ox = c->blk[4 * b + 1]; B.oy = c->blk[4 * b + 2]; B.oz = c->blk[4 * b + 3];
    B.lev = c->rl[b];
    B.pad_ = 0;
    B.off = L.off[b]; B.poff = L.poff[b]; B.ioff = L.ioff[b]; B.foff = L.foff[b];
  }
  c->total = L.total; c->ptotal = L.ptotal; c->itotal = L.itotal; c->ncells = L.ncells;
  // carve the arena: the library allocates no device memory
  arena_regions(&c->cfg, L, c->nb, (char *)dev_arena, c);
  c->ftotal = L.ftotal;
  std::vector<int> cstart(c->nb + 1, 0), citem;
  for (int b = 0; b < c->nb; ++b) {
    const long long n = c->blk[4 * b];
    const int ni = (int)((n * n * n + kChunk - 1) / kChunk);
    cstart[b + 1] = cstart[b] + ni;
    for (int i = 0; i < ni; ++i) citem.push_back(b);
  }
  c->cfl_nitems = cstart[c->nb];
  HIPCHK(c, hipMemcpyAsync(c->d_blocks, c->binfo.data(), c->nb * sizeof(BlockInfo), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_lmap, c->lmap.data(), c->lmap.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_cfl_block_start, cstart.data(), cstart.size() * sizeof(int), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_cfl_item_block, citem.data(), citem.size() * sizeof(int), hipMemcpyHostToDevice,
                           c->stream));
  c->par.assign(c->nb, 0);
  HIPCHK(c, hipMemcpyAsync(c->d_par, c->par.data(), c->nb * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->Qa, host_state, L.total * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (c->jc) HIPCHK(c, hipMemsetAsync(c->jc, 0xff, 3 * L.ncells * sizeof(int), c->stream));  // no seeds yet (-1)
  c->seeds_held = false;
  c->cfl_seeds = false;
  c->cfl_parts = false;
  if (c->phi) HIPCHK(c, hipMemcpyAsync(c->phi, host_phi, L.ptotal * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->h_dtb.assign(c->nb, 0.0);
  build_adjacency(c);
  for (int b = 0; b < c->nb; ++b)
    if (c->blk[4 * b] < 8) return fail(c, TDH_EINVAL, "blocks must have an edge of at least 8 cells");
  c->tile = 0;
  while (c->tile < num_tiles() && !tile_fits(c, c->tile)) c->tile++;
  c->have_mesh = true;
  return install_levels(c, std::vector<int>(c->nb, 0));
}

// Packed EOS table (see Table in tdh_internal.hpp), in doubles: density-row
// pairs of log e, then of (log P, log c_s^2), then the 128-byte cell records,
// then the log10 and 10^x function tables.
struct TableLayout {
  size_t pc_off, rec_off, fn_off, total;
};
static TableLayout table_layout(int nrho, int nT) {
  TableLayout t;
  const size_t np = (size_t)(nrho - 1) * nT;
  t.pc_off = (2 * np + 3) & ~(size_t)3;              // 32-byte alignment of the double4 records
  t.rec_off = (t.pc_off + 4 * np + 15) & ~(size_t)15;  // 128-byte cell records
  const size_t nrec = (size_t)(nrho - 1) * (nT - 1);
  t.fn_off = t.rec_off + 16 * nrec;                    // 128-byte aligned
  t.total = t.fn_off + 2 * 128 + 64;
  return t;
}

extern "C" size_t tdh_table_bytes(int nrho, int nT) {
  if (nrho < 2 || nT < 2 || nrho > 4096 || nT > 4096) return 0;
  return table_layout(nrho, nT).total * sizeof(double);
}

extern "C" tdh_status tdh_set_eos_table(tdh_ctx *c, int nrho, int nT, double lr0, double dlr, double lT0, double dlT,
                                        const double *lP, const double *le, const double *lc2, void *dev_table,
                                        size_t table_bytes) {
  CHECK_CTX(c);
  if (nrho < 2 || nT < 2 || nrho > 4096 || nT > 4096) return fail(c, TDH_ERANGE, "table dimensions out of range");
  if (!lP || !le || !lc2) return fail(c, TDH_EINVAL, "null table array");
  if (!dev_table || ((uintptr_t)dev_table & 255))
    return fail(c, TDH_EINVAL, "table buffer must be non-null, 256-byte aligned");
  if (table_bytes < tdh_table_bytes(nrho, nT))
    return fail(c, TDH_ENOMEM, "table buffer holds %zu bytes, %zu needed", table_bytes, tdh_table_bytes(nrho, nT));
  if (!(dlr > 0.0) || !(dlT > 0.0)) return fail(c, TDH_EINVAL, "table spacings must be positive");
  for (int i = 0; i < nrho; ++i)
    for (int j = 0; j + 1 < nT; ++j)
      if (!(le[(size_t)i * nT + j + 1] > le[(size_t)i * nT + j]))
        return fail(c, TDH_EINVAL, "log e is not increasing in T on row %d", i);
  // pack by density-row pairs
  const TableLayout TL = table_layout(nrho, nT);
  const size_t pc_off = TL.pc_off, rec_off = TL.rec_off, fn_off = TL.fn_off;
  std::vector<double> packed(TL.total, 0.0);
  // log10 and 10^x tables, from the host's extended-precision library
  for (int i = 0; i < 128; ++i) {
    const double ci = 1.0 / (1.0 + (i + 0.5) / 128.0);
    packed[fn_off + 2 * i] = 2.0 * ci;
    packed[fn_off + 2 * i + 1] = (double)-log10l((long double)ci);
  }
  for (int j = 0; j < 64; ++j) packed[fn_off + 256 + j] = (double)exp2l((long double)j / 64.0L);
  for (int i = 0; i + 1 < nrho; ++i)
    for (int j = 0; j < nT; ++j) {
      const size_t a = (size_t)i * nT + j, b = (size_t)(i + 1) * nT + j, q = (size_t)i * nT + j;
      packed[2 * q] = le[a];
      packed[2 * q + 1] = le[b];
      double *pcq = packed.data() + pc_off + 4 * q;
      pcq[0] = lP[a];
      pcq[1] = lP[b];
      pcq[2] = lc2[a];
      pcq[3] = lc2[b];
    }
  for (int i = 0; i + 1 < nrho; ++i)
    for (int j = 0; j + 1 < nT; ++j) {
      double *r = packed.data() + rec_off + 16 * ((size_t)i * (nT - 1) + j);
      const size_t q = (size_t)i * nT + j;
      r[0] = packed[2 * q];
      r[1] = packed[2 * q + 1];
      r[2] = packed[2 * (q + 1)];
      r[3] = packed[2 * (q + 1) + 1];
      for (int v = 0; v < 4; ++v) {
        r[4 + v] = packed[pc_off + 4 * q + v];
        r[8 + v] = packed[pc_off + 4 * (q + 1) + v];
      }
    }
  c->d_table = (double *)dev_table;
  HIPCHK(c, hipMemcpyAsync(c->d_table, packed.data(), packed.size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->tab.nrho = nrho;
  c->tab.nT = nT;
  c->tab.lr0 = lr0;
  c->tab.dlr = dlr;
  c->tab.inv_dlr = 1.0 / dlr;
  c->tab.lT0 = lT0;
  c->tab.dlT = dlT;
  c->tab.le2 = (const double2 *)c->d_table;
  c->tab.pc = (const double4 *)(c->d_table + pc_off);
  c->tab.rec = c->d_table + rec_off;
  c->tab.lg = (const double2 *)(c->d_table + fn_off);
  c->tab.ex = c->d_table + fn_off + 256;
  c->have_table = true;
  c->seeds_held = false;  // cells of another table
  c->cfl_seeds = false;
  c->cfl_parts = false;
  for (auto &g : c->graphs) hipGraphExecDestroy(g.second);
  c->graphs.clear();
  return TDH_OK;
}

static tdh_status ready(tdh_ctx *c) {
  if (!c->have_mesh) return fail(c, TDH_ESTATE, "no mesh: call tdh_init_blocks first");
  if (c->cfg.eos_kind == 1 && !c->have_table) return fail(c, TDH_ESTATE, "tabulated EOS selected but no table set");
  return TDH_OK;
}

// ---------------------------------------------------------------------------
// LAT level assignment (eq lat-factor, bin merging, neighbour limit)
// ---------------------------------------------------------------------------
static std::vector<int> assign_levels(const tdh_ctx *c, const std::vector<double> &dtb, double &dt0) {
  const int nb = c->nb;
  dt0 = INFINITY;
  for (double v : dtb) dt0 = std::min(dt0, v);
  std::vector<int> e(nb);
  for (int b = 0; b < nb; ++b) {
    // floor(log2(dt_b / dt0)) exactly, from the binary exponent of the ratio
    int ex = std::ilogb(dtb[b] / dt0);
    e[b] = std::max(0, std::min(c->cfg.n_lat, ex));
  }
  for (;;) {  // merge sparsely filled top bins into the next lower one
    int top = *std::max_element(e.begin(), e.end());
    if (top == 0) break;
    int cnt = (int)std::count(e.begin(), e.end(), top);
    if ((double)cnt >= c->cfg.merge_frac * nb) break;
    for (int &v : e)
      if (v == top) v = top - 1;
  }
  // neighbour limits, relaxed to their fixed point (the greatest admissible
  // exponents below the CFL bins): one exponent apart on one refinement level;
  // across levels f_fine <= f_coarse <= 2 f_fine, i.e. a fine block's exponent
  // at most its coarse neighbour's, a coarse block's at most one above
  for (bool changed = true; changed;) {
    changed = false;
    for (int b = 0; b < nb; ++b)
      for (int n : c->adj[b]) {
        const int cap = c->rl[b] > c->rl[n] ? e[n] : e[n] + 1;
        if (e[b] > cap) { e[b] = cap; changed = true; }
      }
  }
  const int L = *std::max_element(e.begin(), e.end());
  std::vector<int> lev(nb);
  for (int b = 0; b < nb; ++b) lev[b] = L - e[b];
  return lev;
}

static tdh_status require_window_boundary(tdh_ctx *c) {
  if (c->k != 0) return fail(c, TDH_ESTATE, "a LAT window is in progress (sub-cycle %d)", c->k);
  return TDH_OK;
}

// The CFL reduction of tdh_reduce_dt and tdh_reduce_dt_static: per-item
// partial minima into part, per-block steps into dtb (device), then the level
// assignment on the host.  stage_minima: take the minima the last window's
// second stages left, where they hold this state's (the same values).
static tdh_status reduce_dt_impl(tdh_ctx *c, double *part, double *dtb_dev, bool stage_minima, double *host_dtb,
                                 double *host_dt0, int8_t *host_levels, int *host_lmax) {
  tdh_status s;
  if ((s = ready(c)) || (s = require_window_boundary(c))) return s;
  StageArgs a = base_args(c);
  if (stage_minima && c->cfl_parts) {  // the last window's second stages left the tile minima of this state
    HIPCHK(c, launch_cfl_blocks(c->d_cfl_part, c->nb, c->d_cfl_block_start, c->cfg.cfl, dtb_dev, c->stream));
    c->stats.kernel_launches += 1;
  } else {
    HIPCHK(c, launch_cfl(a, c->cfg.cfl, c->t, c->d_cfl_item_block, c->cfl_nitems, part, c->nb,
                         c->d_cfl_block_start, dtb_dev, c->cus, c->stream));
    c->stats.kernel_launches += 2;
    c->cfl_seeds = c->cfg.eos_kind == 1 && (c->cfg.inv_mode == 2 || c->cfg.inv_mode == 4);
  }
  HIPCHK(c, hipMemcpyAsync(c->h_dtb.data(), dtb_dev, c->nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double> dtb(c->h_dtb.begin(), c->h_dtb.end());
  double dt0;
  std::vector<int> lev = c->cfg.n_lat > 0 ? assign_levels(c, dtb, dt0) : std::vector<int>(c->nb, 0);
  if (c->cfg.n_lat == 0) {
    dt0 = INFINITY;
    for (double v : dtb) dt0 = std::min(dt0, v);
  }
  if (!(dt0 > 0.0) || !std::isfinite(dt0)) return fail(c, TDH_ERANGE, "CFL step is not a positive finite number");
  if ((s = install_levels(c, lev))) return s;
  if (host_dtb) std::copy(dtb.begin(), dtb.end(), host_dtb);
  if (host_dt0) *host_dt0 = dt0;
  if (host_levels)
    for (int b = 0; b < c->nb; ++b) host_levels[b] = (int8_t)lev[b];
  if (host_lmax) *host_lmax = c->Lmax;
  return TDH_OK;
}

extern "C" tdh_status tdh_reduce_dt(tdh_ctx *c, double *host_dtb, double *host_dt0, int8_t *host_levels,
                                    int *host_lmax) {
  CHECK_CTX(c);
  return reduce_dt_impl(c, c->d_cfl_part, c->d_dtb, true, host_dtb, host_dt0, host_levels, host_lmax);
}

extern "C" tdh_status tdh_reduce_dt_static(tdh_ctx *c, double *host_dtb, double *host_dt0, int8_t *host_levels,
                                           int *host_lmax) {
  CHECK_CTX(c);
  if (!c->scratch) return fail(c, TDH_ESTATE, "the device scratch of this context's GPU was not resolved");
  if (!c->have_mesh) return fail(c, TDH_ESTATE, "no mesh: call tdh_init_blocks first");
  const long long need = (long long)c->cfl_nitems + c->nb;
  if (need > (long long)kScratchDoubles)
    return fail(c, TDH_ERANGE, "tdh_reduce_dt_static: %lld work items + %d blocks exceed the %lld-double device scratch "
                               "(meshes up to about 134 M cells)", (long long)c->cfl_nitems, c->nb,
                (long long)kScratchDoubles);
  // every value is written before it is read: nothing needs clearing
  return reduce_dt_impl(c, c->scratch, c->scratch + c->cfl_nitems, false, host_dtb, host_dt0, host_levels, host_lmax);
}

extern "C" tdh_status tdh_set_levels(tdh_ctx *c, const int8_t *host_levels) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = ready(c)) || (s = require_window_boundary(c))) return s;
  if (!host_levels) return fail(c, TDH_EINVAL, "null levels");
  std::vector<int> lev(c->nb);
  for (int b = 0; b < c->nb; ++b) {
    lev[b] = host_levels[b];
    if (lev[b] < 0 || lev[b] > kMaxLevel) return fail(c, TDH_EINVAL, "level of block %d outside [0, 30]", b);
  }
  for (int b = 0; b < c->nb; ++b)
    for (int n : c->adj[b]) {
      if (std::abs(lev[b] - lev[n]) > 1)
        return fail(c, TDH_EINVAL, "neighbours %d and %d differ by more than one level", b, n);
      // a finer block never takes a longer step than its coarser neighbour
      if (c->rl[b] > c->rl[n] && lev[b] < lev[n])
        return fail(c, TDH_EINVAL, "block %d (refined) steps longer than its coarser neighbour %d", b, n);
    }
  return install_levels(c, lev);
}

// ---------------------------------------------------------------------------
// stepping
// ---------------------------------------------------------------------------
static int ctz(int v) { return __builtin_ctz((unsigned)v); }

static int lmin_of(int k, int Lmax) { return k == 0 ? 0 : Lmax - ctz(k); }

static tdh_status collect_timing(tdh_ctx *c) {
  if (c->ev_used == 0) return TDH_OK;
  HIPCHK(c, hipEventSynchronize(c->ev[2 * c->ev_used - 1]));
  for (size_t i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
    c->stage_ms += ms;
    c->stage_launches++;
  }
  c->ev_used = 0;
  return TDH_OK;
}

static tdh_status timed_stage(tdh_ctx *c, const StageArgs &a) {
  const bool t = c->timing && !c->capturing;
  tdh_status s;
  if (c->cfg.eos_kind == 1 && (c->cfg.inv_mode == 2 || c->cfg.inv_mode == 4) && !(a.k == 0 && a.phase == 1)) {
    HIPCHK(c, launch_seed(a, c->cus, c->stream));
    c->stats.kernel_launches++;
  }
  if (t && 2 * (c->ev_used + 1) > c->ev.size())
    if ((s = collect_timing(c))) return s;
  if (t) HIPCHK(c, hipEventRecord(c->ev[2 * c->ev_used], c->stream));
  HIPCHK(c, launch_stage(a, c->tile, c->cus, c->stream));
  if (t) {
    HIPCHK(c, hipEventRecord(c->ev[2 * c->ev_used + 1], c->stream));
    c->ev_used++;
  }
  c->stats.kernel_launches++;
  return TDH_OK;
}

// Seeds of a window's first stage.  Modes 1 and 3 carry seed cells from stage
// to stage; after a state upload a pass over every block finds them once.
// Modes 2 and 4 take them from the CFL pass when it ran on this state, else
// from a pass over every block here.  Outside any captured graph, so a
// window's graph never holds its first seed pass.
static tdh_status ensure_seeds(tdh_ctx *c) {
  if (c->cfg.eos_kind != 1) return TDH_OK;
  const bool carried = c->cfg.inv_mode == 1 || c->cfg.inv_mode == 3;
  const bool per_stage = c->cfg.inv_mode == 2 || c->cfg.inv_mode == 4;
  c->cfl_parts = false;  // this window's second stages overwrite them
  if (!(carried && !c->seeds_held) && !(per_stage && !c->cfl_seeds)) {
    c->cfl_seeds = false;  // consumed by this window
    return TDH_OK;
  }
  StageArgs a = base_args(c);
  a.k = 0;
  a.phase = 1;
  a.Llo = 0;
  a.Lhi = kCntSlots - 2;
  HIPCHK(c, launch_seed(a, c->cus, c->stream));
  c->stats.kernel_launches++;
  if (carried) c->seeds_held = true;
  c->cfl_seeds = false;
  c->cfl_parts = false;
  return TDH_OK;
}

// enqueue sub-cycle k of the current window
static tdh_status enqueue_subcycle(tdh_ctx *c, int k, bool batched) {
  tdh_status s;
  const int lmin = lmin_of(k, c->Lmax);
  StageArgs a = base_args(c);
  a.k = k;
  for (int phase = 1; phase <= 2; ++phase) {
    a.phase = phase;
    if (batched) {
      a.Llo = lmin;
      a.Lhi = kCntSlots - 2;
      if ((s = timed_stage(c, a))) return s;
    } else {
      for (int L = lmin; L <= c->Lmax; ++L) {
        a.Llo = L;
        a.Lhi = L;
        if ((s = timed_stage(c, a))) return s;
      }
    }
  }
  HIPCHK(c, launch_commit(c->d_order, c->d_cnt_ge, lmin, c->d_par, c->stream));
  c->stats.kernel_launches++;
  if (c->Lmax > 0 || c->amr) {  // coarse-fine faces are corrected on every coarse step
    const int fmax = 1 << c->Lmax;
    const int lc = (k + 1 == fmax) ? 0 : c->Lmax - ctz(k + 1);
    a.k = k + 1;
    for (int d = 0; d < 3; ++d) {
      HIPCHK(c, launch_reflux(a, lc, d, c->nmax, 1024, c->stream));
      c->stats.kernel_launches++;
    }
  }
  return TDH_OK;
}

static void account_subcycle(tdh_ctx *c, int k) {
  const int lmin = lmin_of(k, c->Lmax);
  for (int b = 0; b < c->nb; ++b)
    if (c->levels[b] >= lmin) {
      c->par[b] ^= 1;
      const long long n = c->blk[4 * b];
      c->stats.block_updates++;
      c->stats.cell_updates += n * n * n;
    }
  c->stats.sub_cycles++;
}

static void finish_window(tdh_ctx *c) {
  // a fused-form window leaves the CFL minima of its output state and, in modes
  // 2 and 4, that state's table cells (every block's last second stage is in it)
  c->cfl_parts = stage_cfl(c) && tile_is_fused(c->tile);
  c->cfl_seeds = c->cfl_parts && c->cfg.eos_kind == 1 && (c->cfg.inv_mode == 2 || c->cfg.inv_mode == 4);
  c->t = c->t + c->dt_coarse;
  c->k = 0;
  c->stats.windows++;
}

extern "C" tdh_status tdh_step_level(tdh_ctx *c, int level, double dt) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = ready(c))) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, TDH_EINVAL, "dt must be positive and finite");
  const int want = lmin_of(c->k, c->Lmax);
  if (level != want) return fail(c, TDH_ESTATE, "sub-cycle %d of the window advances level %d, not %d", c->k, want, level);
  if (c->k == 0) {
    c->dt_coarse = dt;
    c->dt0 = std::ldexp(dt, -c->Lmax);
    HIPCHK(c, launch_set_window(c->d_win, c->t, c->dt0, c->stream));
    if ((s = ensure_seeds(c))) return s;
  } else if (std::ldexp(dt, level) != c->dt_coarse) {
    return fail(c, TDH_EINVAL, "dt * 2^level must equal the window's coarse step");
  }
  if ((s = enqueue_subcycle(c, c->k, true))) return s;
  account_subcycle(c, c->k);
  c->k++;
  if (c->k == (1 << c->Lmax)) finish_window(c);
  return TDH_OK;
}

extern "C" tdh_status tdh_run_window(tdh_ctx *c, double dt_coarse, int batched, int use_graph) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = ready(c)) || (s = require_window_boundary(c))) return s;
  if (!(dt_coarse > 0.0) || !std::isfinite(dt_coarse)) return fail(c, TDH_EINVAL, "dt must be positive and finite");
  c->dt_coarse = dt_coarse;
  c->dt0 = std::ldexp(dt_coarse, -c->Lmax);
  const int nsub = 1 << c->Lmax;
  HIPCHK(c, launch_set_window(c->d_win, c->t, c->dt0, c->stream));
  if ((s = ensure_seeds(c))) return s;
  if (use_graph) {
    // The graph holds the window's launches for this Lmax; the window time,
    // step and the level-dependent work lists live in device memory, so one
    // capture serves every later window with the same Lmax.
    const auto key = std::make_pair(c->Lmax, batched ? 1 : 0);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
      HIPCHK(c, hipGraphLaunch(it->second, c->stream));
      for (int k = 0; k < nsub; ++k) account_subcycle(c, k);
      c->stats.kernel_launches += 1;
      finish_window(c);
      return TDH_OK;
    }
    hipGraph_t g;
    const auto t_cap = std::chrono::steady_clock::now();
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    for (int k = 0; k < nsub; ++k) {
      if ((s = enqueue_subcycle(c, k, batched != 0))) {
        hipGraph_t dummy;
        hipStreamEndCapture(c->stream, &dummy);
        c->capturing = false;
        return s;
      }
    }
    c->capturing = false;
    HIPCHK(c, hipStreamEndCapture(c->stream, &g));
    hipGraphExec_t ge;
    HIPCHK(c, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    hipGraphDestroy(g);
    c->graphs[key] = ge;
    c->stats.graph_captures++;
    c->stats.capture_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_cap).count();
    HIPCHK(c, hipGraphLaunch(ge, c->stream));
  } else {
    for (int k = 0; k < nsub; ++k)
      if ((s = enqueue_subcycle(c, k, batched != 0))) return s;
  }
  for (int k = 0; k < nsub; ++k) account_subcycle(c, k);
  finish_window(c);
  return TDH_OK;
}

extern "C" tdh_status tdh_get_time(tdh_ctx *c, double *t) {
  CHECK_CTX(c);
  if (!t) return fail(c, TDH_EINVAL, "null output");
  *t = c->t;
  return TDH_OK;
}

extern "C" tdh_status tdh_set_time(tdh_ctx *c, double t) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = require_window_boundary(c))) return s;
  c->t = t;
  return TDH_OK;
}

extern "C" tdh_status tdh_get_state(tdh_ctx *c, double *host) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = ready(c))) return s;
  if (!host) return fail(c, TDH_EINVAL, "null output");
  if (c->k != 0) return fail(c, TDH_ESTATE, "state is only defined between windows");
  for (int b = 0; b < c->nb; ++b) {
    const long long n = c->blk[4 * b];
    const double *src = (c->par[b] ? c->Qb : c->Qa) + c->binfo[b].off;
    HIPCHK(c, hipMemcpyAsync(host + c->binfo[b].off, src, c->nv * n * n * n * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TDH_OK;
}

// ---------------------------------------------------------------------------
// self-gravity: multigrid solve into the stored potential (Sec. Self-gravity solver)
// ---------------------------------------------------------------------------
namespace {
struct MgPlan {
  int nlev = 0;
  MgLevel lv[kMgMaxLevels];
  double *part = nullptr, *scal = nullptr;  // sum partials; mean density, defect norm, mean potential
  size_t bytes = 0;
};
}  // namespace

// levels halve every axis while all are even and at least 4; the layout puts the
// finest potential first (the warm start of the next solve)
static tdh_status mg_plan(tdh_ctx *c, char *base, MgPlan *P) {
  if (c->cfg.grav_kind != 1 || !c->phi)
    return fail(c, TDH_ESTATE, "the self-gravity solve writes the stored potential: grav_kind must be 1");
  for (int d = 0; d < 3; ++d)
    if (c->bc[d] != 0) return fail(c, TDH_EINVAL, "the self-gravity solve needs periodic boundaries on every axis");
  int nx = c->nx, ny = c->ny, nz = c->nz;
  int nlev = 0;
  for (;;) {
    if ((nx & 1) || (ny & 1) || (nz & 1))
      return fail(c, TDH_EINVAL, "multigrid level %d has an odd dimension (%d x %d x %d)", nlev, nx, ny, nz);
    MgLevel &L = P->lv[nlev];
    L.nx = nx; L.ny = ny; L.nz = nz;
    const double s = (double)(1 << nlev);
    const double hx = c->dx[0] * s, hy = c->dx[1] * s, hz = c->dx[2] * s;
    L.hx2 = hx * hx;
    L.wy = (hx / hy) * (hx / hy);
    L.wz = (hx / hz) * (hx / hz);
    L.c0 = 2.0 * (1.0 + L.wy + L.wz);
    ++nlev;
    if (nlev == kMgMaxLevels || nx < 4 || ny < 4 || nz < 4) break;
    nx /= 2; ny /= 2; nz /= 2;
  }
  const MgLevel &Cl = P->lv[nlev - 1];
  if ((long long)Cl.nx * Cl.ny * Cl.nz > mg_coarse_max())
    return fail(c, TDH_ERANGE, "coarsest multigrid level %d x %d x %d exceeds %d cells", Cl.nx, Cl.ny, Cl.nz,
                mg_coarse_max());
  P->nlev = nlev;
  size_t off = 0;  // doubles
  auto take = [&](long long n) { double *p = base ? (double *)base + off : nullptr; off += (size_t)((n + 31) & ~31LL); return p; };
  for (int l = 0; l < nlev; ++l) {
    MgLevel &L = P->lv[l];
    const long long n = (long long)L.nx * L.ny * L.nz;
    L.phi = take(n);
    L.src = take(n);
    L.rphi = l > 0 ? take(n) : nullptr;
  }
  P->part = take(kMgSumParts);
  P->scal = take(4);
  P->bytes = off * sizeof(double);
  return TDH_OK;
}

static hipError_t mg_vcycle(const MgPlan &P, int l, hipStream_t s) {
  hipError_t e;
  const MgLevel &L = P.lv[l];
  if (l == P.nlev - 1) {
    const int t = L.nx + L.ny + L.nz;
    return mg_launch_coarse_solve(L, 2 * t * t, s);
  }
  const MgLevel &C = P.lv[l + 1];
  if ((e = mg_launch_sweep(L, s)) || (e = mg_launch_sweep(L, s)) || (e = mg_launch_restrict(L, C, s)) || (e = mg_vcycle(P, l + 1, s)) || (e = mg_launch_prolong(L, C, s)) ||
      (e = mg_launch_sweep(L, s)) || (e = mg_launch_sweep(L, s)))
    return e;
  return hipSuccess;
}

extern "C" tdh_status tdh_gravity_workspace_bytes(tdh_ctx *c, size_t *host_bytes) {
  CHECK_CTX(c);
  tdh_status st;
  if ((st = ready(c))) return st;
  if (!host_bytes) return fail(c, TDH_EINVAL, "null output");
  if (c->amr) return fail(c, TDH_EINVAL, "the self-gravity solve needs a single-level mesh");
  MgPlan P;
  if ((st = mg_plan(c, nullptr, &P))) return st;
  *host_bytes = P.bytes;
  return TDH_OK;
}

extern "C" tdh_status tdh_gravity_solve(tdh_ctx *c, void *dev_work, size_t bytes, double four_pi_G, int max_cycles,
                                        double tol, int warm, int *host_cycles, double *host_defects) {
  CHECK_CTX(c);
  tdh_status st;
  if ((st = ready(c)) || (st = require_window_boundary(c))) return st;
  if (!dev_work) return fail(c, TDH_EINVAL, "null workspace");
  if (c->amr) return fail(c, TDH_EINVAL, "the self-gravity solve needs a single-level mesh");
  if (!std::isfinite(four_pi_G) || !(tol >= 0.0) || max_cycles < 0 || max_cycles > 1000)
    return fail(c, TDH_EINVAL, "four_pi_G must be finite, tol >= 0 and max_cycles in [0, 1000]");
  MgPlan P;
  if ((st = mg_plan(c, (char *)dev_work, &P))) return st;
  if (bytes < P.bytes) return fail(c, TDH_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, P.bytes);
  const StageArgs a = base_args(c);
  const MgLevel &F = P.lv[0];
  const long long N = (long long)F.nx * F.ny * F.nz;
  const double invN = 1.0 / (double)N;
  hipStream_t s = c->stream;
  HIPCHK(c, mg_launch_gather(a.m, c->d_par, c->Qa, c->Qb, F, s));
  HIPCHK(c, mg_launch_sum(F.src, N, 0, invN, 0, P.part, P.scal + 0, s));
  HIPCHK(c, mg_launch_source(F.src, P.scal + 0, four_pi_G, N, s));
  // a second pass removes the first one's rounding residue from the null space
  HIPCHK(c, mg_launch_sum(F.src, N, 0, invN, 0, P.part, P.scal + 3, s));
  HIPCHK(c, mg_launch_affine(F.src, P.scal + 3, 0.0, N, s));
  if (!warm) HIPCHK(c, mg_launch_affine(F.phi, nullptr, 0.0, N, s));
  auto norm = [&](double *out) -> hipError_t {
    hipError_t e;
    if ((e = mg_launch_defect_norm(F, P.part, P.scal + 1, s))) return e;
    if ((e = hipMemcpyAsync(out, P.scal + 1, sizeof(double), hipMemcpyDeviceToHost, s))) return e;
    return hipStreamSynchronize(s);
  };
  double d = 0.0;
  HIPCHK(c, norm(&d));
  if (host_defects) host_defects[0] = d;
  // one cycle (V-cycle, the extra finest sweep, the defect norm) is captured
  // once per workspace and replayed: about a hundred launches, most of them on
  // levels too small to hide their launch latency
  auto cycle = [&]() -> hipError_t {
    hipError_t e;
    if ((e = mg_vcycle(P, 0, s)) || (e = mg_launch_sweep(F, s)) || (e = mg_launch_defect_norm(F, P.part, P.scal + 1, s)))
      return e;
    return hipSuccess;
  };
  int cyc = 0;
  while (cyc < max_cycles && !(d <= tol)) {
    auto it = c->mg_graphs.find(dev_work);
    if (it == c->mg_graphs.end()) {
      HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const hipError_t e = cycle();
      hipGraph_t g;
      const hipError_t e2 = hipStreamEndCapture(s, &g);
      if (e != hipSuccess) return hip_fail(c, e, "multigrid cycle capture");
      HIPCHK(c, e2);
      hipGraphExec_t ge;
      const hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      HIPCHK(c, e3);
      it = c->mg_graphs.emplace(dev_work, ge).first;
    }
    HIPCHK(c, hipGraphLaunch(it->second, s));
    HIPCHK(c, hipMemcpyAsync(&d, P.scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    ++cyc;
    if (host_defects) host_defects[cyc] = d;
  }
  HIPCHK(c, mg_launch_sum(F.phi, N, 0, invN, 0, P.part, P.scal + 2, s));
  HIPCHK(c, mg_launch_affine(F.phi, P.scal + 2, 0.0, N, s));
  HIPCHK(c, mg_launch_scatter(a.m, c->nb, c->nmax, F, c->phi, s));
  HIPCHK(c, hipStreamSynchronize(s));
  c->cfl_parts = false;  // the CFL's gravity term changed with the potential
  if (host_cycles) *host_cycles = cyc;
  return TDH_OK;
}

// ---------------------------------------------------------------------------
// restart remap, Galilean boost, frame acceleration (Sec. Domain remapping and
// frame conversion; Sec. Moving-frame dynamics and BH treatment)
// ---------------------------------------------------------------------------
extern "C" tdh_status tdh_remap(tdh_ctx *dst, tdh_ctx *src) {
  CHECK_CTX(dst);
  CHECK_CTX(src);
  tdh_status st;
  if ((st = ready(dst)) || (st = require_window_boundary(dst))) return st;
  if ((st = ready(src)) || (st = require_window_boundary(src))) return fail(dst, TDH_ESTATE, "source: %s", g_err.c_str());
  if (dst == src) return fail(dst, TDH_EINVAL, "source and target are the same context");
  if (dst->amr || src->amr) return fail(dst, TDH_EINVAL, "the remap needs single-level meshes");
  if (dst->nv != src->nv) return fail(dst, TDH_EINVAL, "source and target differ in dual energy (%d vs %d variables)",
                                      src->nv, dst->nv);
  // the target grid coincides with the source grid if the spacings are equal and
  // the origins a whole number of cells apart
  int coincident = 1, shift[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    const double sft = (dst->x0[d] - src->x0[d]) / src->dx[d];
    if (dst->dx[d] != src->dx[d] || sft != std::floor(sft) || std::fabs(sft) > 1e9) coincident = 0;
    else shift[d] = (int)sft;
  }
  HIPCHK(dst, hipStreamSynchronize(src->stream));
  const StageArgs sa = base_args(src), da = base_args(dst);
  HIPCHK(dst, launch_remap(sa.m, src->d_par, src->Qa, src->Qb, da.m, dst->Qa, da.p, src->t, dst->nv, coincident, shift,
                           dst->stream));
  if (dst->jc) HIPCHK(dst, hipMemsetAsync(dst->jc, 0xff, 3 * dst->ncells * sizeof(int), dst->stream));
  dst->seeds_held = false;
  dst->cfl_seeds = false;
  dst->cfl_parts = false;
  dst->par.assign(dst->nb, 0);
  HIPCHK(dst, hipMemcpyAsync(dst->d_par, dst->par.data(), dst->nb * sizeof(int), hipMemcpyHostToDevice, dst->stream));
  HIPCHK(dst, hipStreamSynchronize(dst->stream));
  dst->t = src->t;
  return TDH_OK;
}

extern "C" tdh_status tdh_galilean_boost(tdh_ctx *c, const double *host_V, double rho_skip) {
  CHECK_CTX(c);
  tdh_status st;
  if ((st = ready(c)) || (st = require_window_boundary(c))) return st;
  if (!host_V) return fail(c, TDH_EINVAL, "null velocity");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(host_V[d])) return fail(c, TDH_EINVAL, "velocity must be finite");
  const StageArgs a = base_args(c);
  HIPCHK(c, launch_boost(a.m, c->d_par, c->Qa, c->Qb, c->nv, host_V, rho_skip, c->stream));
  if (c->jc) HIPCHK(c, hipMemsetAsync(c->jc, 0xff, 3 * c->ncells * sizeof(int), c->stream));  // energies moved
  c->seeds_held = false;
  c->cfl_seeds = false;
  c->cfl_parts = false;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_frame_acceleration(tdh_ctx *c, double rho_min, double *host_A) {
  CHECK_CTX(c);
  tdh_status st;
  if ((st = ready(c)) || (st = require_window_boundary(c))) return st;
  if (!host_A) return fail(c, TDH_EINVAL, "null output");
  if (c->cfg.grav_kind != 2) return fail(c, TDH_ESTATE, "the frame acceleration needs the point mass (grav_kind 2)");
  if (c->amr) return fail(c, TDH_EINVAL, "the frame acceleration needs a single-level mesh");
  const StageArgs a = base_args(c);
  double *part = c->d_facc, *out = c->d_facc + 4 * frame_acceleration_parts();
  HIPCHK(c, launch_frame_acceleration(a.m, c->d_par, c->Qa, c->Qb, a.p, c->t, rho_min, part, out, c->stream));
  HIPCHK(c, hipMemcpyAsync(host_A, out, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_get_potential(tdh_ctx *c, double *host_phi) {
  CHECK_CTX(c);
  tdh_status st;
  if ((st = ready(c))) return st;
  if (!host_phi) return fail(c, TDH_EINVAL, "null output");
  if (!c->phi) return fail(c, TDH_ESTATE, "no stored potential (grav_kind is not 1)");
  HIPCHK(c, hipMemcpyAsync(host_phi, c->phi, c->ptotal * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_set_state(tdh_ctx *c, const double *host) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = ready(c)) || (s = require_window_boundary(c))) return s;
  if (!host) return fail(c, TDH_EINVAL, "null input");
  HIPCHK(c, hipMemcpyAsync(c->Qa, host, c->total * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (c->jc) HIPCHK(c, hipMemsetAsync(c->jc, 0xff, 3 * c->ncells * sizeof(int), c->stream));  // stale seeds go
  c->seeds_held = false;
  c->cfl_seeds = false;
  c->cfl_parts = false;
  c->par.assign(c->nb, 0);
  HIPCHK(c, hipMemcpyAsync(c->d_par, c->par.data(), c->nb * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_get_seed_cells(tdh_ctx *c, int32_t *host) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = ready(c))) return s;
  if (!host) return fail(c, TDH_EINVAL, "null output");
  if (!c->jc) return fail(c, TDH_ESTATE, "no seed cells without a table EOS");
  if (c->k != 0) return fail(c, TDH_ESTATE, "seed cells are only defined between windows");
  for (int b = 0; b < c->nb; ++b) {
    const long long n = c->blk[4 * b];
    const long long cell0 = c->binfo[b].off / c->nv;
    const int *src = c->jc + (size_t)c->par[b] * c->ncells + cell0;  // segment of the current buffer
    HIPCHK(c, hipMemcpyAsync(host + cell0, src, n * n * n * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_eos_invert_batch(tdh_ctx *c, const double *lr, const double *le, double *lT, int32_t *j,
                                           int32_t *iters, int64_t n, int mode) {
  CHECK_CTX(c);
  if (!c->have_table) return fail(c, TDH_ESTATE, "no EOS table");
  if (n < 0 || n > (1LL << 31)) return fail(c, TDH_ERANGE, "n out of range");
  if (mode < 0 || mode > 2) return fail(c, TDH_EINVAL, "mode must be 0, 1 or 2");
  if (mode == 1 && !c->have_mlp) return fail(c, TDH_ESTATE, "mode 1 needs the seed network (tdh_mlp_init)");
  if (!lr || !le) return fail(c, TDH_EINVAL, "null input");
  HIPCHK(c, launch_eos_invert(c->tab, c->seed, c->cfg.newton_max_iter, lr, le, lT, j, iters, n, mode, c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_eos_eval_batch(tdh_ctx *c, const double *rho, const double *U, double *P, double *cs,
                                         int64_t n) {
  CHECK_CTX(c);
  if (c->cfg.eos_kind == 1 && !c->have_table) return fail(c, TDH_ESTATE, "no EOS table");
  if (n < 0 || n > (1LL << 31)) return fail(c, TDH_ERANGE, "n out of range");
  if (!rho || !U || !P || !cs) return fail(c, TDH_EINVAL, "null argument");
  HIPCHK(c, launch_eos_eval(make_phys(c->cfg), c->tab, rho, U, P, cs, n, c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_get_stats(tdh_ctx *c, tdh_stats *out) {
  CHECK_CTX(c);
  if (!out) return fail(c, TDH_EINVAL, "null output");
  *out = c->stats;
  return TDH_OK;
}

static bool tile_fits(const tdh_ctx *c, int id) {
  int d[4];
  tile_shape(id, d);
  if (d[0] == 0) return d[1] > 0;  // the split form fits every mesh
  return d[0] > 0 && c->lat % d[0] == 0 && c->lat % d[1] == 0 && c->lat % d[2] == 0;
}

extern "C" int tdh_num_tiles(void) { return num_tiles(); }

extern "C" tdh_status tdh_tile_shape(int id, int *dims) {
  if (!dims || id < 0 || id >= num_tiles()) return fail(nullptr, TDH_EINVAL, "tile id out of range");
  int d[4];
  tile_shape(id, d);
  for (int i = 0; i < 4; ++i) dims[i] = d[i];
  return TDH_OK;
}

extern "C" tdh_status tdh_set_tile(tdh_ctx *c, int id) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = ready(c)) || (s = require_window_boundary(c))) return s;
  if (id < 0 || id >= num_tiles()) return fail(c, TDH_EINVAL, "tile id out of range");
  if (!tile_fits(c, id)) return fail(c, TDH_EINVAL, "tile %d does not divide the smallest block", id);
  if (id != c->tile) {
    for (auto &g : c->graphs) hipGraphExecDestroy(g.second);
    c->graphs.clear();
  }
  c->tile = id;
  return TDH_OK;
}

// Time one stage-1 launch over every block for each tile shape that fits and
// keep the fastest.  Stage 1 only writes the stage buffers, which the next
// sub-cycle overwrites, so the state is unchanged.
extern "C" tdh_status tdh_autotune(tdh_ctx *c, int reps, int *host_best, float *host_ms) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = ready(c)) || (s = require_window_boundary(c))) return s;
  if (reps < 1 || reps > 100) return fail(c, TDH_EINVAL, "reps must be in [1, 100]");
  const std::vector<int> saved = c->levels;
  const int saved_lmax = c->Lmax;
  if ((s = install_levels(c, std::vector<int>(c->nb, 0)))) return s;
  HIPCHK(c, launch_set_window(c->d_win, c->t, c->dt_coarse > 0.0 ? c->dt_coarse : 1e-30, c->stream));
  StageArgs a = base_args(c);
  // time the kernel the run's windows will use: with levels when LAT is configured
  a.lmax = std::max(saved_lmax, c->cfg.n_lat > 0 ? 1 : 0);
  a.cfl_part = nullptr;
  a.k = 0;
  a.phase = 1;
  a.Llo = 0;
  a.Lhi = kCntSlots - 2;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  int best = -1;
  float best_ms = 0.0f;
  for (int id = 0; id < num_tiles(); ++id) {
    float ms = -1.0f;
    if (tile_fits(c, id)) {
      HIPCHK(c, launch_stage(a, id, c->cus, c->stream));  // warm-up
      HIPCHK(c, hipEventRecord(e0, c->stream));
      for (int r = 0; r < reps; ++r) HIPCHK(c, launch_stage(a, id, c->cus, c->stream));
      HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipEventSynchronize(e1));
      HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
      ms /= reps;
      if (best < 0 || ms < best_ms) { best = id; best_ms = ms; }
    }
    if (host_ms) host_ms[id] = ms;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if ((s = install_levels(c, saved))) return s;
  if (best >= 0 && best != c->tile) {
    for (auto &g : c->graphs) hipGraphExecDestroy(g.second);
    c->graphs.clear();
    c->tile = best;
  }
  if (host_best) *host_best = c->tile;
  return TDH_OK;
}

extern "C" tdh_status tdh_get_tile(tdh_ctx *c, int *id) {
  CHECK_CTX(c);
  if (!id) return fail(c, TDH_EINVAL, "null output");
  *id = c->tile;
  return TDH_OK;
}

extern "C" tdh_status tdh_set_timing(tdh_ctx *c, int on) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = collect_timing(c))) return s;
  if (on && c->ev.empty()) {
    c->ev.resize(512);
    for (hipEvent_t &e : c->ev) HIPCHK(c, hipEventCreate(&e));
  }
  c->timing = on != 0;
  c->stage_ms = 0.0;
  c->stage_launches = 0;
  return TDH_OK;
}

extern "C" tdh_status tdh_get_stage_time(tdh_ctx *c, double *host_ms, int64_t *host_launches) {
  CHECK_CTX(c);
  tdh_status s;
  if ((s = collect_timing(c))) return s;
  if (host_ms) *host_ms = c->stage_ms;
  if (host_launches) *host_launches = c->stage_launches;
  return TDH_OK;
}

// ---------------------------------------------------------------------------
// learned EOS seed network
// ---------------------------------------------------------------------------

static void invalidate_graphs(tdh_ctx *c) {
  for (auto &g : c->graphs) hipGraphExecDestroy(g.second);
  c->graphs.clear();
}

extern "C" tdh_status tdh_mlp_init(tdh_ctx *c, const float *host_params, double lr_lo, double lr_hi, double le_lo,
                                   double le_hi, double lt_lo, double lt_hi) {
  CHECK_CTX(c);
  if (!host_params) return fail(c, TDH_EINVAL, "null parameters");
  if (!(lr_hi > lr_lo) || !(le_hi > le_lo) || !(lt_hi > lt_lo)) return fail(c, TDH_EINVAL, "empty normalisation range");
  if (!c->have_mesh) return fail(c, TDH_ESTATE, "no mesh: the network's buffers are in the arena (tdh_init_blocks)");
  if (!c->d_mw) return fail(c, TDH_ESTATE, "the learned seed serves the table EOS: a context with eos_kind 1");
  std::vector<float> zero(kMlpParams, 0.0f);
  HIPCHK(c, hipMemcpyAsync(c->d_mw, host_params, kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_mm, zero.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_mv, zero.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
  MlpDev &w = c->seed.w;
  w.b1 = c->d_mb;
  w.b2 = c->d_mb + 64;
  w.b3 = c->d_mb + 128;
  w.w1b = c->d_mwb;
  w.w2b = c->d_mwb + 128;
  w.w2tb = c->d_mwb + 128 + 4096;
  w.w3b = c->d_mwb + 128 + 8192;
  HIPCHK(c, mlp_launch_pack(c->d_mw, (short *)w.w1b, (short *)w.w2b, (short *)w.w2tb, (short *)w.w3b, (float *)w.b1,
                            (float *)w.b2, (float *)w.b3, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->seed.lr_lo = lr_lo; c->seed.lr_hi = lr_hi;
  c->seed.le_lo = le_lo; c->seed.le_hi = le_hi;
  c->seed.lt_lo = lt_lo; c->seed.lt_hi = lt_hi;
  c->seed.enabled = 0;
  c->have_mlp = true;
  c->mlp_steps_done = 0;
  invalidate_graphs(c);
  return TDH_OK;
}

extern "C" tdh_status tdh_mlp_train(tdh_ctx *c, const double *dev_in, const double *dev_lT, int64_t n, int steps,
                                    int batch, float lr, uint64_t seed, float *host_loss) {
  CHECK_CTX(c);
  if (!c->have_mlp) return fail(c, TDH_ESTATE, "call tdh_mlp_init first");
  if (!dev_in || !dev_lT || n < 64) return fail(c, TDH_EINVAL, "need at least 64 samples");
  if (batch < 64 || batch % 64 || batch > kMlpMaxBatch) return fail(c, TDH_EINVAL, "batch must be a multiple of 64 up to 65536");
  if (steps < 1 || steps > kMlpMaxSteps) return fail(c, TDH_ERANGE, "steps must be in [1, 2^20]");
  if (!(lr > 0.0f)) return fail(c, TDH_EINVAL, "lr must be positive");
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  MlpDev &w = c->seed.w;
  for (int st = 0; st < steps; ++st) {
    const int t = ++c->mlp_steps_done;
    const float lr_t = (float)(0.5 * lr * (1.0 + std::cos(M_PI * st / (double)steps)));  // cosine decay
    HIPCHK(c, mlp_launch_fwd_bwd(w, c->seed, dev_in, dev_lT, n, batch, seed, t, 1, c->d_mpart, c->d_mloss_part,
                                 c->d_mgrad, c->d_mloss + st, c->stream));
    const float c1 = (float)(1.0 - std::pow((double)b1, t)), c2 = (float)(1.0 - std::pow((double)b2, t));
    HIPCHK(c, mlp_launch_adam(c->d_mw, c->d_mm, c->d_mv, c->d_mgrad, lr_t, b1, b2, eps, c1, c2, c->stream));
    HIPCHK(c, mlp_launch_pack(c->d_mw, (short *)w.w1b, (short *)w.w2b, (short *)w.w2tb, (short *)w.w3b, (float *)w.b1,
                              (float *)w.b2, (float *)w.b3, c->stream));
  }
  if (host_loss)
    HIPCHK(c, hipMemcpyAsync(host_loss, c->d_mloss, steps * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  invalidate_graphs(c);
  return TDH_OK;
}

extern "C" tdh_status tdh_mlp_adam_step(tdh_ctx *c, const float *host_grad, float lr) {
  CHECK_CTX(c);
  if (!c->have_mlp) return fail(c, TDH_ESTATE, "call tdh_mlp_init first");
  if (!host_grad) return fail(c, TDH_EINVAL, "null gradient");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(c, TDH_EINVAL, "lr must be positive and finite");
  if (c->mlp_steps_done >= kMlpMaxSteps) return fail(c, TDH_ERANGE, "more than 2^20 Adam steps");
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  HIPCHK(c, hipMemcpyAsync(c->d_mgrad, host_grad, kMlpParams * sizeof(float), hipMemcpyHostToDevice, c->stream));
  const int t = ++c->mlp_steps_done;
  const float c1 = (float)(1.0 - std::pow((double)b1, t)), c2 = (float)(1.0 - std::pow((double)b2, t));
  HIPCHK(c, mlp_launch_adam(c->d_mw, c->d_mm, c->d_mv, c->d_mgrad, lr, b1, b2, eps, c1, c2, c->stream));
  MlpDev &w = c->seed.w;
  HIPCHK(c, mlp_launch_pack(c->d_mw, (short *)w.w1b, (short *)w.w2b, (short *)w.w2tb, (short *)w.w3b, (float *)w.b1,
                            (float *)w.b2, (float *)w.b3, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  invalidate_graphs(c);
  return TDH_OK;
}

extern "C" tdh_status tdh_mlp_loss_grad(tdh_ctx *c, const double *dev_in, const double *dev_lT, int64_t n,
                                        float *host_loss, float *host_grad) {
  CHECK_CTX(c);
  if (!c->have_mlp) return fail(c, TDH_ESTATE, "call tdh_mlp_init first");
  if (!dev_in || !dev_lT || n < 64 || n % 64 || n > kMlpMaxBatch)
    return fail(c, TDH_EINVAL, "n must be a multiple of 64 up to 65536");
  HIPCHK(c, mlp_launch_fwd_bwd(c->seed.w, c->seed, dev_in, dev_lT, n, (int)n, 0, 0, 0, c->d_mpart, c->d_mloss_part,
                               c->d_mgrad, c->d_mloss, c->stream));
  if (host_grad)
    HIPCHK(c, hipMemcpyAsync(host_grad, c->d_mgrad, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  if (host_loss) HIPCHK(c, hipMemcpyAsync(host_loss, c->d_mloss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_mlp_forward(tdh_ctx *c, const double *dev_in, double *dev_lT, int64_t n) {
  CHECK_CTX(c);
  if (!c->have_mlp) return fail(c, TDH_ESTATE, "call tdh_mlp_init first");
  if (!dev_in || !dev_lT || n < 0 || n > (1LL << 31)) return fail(c, TDH_EINVAL, "bad arguments");
  HIPCHK(c, mlp_launch_forward(c->seed.w, c->seed, dev_in, dev_lT, n, c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_mlp_get_params(tdh_ctx *c, float *host_params) {
  CHECK_CTX(c);
  if (!c->have_mlp) return fail(c, TDH_ESTATE, "call tdh_mlp_init first");
  if (!host_params) return fail(c, TDH_EINVAL, "null output");
  HIPCHK(c, hipMemcpyAsync(host_params, c->d_mw, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return TDH_OK;
}

extern "C" tdh_status tdh_mlp_enable_seed(tdh_ctx *c, int on) {
  CHECK_CTX(c);
  if (on && !c->have_mlp) return fail(c, TDH_ESTATE, "call tdh_mlp_init first");
  c->seed.enabled = on ? 1 : 0;
  invalidate_graphs(c);
  return TDH_OK;
}
