// C-ABI of libetdfb: context management, argument checks and the sequence
// of launches behind each entry point declared in include/etdfb.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/etdfb.h"
#include "etdfb_internal.h"
#include "launch.h"
#include "levelset.h"

using namespace etdfb;

constexpr int NCOUNTERS = 96;   // device counters of a context (see etd_ctx::counters)

struct etd_ctx {
  int device = 0;
  // components of u (eq. 3.1 with u in R^m) and their Lotka-Volterra reaction
  int species = 1;
  double sp_a[MAX_SPECIES] = {};
  double sp_b[MAX_SPECIES * MAX_SPECIES] = {};
  hipStream_t stream = nullptr;
  etd_grid grid{};
  etd_physics phys{};
  etd_krylov_opts opts{};
  BoxHost box{};
  int ntiles = 0;         // tiles of the box
  size_t nodes = 0;       // nodes of the box
  size_t ld = 0;          // doubles per workspace vector
  // geometry
  uint8_t* mask = nullptr;
  int* tile_flag = nullptr;
  int* tile_map = nullptr;
  int* slot_tile = nullptr;
  uint64_t* comp_bits = nullptr;
  uint64_t* irr_bits = nullptr;
  double* cdiag = nullptr;
  int* nbr = nullptr;        // face-neighbour slots, NBR_STRIDE per slot
  int* tile_vb = nullptr;    // tiles with a node |rho| < h
  int* band_tmp = nullptr;   // 2 * ntiles: tile distance passes
  int* band_list = nullptr;  // level-set tile lists SC, SV, U, LS_NLISTS * ntiles
  int* counters = nullptr;   // [0] n_active, [1] status, [2..3] case counts, [4] unknowns,
                             // [LS_CNT_C..LS_NCOUNTERS) level-set list counts
  // persistent kernel state
  double* ws = nullptr;
  double* part = nullptr;
  unsigned* flags = nullptr;
  BarrierDev* bar = nullptr;
  int n_cu = 0;
  double clock_khz = 1.0;   // device wall clock (ticks per millisecond)
  int tmax = 1;
  KrylovStateDev* st = nullptr;
  int max_grid = 0;                 // co-resident blocks, the larger of the two builds (array sizes)
  int max_grid_kb[2] = {0, 0};      // co-resident blocks of each Krylov build (KrylovBuild)
  int kb_fixed = -1;                // a build this context always uses (-1: chosen per geometry)
  int kb = KB_LARGE;                // the build of the next Krylov launch
  int grid_blocks = 1;
  int n_active_host = 0;
  bool have_geometry = false;
  // level-set scratch (box arrays) and its one-instance table
  LevelsetScratch ls{};
  LevelsetBatch lsb{};
  int ncum_c[LS_C_MAX + 1] = {};   // level-set list counts of the last build
  int ncum_v[LS_V_MAX + 1] = {};
  int nu_host = 0;
  // geometry-build table of this context (one instance)
  GeomBatch gb{};
  // variable beta and Dirichlet data (etd_geometry_build_var; allocated on
  // its first call): face coefficients and diagonal, boundary taps and their
  // compact numbering
  bool var_mode = false;
  double* vcoef = nullptr;
  int* tap_n = nullptr;
  double* tap_coef = nullptr;
  double* tap_pt = nullptr;
  int* tap_off = nullptr;
  int ntaps = 0;
  std::vector<double> h_tap_pts;   // compact tap points, dim per tap
  // pinned host mirror for small readbacks
  int* h_counters = nullptr;
  KrylovStateDev* h_state = nullptr;
  // event timing
  bool profiling = false;
  struct Timer {
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
    double ms = 0.0;
    int count = 0;
  } t_krylov, t_levelset, t_geometry;
};

struct etd_batch {
  int count = 0;
  int dim = 2;
  hipStream_t stream = nullptr;
  std::vector<etd_ctx*> inst;
  int capacity = 1;           // co-resident blocks of the batched launch
  int group_limit = 0;        // max blocks per instance (0: no limit)
  int nchunks = 1;            // launches per step (instances per launch <= capacity)
  KrylovDev* d_params = nullptr;
  KrylovDev* h_params = nullptr;
  LevelsetBatch lsb{};        // level-set table of all instances
  GeomBatch gb{};             // geometry table of all instances
  const double** h_uptr = nullptr;   // user box arrays of the current step (pinned), 2 count:
  const double** d_uptr = nullptr;   // u, then F(U_{n-1}) of a multistep step
  int ms_first = 0;                  // KrylovDev::first of the multistep step being scheduled
  hipEvent_t uptr_done = nullptr;    // the last upload of h_uptr has been read
  bool uptr_pending = false;
  long geom_gen = 0;                 // geometry builds so far
  // recorded frozen-domain step (etd_batch_graph_steps) and its key
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;  // capture stream (default priority)
  int g_scheme = 0;
  double g_h = 0.0;
  long g_geom = -1;
  int g_limit = -1;
  int g_stage = -2;
  std::vector<double*> g_u;
  KrylovDev* d_gparams = nullptr;    // graph-owned parameter copies
  int* d_gblk = nullptr;
  const double** d_guptr = nullptr;
  // recorded free-boundary step (etd_batch_graph_free_steps): without and
  // with the reinitialisation, each with level-set and geometry tables,
  // parameters and pointers of its own (an eager call rewrites the shared
  // ones), and the key
  hipGraph_t fgraph[2] = {nullptr, nullptr};
  hipGraphExec_t fgexec[2] = {nullptr, nullptr};
  LevelsetBatch flsb{};
  GeomBatch fgb{};
  bool f_alloc = false;
  int f_scheme = 0;
  double f_h = 0.0;
  int f_limit = -1;
  int f_stage = -2;
  std::vector<double*> f_u, f_rho;
  KrylovDev* d_fparams = nullptr;
  int* d_fblk = nullptr;
  const double** d_fuptr = nullptr;
  // replayed free-boundary steps moved the boundaries on the device: the
  // host's list sizes and active-tile counts are re-read before an eager call
  bool host_stale = false;
  int stage_min = -1;         // LDS-staged Lanczos pass from this many active tiles (-1: default)
  int* d_blk = nullptr;       // block -> instance, capacity entries per chunk
  int* h_blk = nullptr;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  bool profiling = false;
  etd_ctx::Timer t_krylov, t_levelset, t_geometry;
};

namespace {

hipError_t timer_begin(bool on, hipStream_t st, etd_ctx::Timer& t) {
  if (!on) return hipSuccess;
  if (t.used == t.start.size()) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    t.start.push_back(a);
    t.stop.push_back(b);
  }
  return hipEventRecord(t.start[t.used], st);
}

hipError_t timer_end(bool on, hipStream_t st, etd_ctx::Timer& t) {
  if (!on) return hipSuccess;
  hipError_t e = hipEventRecord(t.stop[t.used], st);
  ++t.used;
  return e;
}

// fold recorded pairs into ms (stream must be synchronised)
hipError_t timer_collect(etd_ctx::Timer& t) {
  for (size_t i = 0; i < t.used; ++i) {
    float ms = 0.0f;
    hipError_t e = hipEventElapsedTime(&ms, t.start[i], t.stop[i]);
    if (e != hipSuccess) return e;
    t.ms += ms;
    ++t.count;
  }
  t.used = 0;
  return hipSuccess;
}

void timer_free(etd_ctx::Timer& t) {
  for (auto e : t.start) (void)hipEventDestroy(e);
  for (auto e : t.stop) (void)hipEventDestroy(e);
  t.start.clear();
  t.stop.clear();
}

int check_hip(hipError_t e) { return e == hipSuccess ? ETD_OK : ETD_ERR_HIP; }

// Persistent-kernel job of an ETD scheme (valid schemes only).
int job_of(int scheme) {
  switch (scheme) {
    case ETD_SCHEME_ETD1: return JOB_ETD1;
    case ETD_SCHEME_ETD3RK: return JOB_ETD3RK;
    case ETD_SCHEME_ETD4RK: return JOB_ETD4RK;
    case ETD_SCHEME_ETD3RK_SIMUL: return JOB_ETD3RK_SIMUL;
    case ETD_SCHEME_ETD4RK_SIMUL: return JOB_ETD4RK_SIMUL;
    default: return JOB_ETD2RK;
  }
}

// Zero the accumulated measurement fields of a device state (stream-ordered;
// the source is a static host block, so it outlives the copy).
hipError_t reset_counters(KrylovStateDev* st, hipStream_t s) {
  static const KrylovStateDev zero{};
  const size_t off = offsetof(KrylovStateDev, alg_bytes_total);
  return hipMemcpyAsync((char*)st + off, (const char*)&zero + off, sizeof(KrylovStateDev) - off,
                        hipMemcpyHostToDevice, s);
}

#define HIP_TRY(x)                         \
  do {                                     \
    hipError_t _e = (x);                   \
    if (_e != hipSuccess) return ETD_ERR_HIP; \
  } while (0)


GeomDev geom_view(const etd_ctx* c) {
  GeomDev g{};
  g.dim = c->box.dim;
  g.nx = c->box.nx; g.ny = c->box.ny; g.nz = c->box.nz;
  g.ntx = c->box.ntx; g.nty = c->box.nty; g.ntz = c->box.ntz;
  g.tile_map = c->tile_map;
  g.slot_tile = c->slot_tile;
  g.comp_bits = c->comp_bits;
  g.irr_bits = c->irr_bits;
  g.cdiag = c->cdiag;
  g.nbr = c->nbr;
  g.n_active = c->counters + (c->species > 1 ? 5 : 0);
  g.n_unknowns = c->counters + (c->species > 1 ? 6 : 4);
  g.coef = c->phys.beta / (c->box.dx * c->box.dx);
  g.dx = c->box.dx;
  g.vcoef = c->var_mode ? c->vcoef : nullptr;
  g.vld = c->ld;
  return g;
}

KrylovDev krylov_params(const etd_ctx* c, int mode, int sync_master_min = SYNC_MASTER_MIN_BLOCKS) {
  KrylovDev P{};
  P.g = geom_view(c);
  P.ws = c->ws;
  P.ld = c->ld;
  P.part = c->part;
  P.flags = c->flags;
  P.bar = c->bar;
  P.tmax = c->tmax;
  P.status = c->counters + 1;
  P.st = c->st;
  P.tol = c->opts.tol;
  P.m_min = c->opts.m_min;
  P.m_max = c->opts.m_max;
  P.m_step = c->opts.m_step;
  P.max_substeps = c->opts.max_substeps;
  P.ra = c->phys.a;
  P.rb = c->phys.b;
  P.mode = mode;
  P.species = c->species;
  for (int s = 0; s < MAX_SPECIES; ++s) P.sa[s] = c->sp_a[s];
  for (int s = 0; s < MAX_SPECIES * MAX_SPECIES; ++s) P.sb[s] = c->sp_b[s];
  // ETDFB_STAGE_MIN in the environment overrides the size from which the
  // LDS-staged Lanczos pass is used (tests take it down to small problems)
  P.stage_min = STAGE_MIN_TILES;
  if (const char* env = getenv("ETDFB_STAGE_MIN")) P.stage_min = atoi(env);
  // ETDFB_SYNC_MASTER overrides the block count from which block 0 alone
  // reduces at a grid synchronisation (tests force either form)
  P.sync_master_min = sync_master_min;
  if (const char* env = getenv("ETDFB_SYNC_MASTER")) P.sync_master_min = atoi(env);
  return P;
}

// Grid of the persistent kernel: enough blocks for one loop trip over the
// active tiles (KB_TILES tiles per block and trip), at most the number of
// co-resident blocks.  ETDFB_GRID in the environment overrides the count.
void choose_launch(etd_ctx* c) {
  const int nact = c->n_active_host > 0 ? c->n_active_host * c->species : 1;
  // 512-thread blocks when every active tile fits one loop trip of them
  // (more blocks on more CUs, twice the registers per thread), else 1024;
  // ETDFB_KBLOCK (512 or 1024) in the environment forces a build
  int kb = (nact <= KB_TILES[KB_SMALL] * c->max_grid_kb[KB_SMALL]) ? KB_SMALL : KB_LARGE;
  if (const char* env = getenv("ETDFB_KBLOCK")) {
    const int v = atoi(env);
    if (v == KB_THREADS[KB_SMALL]) kb = KB_SMALL;
    if (v == KB_THREADS[KB_LARGE]) kb = KB_LARGE;
  }
  if (c->kb_fixed >= 0) kb = c->kb_fixed;
  int g = (nact + KB_TILES[kb] - 1) / KB_TILES[kb];
  if (g > c->max_grid_kb[kb]) g = c->max_grid_kb[kb];
  if (const char* env = getenv("ETDFB_GRID")) {
    const int v = atoi(env);
    if (v >= 1 && v <= c->max_grid_kb[kb]) g = v;
  }
  c->kb = kb;
  c->grid_blocks = g < 1 ? 1 : g;
  c->tmax = 1;
}

int run_krylov(etd_ctx* c, const KrylovDev& P) {
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  if (timer_begin(c->profiling, c->stream, c->t_krylov) != hipSuccess) return ETD_ERR_HIP;
  hipError_t e = launch_krylov(c->kb, c->box.dim, P, c->grid_blocks, c->stream);
  if (e != hipSuccess) return ETD_ERR_HIP;
  return check_hip(timer_end(c->profiling, c->stream, c->t_krylov));
}

int gather_to(etd_ctx* c, const double* box, int vec) {
  int grid = c->n_active_host > 0 ? c->n_active_host : 1;
  return check_hip(launch_gather(c->box, box, c->slot_tile, c->comp_bits, c->counters + 0,
                                 c->ws + (size_t)vec * c->ld, grid, c->stream));
}

// tiles: box is already 0 at every node outside the active tiles (u after
// a level-set step: the restriction wrote it over the whole box), so only
// the active tiles are written.
int scatter_from(etd_ctx* c, int vec, double* box, bool tiles = false) {
  if (tiles) {
    const int grid = c->n_active_host > 0 ? c->n_active_host : 1;
    return check_hip(launch_scatter_tiles(c->box, c->ws + (size_t)vec * c->ld, c->slot_tile, c->comp_bits,
                                          c->counters + 0, box, grid, c->stream));
  }
  return check_hip(launch_scatter(c->box, c->ws + (size_t)vec * c->ld, c->tile_map, c->comp_bits, box,
                                  c->stream));
}

int fill_stats(etd_ctx* c, etd_stats* s) {
  HIP_TRY(hipMemcpyAsync(c->h_counters, c->counters, NCOUNTERS * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(c->h_state, c->st, sizeof(KrylovStateDev), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  s->substeps = c->h_state->substeps;
  s->rejected = c->h_state->rejected;
  s->matvecs = c->h_state->matvecs;
  s->m_last = c->h_state->m_last;
  s->expms = c->h_state->expms;
  // the unknowns of the (stacked) system: m copies of the tiles and points
  s->n_active_tiles = c->h_counters[c->species > 1 ? 5 : 0];
  s->n_unknowns = c->h_counters[c->species > 1 ? 6 : 4];
  s->status = c->h_counters[1];
  s->err_est = c->h_state->err_est;
  s->t_done = c->h_state->t_done;
  return ETD_OK;
}

int latched_status(etd_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->h_counters, c->counters, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  int st = c->h_counters[1];
  if (st != 0) {
    int zero = 0;
    HIP_TRY(hipMemcpyAsync(c->counters + 1, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return st;
}

// Geometry build (Section 2): classification, tile compaction, Case 1-3
// coefficients and the face-neighbour table, then an asynchronous copy of
// the counters to pinned memory.  geometry_finish() reads them after the
// caller has synchronised the stream.
const int GEOM_RADII[5] = {LS_C_MAX, LS_V_MAX, LS_CNT_C, LS_CNT_V, LS_CNT_U};
static_assert(LS_NCOUNTERS <= NCOUNTERS, "the level-set list counts must fit the counters");

// One entry of a geometry table: the context's arrays.
GeomInst geom_inst(const etd_ctx* c) {
  GeomInst I{};
  I.b = c->box;
  I.mask = c->mask;
  I.tile_flag = c->tile_flag;
  I.tile_vb = c->tile_vb;
  I.tile_map = c->tile_map;
  I.slot_tile = c->slot_tile;
  I.comp_bits = c->comp_bits;
  I.irr_bits = c->irr_bits;
  I.cdiag = c->cdiag;
  I.nbr = c->nbr;
  I.band_tmp = c->band_tmp;
  I.band_list = c->band_list;
  I.counters = c->counters;
  I.ws = c->ws;
  I.ld = c->ld;
  I.nodes = c->nodes;
  I.ntiles = c->ntiles;
  return I;
}

int geometry_enqueue(etd_ctx* c, const double* rho) {
  HIP_TRY(timer_begin(c->profiling, c->stream, c->t_geometry));
  c->gb.h_tab[0].rho = rho;
  HIP_TRY(launch_geometry(c->gb, GEOM_RADII, c->stream));
  if (c->species > 1) HIP_TRY(launch_replicate_species(c->gb, c->species, c->stream));
  HIP_TRY(timer_end(c->profiling, c->stream, c->t_geometry));
  return ETD_OK;
}

// After the build and a stream synchronisation: cnt holds the context's
// NCOUNTERS counters.
int geometry_finish(etd_ctx* c, const int* cnt) {
  memcpy(c->h_counters, cnt, sizeof(int) * NCOUNTERS);
  c->n_active_host = c->h_counters[0];
  for (int q = 0; q <= LS_C_MAX; ++q) c->ncum_c[q] = c->h_counters[LS_CNT_C + q];
  for (int q = 0; q <= LS_V_MAX; ++q) c->ncum_v[q] = c->h_counters[LS_CNT_V + q];
  c->nu_host = c->h_counters[LS_CNT_U];
  choose_launch(c);
  c->have_geometry = true;
  if (c->h_counters[1] == ST_DOMAIN) {
    int zero = 0;
    HIP_TRY(hipMemcpyAsync(c->counters + 1, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return ETD_ERR_DOMAIN;
  }
  return ETD_OK;
}

// The level-set view of a context (its scratch, band and the user arrays).
LsInst levelset_inst(etd_ctx* c, double* rho, double* u, double* f = nullptr) {
  LsInst I{};
  I.dim = c->box.dim;
  I.nx = c->box.nx; I.ny = c->box.ny; I.nz = c->box.nz;
  I.ntx = c->box.ntx; I.nty = c->box.nty; I.ntz = c->box.ntz;
  for (int q = 0; q <= LS_C_MAX; ++q) I.ncum_c[q] = c->ncum_c[q];
  for (int q = 0; q <= LS_V_MAX; ++q) I.ncum_v[q] = c->ncum_v[q];
  I.nu = c->nu_host;
  I.h = c->box.dx;
  I.mu = c->phys.mu;
  I.rho = rho;
  I.u = u;
  I.f = f;
  I.buf = c->ls.buf;
  I.nodes = c->ls.nodes;
  I.known = c->ls.known;
  I.dist = c->ls.dist;
  I.band = c->band_list;
  I.tdist = c->band_tmp + (size_t)((c->box.dim - 1) & 1) * c->ntiles;
  I.rr = LS_V_MAX;
  I.status = c->counters + 1;
  I.cnt = c->counters;
  I.host_dirty = &c->ls.dirty;
  return I;
}

// After levelset_begin and a synchronisation: some instance's maximum
// extended speed would move its front more than LS_MAX_FRONT_NODES nodes
// over dt (the extrapolation's reach; nothing has been changed yet).
bool front_too_fast(const LevelsetBatch& b) {
  for (int i = 0; i < b.count; ++i)
    if (!(b.h_vmax[i] * b.dt <= LS_MAX_FRONT_NODES * b.h_inst[i].h)) return true;
  return false;
}

void free_all(etd_ctx* c) {
  void* ptrs[] = {c->mask, c->tile_flag, c->tile_map, c->slot_tile, c->comp_bits, c->irr_bits, c->cdiag,
                  c->nbr, c->tile_vb, c->band_tmp, c->band_list, c->counters, c->ws, c->part, c->flags, c->bar, c->st,
                  c->vcoef, c->tap_n, c->tap_coef, c->tap_pt, c->tap_off};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  levelset_free(c->ls);
  levelset_batch_free(c->lsb);
  geom_batch_free(c->gb);
  timer_free(c->t_krylov);
  timer_free(c->t_levelset);
  timer_free(c->t_geometry);
  if (c->h_counters) (void)hipHostFree(c->h_counters);
  if (c->h_state) (void)hipHostFree(c->h_state);
}

}  // namespace

extern "C" {

const char* etd_status_string(int s) {
  switch (s) {
    case ETD_OK: return "ok";
    case ETD_ERR_INVALID: return "invalid argument";
    case ETD_ERR_HIP: return "HIP runtime error";
    case ETD_ERR_NO_DEVICE: return "no gfx950 device";
    case ETD_ERR_KRYLOV: return "Krylov method did not reach the tolerance";
    case ETD_ERR_NONFINITE: return "non-finite value in a reduction";
    case ETD_ERR_DOMAIN: return "computational point within 2 layers of the box edge";
    case ETD_ERR_BARRIER: return "grid barrier timed out";
    case ETD_ERR_NO_GEOMETRY: return "no geometry built";
    case ETD_ERR_FRONT: return "boundary moved beyond the reach of the level-set sweeps";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {

// Context creation for `species` components (1: the scalar problem).
int ctx_create(const etd_grid* grid, const etd_physics* phys, const etd_krylov_opts* opts, void* hip_stream,
               const etd_species* sp, etd_ctx** out) {
  if (!grid || !phys || !out) return ETD_ERR_INVALID;
  *out = nullptr;
  if (grid->dim != 2 && grid->dim != 3) return ETD_ERR_INVALID;
  for (int d = 0; d < grid->dim; ++d) {
    if (grid->n[d] < 5) return ETD_ERR_INVALID;
    if (!(grid->hi[d] > grid->lo[d])) return ETD_ERR_INVALID;
  }
  const double dx = (grid->hi[0] - grid->lo[0]) / (grid->n[0] - 1);
  for (int d = 1; d < grid->dim; ++d) {
    const double dd = (grid->hi[d] - grid->lo[d]) / (grid->n[d] - 1);
    if (fabs(dd - dx) > 1e-12 * dx) return ETD_ERR_INVALID;
  }
  if (!(phys->beta > 0.0) || !isfinite(phys->a) || !isfinite(phys->b) || !(phys->mu >= 0.0))
    return ETD_ERR_INVALID;
  etd_krylov_opts o{1e-10, 8, 64, 4, 64};
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.m_min < 1 || o.m_max > MMAX_LIMIT || o.m_min > o.m_max || o.m_step < 1 ||
      o.max_substeps < 1)
    return ETD_ERR_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return ETD_ERR_NO_DEVICE;
  etd_ctx* c = new etd_ctx();
  if (sp) {
    c->species = sp->m;
    for (int s = 0; s < sp->m; ++s) {
      c->sp_a[s] = sp->a[s];
      for (int j = 0; j < sp->m; ++j) c->sp_b[s * MAX_SPECIES + j] = sp->b[s * ETD_MAX_SPECIES + j];
    }
  }
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return ETD_ERR_NO_DEVICE; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) { delete c; return ETD_ERR_HIP; }
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) { delete c; return ETD_ERR_NO_DEVICE; }
  c->stream = (hipStream_t)hip_stream;
  c->grid = *grid;
  c->phys = *phys;
  c->opts = o;
  BoxHost& b = c->box;
  b.dim = grid->dim;
  b.nx = grid->n[0];
  b.ny = grid->n[1];
  b.nz = grid->dim == 3 ? grid->n[2] : 1;
  if (b.dim == 2) { b.tx = 32; b.ty = 8; b.tz = 1; } else { b.tx = 16; b.ty = 4; b.tz = 4; }
  b.ntx = (b.nx + b.tx - 1) / b.tx;
  b.nty = (b.ny + b.ty - 1) / b.ty;
  b.ntz = (b.nz + b.tz - 1) / b.tz;
  for (int d = 0; d < 3; ++d) b.lo[d] = d < grid->dim ? grid->lo[d] : 0.0;
  b.dx = dx;
  c->ntiles = b.ntx * b.nty * b.ntz;
  c->nodes = (size_t)b.nx * b.ny * b.nz;
  // every species has its copy of the active tiles in the vectors
  const size_t ktiles = (size_t)c->ntiles * c->species;
  c->ld = ktiles * TILE_PTS;
  c->n_cu = prop.multiProcessorCount;
  {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && khz > 0)
      c->clock_khz = khz;
  }
  for (int k = 0; k < 2; ++k)
    c->max_grid_kb[k] = krylov_max_blocks_per_cu(k, b.dim) * prop.multiProcessorCount;
  c->max_grid = c->max_grid_kb[0] > c->max_grid_kb[1] ? c->max_grid_kb[0] : c->max_grid_kb[1];
  if (c->max_grid_kb[KB_LARGE] < 1 || c->max_grid_kb[KB_SMALL] < 1) { delete c; return ETD_ERR_HIP; }
  bool ok = true;
  ok &= hipMalloc(&c->mask, c->nodes) == hipSuccess;
  ok &= hipMalloc(&c->tile_flag, sizeof(int) * c->ntiles) == hipSuccess;
  ok &= hipMalloc(&c->tile_map, sizeof(int) * c->ntiles) == hipSuccess;
  ok &= hipMalloc(&c->slot_tile, sizeof(int) * ktiles) == hipSuccess;
  ok &= hipMalloc(&c->comp_bits, sizeof(uint64_t) * 4 * ktiles) == hipSuccess;
  ok &= hipMalloc(&c->irr_bits, sizeof(uint64_t) * 4 * ktiles) == hipSuccess;
  ok &= hipMalloc(&c->cdiag, sizeof(double) * c->ld) == hipSuccess;
  ok &= hipMalloc(&c->nbr, sizeof(int) * NBR_STRIDE * ktiles) == hipSuccess;
  ok &= hipMalloc(&c->tile_vb, sizeof(int) * (size_t)c->ntiles) == hipSuccess;
  ok &= hipMalloc(&c->band_tmp, sizeof(int) * 2 * (size_t)c->ntiles) == hipSuccess;
  ok &= hipMalloc(&c->band_list, sizeof(int) * LS_NLISTS * (size_t)c->ntiles) == hipSuccess;
  ok &= hipMalloc(&c->counters, sizeof(int) * NCOUNTERS) == hipSuccess;
  ok &= hipMalloc(&c->ws, sizeof(double) * c->ld * NVEC) == hipSuccess;
  ok &= hipMalloc(&c->part, sizeof(double) * 2 * (size_t)c->max_grid * PART_STRIDE) == hipSuccess;
  ok &= hipMalloc(&c->flags, sizeof(unsigned) * (size_t)c->max_grid) == hipSuccess;
  ok &= hipMalloc(&c->bar, sizeof(BarrierDev)) == hipSuccess;
  ok &= hipMalloc(&c->st, sizeof(KrylovStateDev)) == hipSuccess;
  ok &= hipHostMalloc(&c->h_counters, sizeof(int) * NCOUNTERS) == hipSuccess;
  ok &= hipHostMalloc(&c->h_state, sizeof(KrylovStateDev)) == hipSuccess;
  ok &= levelset_alloc(c->ls, c->nodes) == hipSuccess;
  ok &= levelset_batch_alloc(c->lsb, 1, b.dim) == hipSuccess;
  ok &= geom_batch_alloc(c->gb, 1, NCOUNTERS) == hipSuccess;
  if (!ok) {
    free_all(c);
    delete c;
    return ETD_ERR_HIP;
  }
  KrylovStateDev s0{};
  for (int k = 0; k <= PMAX; ++k) {
    s0.m_guess[k] = o.m_min;
    s0.tau_frac[k] = 1.0;
  }
  int zeros[NCOUNTERS] = {};
  ok &= hipMemcpy(c->st, &s0, sizeof(s0), hipMemcpyHostToDevice) == hipSuccess;
  ok &= hipMemcpy(c->counters, zeros, sizeof(zeros), hipMemcpyHostToDevice) == hipSuccess;
  ok &= hipMemset(c->ws, 0, sizeof(double) * c->ld * NVEC) == hipSuccess;
  ok &= hipMemset(c->bar, 0, sizeof(BarrierDev)) == hipSuccess;
  if (ok) {
    c->gb.h_tab[0] = geom_inst(c);
    ok &= geom_batch_prefix(c->gb) == hipSuccess;
  }
  ok &= hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    free_all(c);
    delete c;
    return ETD_ERR_HIP;
  }
  *out = c;
  return ETD_OK;
}

}  // namespace

extern "C" {

int etd_ctx_create(const etd_grid* grid, const etd_physics* phys, const etd_krylov_opts* opts,
                   void* hip_stream, etd_ctx** out) {
  return ctx_create(grid, phys, opts, hip_stream, nullptr, out);
}

int etd_ctx_create_species(const etd_grid* grid, const etd_physics* phys, const etd_species* sp,
                           const etd_krylov_opts* opts, void* hip_stream, etd_ctx** out) {
  if (out) *out = nullptr;
  if (!sp || sp->m < 1 || sp->m > ETD_MAX_SPECIES) return ETD_ERR_INVALID;
  for (int s = 0; s < sp->m; ++s) {
    if (!isfinite(sp->a[s])) return ETD_ERR_INVALID;
    for (int j = 0; j < sp->m; ++j)
      if (!isfinite(sp->b[s * ETD_MAX_SPECIES + j])) return ETD_ERR_INVALID;
  }
  return ctx_create(grid, phys, opts, hip_stream, sp, out);
}

int etd_step_species(etd_ctx* c, int32_t scheme, double h, double* const* u, etd_stats* stats) {
  if (!c || !u || !(h >= 0.0) || !isfinite(h)) return ETD_ERR_INVALID;
  if (scheme < ETD_SCHEME_ETD1 || scheme > ETD_SCHEME_ETD4RK_SIMUL) return ETD_ERR_INVALID;
  for (int s = 0; s < c->species; ++s) {
    if (!u[s]) return ETD_ERR_INVALID;
    for (int j = 0; j < s; ++j)
      if (u[j] == u[s]) return ETD_ERR_INVALID;
  }
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  const size_t stride = (size_t)c->n_active_host * TILE_PTS;
  const int grid = c->n_active_host > 0 ? c->n_active_host : 1;
  for (int s = 0; s < c->species; ++s)
    HIP_TRY(launch_gather(c->box, u[s], c->slot_tile, c->comp_bits, c->counters + 0,
                          c->ws + (size_t)V_X0 * c->ld + s * stride, grid, c->stream));
  KrylovDev P = krylov_params(c, job_of(scheme));
  P.h = h;
  int r = run_krylov(c, P);
  if (r) return r;
  for (int s = 0; s < c->species; ++s)
    HIP_TRY(launch_scatter(c->box, c->ws + (size_t)V_U * c->ld + s * stride, c->tile_map, c->comp_bits, u[s],
                           c->stream));
  if (stats) {
    r = fill_stats(c, stats);
    if (r) return r;
    int st = latched_status(c);
    if (st) return st;
  }
  return ETD_OK;
}

int etd_ctx_destroy(etd_ctx* c) {
  if (!c) return ETD_ERR_INVALID;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return ETD_OK;
}

int etd_ctx_set_stream(etd_ctx* c, void* s) {
  if (!c) return ETD_ERR_INVALID;
  c->stream = (hipStream_t)s;
  return ETD_OK;
}

int etd_ctx_set_beta(etd_ctx* c, double beta) {
  if (!c || !(beta > 0.0) || !isfinite(beta)) return ETD_ERR_INVALID;
  if (c->var_mode) return ETD_ERR_INVALID;
  c->phys.beta = beta;
  return ETD_OK;
}

int etd_geometry_build(etd_ctx* c, const double* rho) {
  if (!c || !rho) return ETD_ERR_INVALID;
  c->var_mode = false;
  int r = geometry_enqueue(c, rho);
  if (r) return r;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return geometry_finish(c, c->gb.h_cnt);
}

int etd_geometry_build_var(etd_ctx* c, const double* rho, const double* const* beta_face) {
  if (!c || !rho || !beta_face || c->species > 1) return ETD_ERR_INVALID;
  for (int d = 0; d < c->box.dim; ++d)
    if (!beta_face[d]) return ETD_ERR_INVALID;
  if (!c->vcoef) {
    const size_t ld = c->ld;
    bool ok = true;
    ok &= hipMalloc(&c->vcoef, sizeof(double) * ld * (2 * c->box.dim + 1)) == hipSuccess;
    ok &= hipMalloc(&c->tap_n, sizeof(int) * ld) == hipSuccess;
    ok &= hipMalloc(&c->tap_coef, sizeof(double) * ld * TAPS_PER) == hipSuccess;
    ok &= hipMalloc(&c->tap_pt, sizeof(double) * ld * TAPS_PER * 3) == hipSuccess;
    ok &= hipMalloc(&c->tap_off, sizeof(int) * ld) == hipSuccess;
    if (!ok) return ETD_ERR_HIP;
  }
  c->var_mode = false;
  GeomInst& I = c->gb.h_tab[0];
  for (int d = 0; d < 3; ++d) I.beta_face[d] = d < c->box.dim ? beta_face[d] : nullptr;
  I.vcoef = c->vcoef;
  I.tap_n = c->tap_n;
  I.tap_coef = c->tap_coef;
  I.tap_pt = c->tap_pt;
  int r = geometry_enqueue(c, rho);
  if (r) return r;
  HIP_TRY(launch_geometry_var(c->gb, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int d = 0; d < 3; ++d) I.beta_face[d] = nullptr;
  r = geometry_finish(c, c->gb.h_cnt);
  if (r) return r;
  // compact tap numbering (point order: slot, local index, tap), on the host
  const size_t npts = (size_t)c->n_active_host * TILE_PTS;
  std::vector<int> tn(npts), off(npts);
  std::vector<double> pts(npts * TAPS_PER * 3);
  if (npts) {
    HIP_TRY(hipMemcpy(tn.data(), c->tap_n, sizeof(int) * npts, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pts.data(), c->tap_pt, sizeof(double) * npts * TAPS_PER * 3, hipMemcpyDeviceToHost));
  }
  int acc = 0;
  c->h_tap_pts.clear();
  for (size_t p = 0; p < npts; ++p) {
    off[p] = acc;
    for (int k = 0; k < tn[p]; ++k)
      for (int d = 0; d < c->box.dim; ++d) c->h_tap_pts.push_back(pts[(p * TAPS_PER + k) * 3 + d]);
    acc += tn[p];
  }
  c->ntaps = acc;
  if (npts) HIP_TRY(hipMemcpy(c->tap_off, off.data(), sizeof(int) * npts, hipMemcpyHostToDevice));
  c->var_mode = true;
  return ETD_OK;
}

int etd_boundary_taps(etd_ctx* c, int32_t capacity, double* points, int32_t* count) {
  if (!c || !count || capacity < 0) return ETD_ERR_INVALID;
  if (!c->var_mode) return ETD_ERR_NO_GEOMETRY;
  *count = c->ntaps;
  if (points) {
    if (capacity < c->ntaps) return ETD_ERR_INVALID;
    memcpy(points, c->h_tap_pts.data(), sizeof(double) * c->h_tap_pts.size());
  }
  return ETD_OK;
}

int etd_forcing_assemble(etd_ctx* c, const double* ub, const double* src, double* out) {
  if (!c || !out || (c->ntaps > 0 && !ub) || out == src || (const double*)out == ub) return ETD_ERR_INVALID;
  if (!c->var_mode) return ETD_ERR_NO_GEOMETRY;
  return check_hip(launch_forcing(c->box, c->tile_map, c->comp_bits, c->tap_n, c->tap_coef, c->tap_off, ub, src,
                                  out, c->stream));
}

int etd_operator_apply(etd_ctx* c, const double* v, double* out) {
  if (!c || !v || !out || v == out || c->species > 1) return ETD_ERR_INVALID;
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  int r = gather_to(c, v, V_B0);
  if (r) return r;
  r = run_krylov(c, krylov_params(c, JOB_APPLY));
  if (r) return r;
  return scatter_from(c, V_U, out);
}

int phi_combination_apply(etd_ctx* c, double t, int32_t p, const double* const* b, double* out,
                          etd_stats* stats) {
  if (!c || !b || !out || p < 0 || p > PMAX || !(t >= 0.0) || !isfinite(t) || c->species > 1) return ETD_ERR_INVALID;
  for (int k = 0; k <= p; ++k) {
    if (!b[k]) return ETD_ERR_INVALID;
    if (b[k] == out) return ETD_ERR_INVALID;
  }
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  for (int k = 0; k <= p; ++k) {
    int r = gather_to(c, b[k], V_B0 + k);
    if (r) return r;
  }
  KrylovDev P = krylov_params(c, JOB_PHI);
  P.p = p;
  P.t = t;
  int r = run_krylov(c, P);
  if (r) return r;
  r = scatter_from(c, V_U, out);
  if (r) return r;
  if (stats) {
    r = fill_stats(c, stats);
    if (r) return r;
    int st = latched_status(c);
    if (st) return st;
  }
  return ETD_OK;
}

int phi_combination_apply_multi(etd_ctx* c, double t, int32_t p, const double* const* b, double t_mid,
                                double* out_mid, double* out, etd_stats* stats) {
  if (!c || !b || !out || !out_mid || out == out_mid || p < 0 || p > PMAX || !(t > 0.0) || !isfinite(t) ||
      !(t_mid > 0.0) || !(t_mid <= t) || c->species > 1)
    return ETD_ERR_INVALID;
  for (int k = 0; k <= p; ++k)
    if (!b[k] || b[k] == out || b[k] == out_mid) return ETD_ERR_INVALID;
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  for (int k = 0; k <= p; ++k) {
    int r = gather_to(c, b[k], V_B0 + k);
    if (r) return r;
  }
  KrylovDev P = krylov_params(c, JOB_PHI);
  P.p = p;
  P.t = t;
  P.t_mid = t_mid;
  int r = run_krylov(c, P);
  if (r) return r;
  if ((r = scatter_from(c, V_U, out))) return r;
  if ((r = scatter_from(c, V_F, out_mid))) return r;
  if (stats) {
    r = fill_stats(c, stats);
    if (r) return r;
    int st = latched_status(c);
    if (st) return st;
  }
  return ETD_OK;
}

// Steps 1-2 of a context, u (and f, when given: extended from the same
// computational points in the same launches) updated in place; nothing
// changes when the front guard refuses the step.
static int advance_fields(etd_ctx* c, double* rho, double* u, double* f, double dt, int32_t reinit) {
  if (!c->have_geometry) {
    int r = etd_geometry_build(c, rho);
    if (r) return r;
  }
  c->lsb.h_inst[0] = levelset_inst(c, rho, u, f);
  HIP_TRY(timer_begin(c->profiling, c->stream, c->t_levelset));
  HIP_TRY(levelset_begin(c->lsb, dt, reinit, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (front_too_fast(c->lsb)) return ETD_ERR_FRONT;
  HIP_TRY(levelset_end(c->lsb, c->stream));
  HIP_TRY(timer_end(c->profiling, c->stream, c->t_levelset));
  return etd_geometry_build(c, rho);
}

int levelset_advance(etd_ctx* c, double* rho, double* u, double dt, int32_t reinit) {
  if (!c || !rho || !u || !(dt >= 0.0) || !isfinite(dt)) return ETD_ERR_INVALID;
  if (c->var_mode || c->species > 1) return ETD_ERR_INVALID;
  return advance_fields(c, rho, u, nullptr, dt, reinit);
}

int etd_step(etd_ctx* c, int32_t scheme, double h, double* u, double* rho, int32_t reinit,
             etd_stats* stats) {
  if (!c || !u || !(h >= 0.0) || !isfinite(h) || c->species > 1) return ETD_ERR_INVALID;
  if (scheme < ETD_SCHEME_ETD1 || scheme > ETD_SCHEME_ETD4RK_SIMUL) return ETD_ERR_INVALID;
  if (rho) {
    int r = levelset_advance(c, rho, u, h, reinit);
    if (r) return r;
  }
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  int r = gather_to(c, u, V_X0);
  if (r) return r;
  KrylovDev P = krylov_params(c, job_of(scheme));
  P.h = h;
  r = run_krylov(c, P);
  if (r) return r;
  r = scatter_from(c, V_U, u, rho != nullptr);
  if (r) return r;
  if (stats) {
    r = fill_stats(c, stats);
    if (r) return r;
    int st = latched_status(c);
    if (st) return st;
  }
  return ETD_OK;
}

int etd_step_forced(etd_ctx* c, int32_t scheme, double h, double* u, const double* const* g, etd_stats* stats) {
  if (!c || !u || !g || !(h >= 0.0) || !isfinite(h) || c->species > 1) return ETD_ERR_INVALID;
  if (scheme < ETD_SCHEME_ETD1 || scheme > ETD_SCHEME_ETD4RK_SIMUL) return ETD_ERR_INVALID;
  // the stage times each scheme evaluates F at: 0 = t_n, 1 = t_n + h/2, 2 = t_n + h
  const bool need[3] = {true, scheme >= ETD_SCHEME_ETD3RK, scheme >= ETD_SCHEME_ETD2RK};
  for (int k = 0; k < 3; ++k) {
    if (need[k] && !g[k]) return ETD_ERR_INVALID;
    if (need[k] && g[k] == u) return ETD_ERR_INVALID;
  }
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  int r = gather_to(c, u, V_X0);
  if (r) return r;
  for (int k = 0; k < 3; ++k)
    if (need[k] && (r = gather_to(c, g[k], V_FG0 + k))) return r;
  KrylovDev P = krylov_params(c, job_of(scheme));
  P.h = h;
  P.forced = 1;
  r = run_krylov(c, P);
  if (r) return r;
  r = scatter_from(c, V_U, u);
  if (r) return r;
  if (stats) {
    r = fill_stats(c, stats);
    if (r) return r;
    int st = latched_status(c);
    if (st) return st;
  }
  return ETD_OK;
}

int etd_multistep_step(etd_ctx* c, double h, double* u, double* f_prev, int32_t first, double* rho,
                       int32_t reinit, etd_stats* stats) {
  if (!c || !u || !f_prev || f_prev == u || f_prev == rho || !(h >= 0.0) || !isfinite(h)) return ETD_ERR_INVALID;
  if ((rho && c->var_mode) || c->species > 1) return ETD_ERR_INVALID;
  if (rho) {
    // F_{n-1} extended with u from the computational points of the current
    // rho, in the same launches
    int r = advance_fields(c, rho, u, first ? nullptr : f_prev, h, reinit);
    if (r) return r;
  }
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  int r = gather_to(c, u, V_X0);
  if (r) return r;
  if (!first) {
    r = gather_to(c, f_prev, V_G);
    if (r) return r;
  }
  KrylovDev P = krylov_params(c, JOB_ETD2);
  P.h = h;
  P.first = first ? 1 : 0;
  r = run_krylov(c, P);
  if (r) return r;
  r = scatter_from(c, V_U, u, rho != nullptr);
  if (r) return r;
  r = scatter_from(c, V_G, f_prev);
  if (r) return r;
  if (stats) {
    r = fill_stats(c, stats);
    if (r) return r;
    int st = latched_status(c);
    if (st) return st;
  }
  return ETD_OK;
}

int etd_adjoint_step(etd_ctx* c, int32_t scheme, double h, const double* u_n, const double* gbar_np1,
                     double* gbar_n, double* dL_dbeta) {
  if (!c || !u_n || !gbar_np1 || !gbar_n || !dL_dbeta || !(h >= 0.0) || !isfinite(h)) return ETD_ERR_INVALID;
  if (scheme != ETD_SCHEME_ETD2RK || gbar_n == u_n || c->var_mode || c->species > 1) return ETD_ERR_INVALID;
  if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  int r = gather_to(c, u_n, V_X0);
  if (r) return r;
  r = gather_to(c, gbar_np1, V_G);
  if (r) return r;
  KrylovDev P = krylov_params(c, JOB_ADJ_ETD2RK);
  P.h = h;
  P.beta = c->phys.beta;
  P.dbeta = dL_dbeta;
  r = run_krylov(c, P);
  if (r) return r;
  return scatter_from(c, V_U, gbar_n);
}

int etd_ctx_sync(etd_ctx* c) {
  if (!c) return ETD_ERR_INVALID;
  return latched_status(c);
}

int etd_ctx_stats(etd_ctx* c, etd_stats* s) {
  if (!c || !s) return ETD_ERR_INVALID;
  return fill_stats(c, s);
}

int etd_ctx_profile_enable(etd_ctx* c, int32_t enable) {
  if (!c) return ETD_ERR_INVALID;
  c->profiling = enable != 0;
  return ETD_OK;
}

int etd_ctx_profile_read(etd_ctx* c, etd_profile* out, int32_t reset) {
  if (!c || !out) return ETD_ERR_INVALID;
  HIP_TRY(hipMemcpyAsync(c->h_state, c->st, sizeof(KrylovStateDev), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(c->h_counters, c->counters, NCOUNTERS * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(timer_collect(c->t_krylov));
  HIP_TRY(timer_collect(c->t_levelset));
  HIP_TRY(timer_collect(c->t_geometry));
  out->krylov_ms = c->t_krylov.ms;
  out->levelset_ms = c->t_levelset.ms;
  out->geometry_ms = c->t_geometry.ms;
  out->krylov_launches = c->t_krylov.count;
  out->levelset_calls = c->t_levelset.count;
  out->geometry_calls = c->t_geometry.count;
  out->alg_bytes = c->h_state->alg_bytes_total;
  out->n_unknowns = c->h_counters[c->species > 1 ? 6 : 4];
  out->krylov_device_ms = c->h_state->ticks_total / c->clock_khz;
  out->krylov_sync_ms = c->h_state->ticks_sync / c->clock_khz;
  out->krylov_expm_ms = c->h_state->ticks_expm / c->clock_khz;
  out->krylov_pass_ms = c->h_state->ticks_pass / c->clock_khz;
  out->krylov_prologue_ms = c->h_state->ticks_pro / c->clock_khz;
  out->krylov_gap_ms = c->h_state->ticks_gap / c->clock_khz;
  out->krylov_syncs = c->h_state->syncs;
  out->krylov_expms = c->h_state->expm_calls;
  if (reset) {
    c->t_krylov.ms = c->t_levelset.ms = c->t_geometry.ms = 0.0;
    c->t_krylov.count = c->t_levelset.count = c->t_geometry.count = 0;
    HIP_TRY(reset_counters(c->st, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return ETD_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch

namespace {

void graph_drop(etd_batch* B);
void fgraph_drop(etd_batch* B);

void batch_free(etd_batch* B) {
  for (etd_ctx* c : B->inst)
    if (c) etd_ctx_destroy(c);
  B->inst.clear();
  if (B->d_params) (void)hipFree(B->d_params);
  if (B->d_blk) (void)hipFree(B->d_blk);
  if (B->h_params) (void)hipHostFree(B->h_params);
  if (B->h_blk) (void)hipHostFree(B->h_blk);
  if (B->staged) (void)hipEventDestroy(B->staged);
  if (B->uptr_done) (void)hipEventDestroy(B->uptr_done);
  if (B->h_uptr) (void)hipHostFree(B->h_uptr);
  if (B->d_uptr) (void)hipFree(B->d_uptr);
  levelset_batch_free(B->lsb);
  geom_batch_free(B->gb);
  graph_drop(B);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  if (B->d_gparams) (void)hipFree(B->d_gparams);
  if (B->d_gblk) (void)hipFree(B->d_gblk);
  if (B->d_guptr) (void)hipFree(B->d_guptr);
  fgraph_drop(B);
  levelset_batch_free(B->flsb);
  geom_batch_free(B->fgb);
  if (B->d_fparams) (void)hipFree(B->d_fparams);
  if (B->d_fblk) (void)hipFree(B->d_fblk);
  if (B->d_fuptr) (void)hipFree(B->d_fuptr);
  timer_free(B->t_krylov);
  timer_free(B->t_levelset);
  timer_free(B->t_geometry);
}

// Block schedule of chunk ch (instances i0 .. i0+n-1, at most `capacity`):
// every instance gets one block; the remaining co-resident blocks go to the
// instances in proportion to the blocks they could use (one loop trip over
// their active tiles), capped by group_limit.  Fills params[0..n) and
// blk[0..blocks); returns the number of blocks, *coop whether some instance
// has more than one block.
int batch_schedule(const etd_batch* B, int ch, int mode, double h, KrylovDev* params, int* blk, bool* coop) {
  const int C = B->capacity;
  const int i0 = ch * C;
  const int i1 = (i0 + C < B->count) ? i0 + C : B->count;
  const int n = i1 - i0;
  std::vector<int> want(n), g(n, 1);
  long total_want = 0;
  for (int i = 0; i < n; ++i) {
    const int nact = B->inst[i0 + i]->n_active_host > 0 ? B->inst[i0 + i]->n_active_host : 1;
    int w = (nact + KB_TILES[KB_LARGE] - 1) / KB_TILES[KB_LARGE];
    if (B->group_limit > 0 && w > B->group_limit) w = B->group_limit;
    want[i] = w;
    total_want += w - 1;
  }
  const long budget = C - n;
  for (int i = 0; i < n; ++i) {
    if (total_want <= budget) g[i] = want[i];
    else g[i] = 1 + (int)((budget * (long)(want[i] - 1)) / (total_want > 0 ? total_want : 1));
  }
  int blocks = 0;
  *coop = false;
  for (int i = 0; i < n; ++i) {
    // the groups of a batch keep the all-to-all synchronisation (measured
    // faster on batch64 in every group size it has)
    KrylovDev P = krylov_params(B->inst[i0 + i], mode, INT32_MAX);
    P.h = h;
    P.first = B->ms_first;
    if (B->stage_min >= 0) P.stage_min = B->stage_min;
    P.g_first = blocks;
    P.g_size = g[i];
    params[i] = P;
    for (int k = 0; k < g[i]; ++k) blk[blocks + k] = i;
    blocks += g[i];
    *coop |= g[i] > 1;
  }
  return blocks;
}

// One batched launch per chunk of at most `capacity` instances (schedule
// above); cooperative when some instance has more than one block.
int batch_run_krylov(etd_batch* B, int mode, double h) {
  if (B->staged_pending) {
    HIP_TRY(hipEventSynchronize(B->staged));
    B->staged_pending = false;
  }
  HIP_TRY(timer_begin(B->profiling, B->stream, B->t_krylov));
  const int C = B->capacity;
  for (int ch = 0; ch < B->nchunks; ++ch) {
    const int i0 = ch * C;
    const int n = ((i0 + C < B->count) ? i0 + C : B->count) - i0;
    bool coop = false;
    int* blk = B->h_blk + (size_t)ch * C;
    const int blocks = batch_schedule(B, ch, mode, h, B->h_params + i0, blk, &coop);
    HIP_TRY(hipMemcpyAsync(B->d_params + i0, B->h_params + i0, sizeof(KrylovDev) * n, hipMemcpyHostToDevice,
                           B->stream));
    HIP_TRY(hipMemcpyAsync(B->d_blk + (size_t)ch * C, blk, sizeof(int) * blocks, hipMemcpyHostToDevice,
                           B->stream));
    HIP_TRY(launch_krylov_group(KB_LARGE, B->dim, B->d_params + i0, n, B->d_blk + (size_t)ch * C, blocks, coop,
                                B->stream));
  }
  HIP_TRY(hipEventRecord(B->staged, B->stream));
  B->staged_pending = true;
  HIP_TRY(timer_end(B->profiling, B->stream, B->t_krylov));
  return ETD_OK;
}

void graph_drop(etd_batch* B) {
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->gexec = nullptr;
  B->graph = nullptr;
  B->g_geom = -1;
}

// Record the frozen-domain step (scheme, h, u) as a graph: parameters into
// the graph's own device buffers (synchronous copies), then the captured
// gather, group-barrier reset, Krylov launch (an ordinary launch: its
// blocks fit the co-resident capacity) and scatter.
int graph_record(etd_batch* B, int scheme, double h, double* const* u) {
  graph_drop(B);
  const int n = B->count;
  const int mode = job_of(scheme);
  std::vector<KrylovDev> params(n);
  std::vector<int> blk(B->capacity);
  bool coop = false;
  const int blocks = batch_schedule(B, 0, mode, h, params.data(), blk.data(), &coop);
  HIP_TRY(hipStreamSynchronize(B->stream));
  HIP_TRY(hipMemcpy(B->d_gparams, params.data(), sizeof(KrylovDev) * n, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(B->d_gblk, blk.data(), sizeof(int) * blocks, hipMemcpyHostToDevice));
  std::vector<const double*> up(u, u + n);
  HIP_TRY(hipMemcpy(B->d_guptr, up.data(), sizeof(double*) * n, hipMemcpyHostToDevice));
  // recorded on the batch's own stream (the caller's may be the legacy
  // default stream, which cannot be captured); replayed on the caller's
  if (!B->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = B->cap_stream;
  HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  hipError_t e = launch_gather_batch(B->gb, B->d_guptr, V_X0, cs);
  if (e == hipSuccess) e = launch_krylov_group(KB_LARGE, B->dim, B->d_gparams, n, B->d_gblk, blocks, false, cs);
  if (e == hipSuccess) e = launch_scatter_batch(B->gb, (double* const*)B->d_guptr, V_U, cs);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(cs, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return ETD_ERR_HIP;
  }
  B->graph = g;
  if (hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
    graph_drop(B);
    return ETD_ERR_HIP;
  }
  B->g_scheme = scheme;
  B->g_h = h;
  B->g_geom = B->geom_gen;
  B->g_limit = B->group_limit;
  B->g_stage = B->stage_min;
  B->g_u.assign(u, u + n);
  return ETD_OK;
}

void fgraph_drop(etd_batch* B) {
  for (int r = 0; r < 2; ++r) {
    if (B->fgexec[r]) (void)hipGraphExecDestroy(B->fgexec[r]);
    if (B->fgraph[r]) (void)hipGraphDestroy(B->fgraph[r]);
    B->fgexec[r] = nullptr;
    B->fgraph[r] = nullptr;
  }
  B->f_u.clear();
  B->f_rho.clear();
}

// Record one free-boundary step of every instance (scheme, h; u and rho
// updated in place) twice, without and with the reinitialisation: the
// level set and the geometry device-sized (launch rows from the device
// counters, fixed grids, the front guard checked on the device), then the
// gather, the batched Krylov launch (the block schedule of the current
// active tiles; an ordinary launch, as in graph_record) and the scatter.
int graph_free_record(etd_batch* B, int scheme, double h, double* const* u, double* const* rho) {
  fgraph_drop(B);
  const int n = B->count;
  if (!B->f_alloc) {
    bool ok = levelset_batch_alloc(B->flsb, n, B->dim) == hipSuccess;
    ok &= geom_batch_alloc(B->fgb, n, NCOUNTERS) == hipSuccess;
    ok &= hipMalloc(&B->d_fparams, sizeof(KrylovDev) * n) == hipSuccess;
    ok &= hipMalloc(&B->d_fblk, sizeof(int) * (size_t)B->capacity) == hipSuccess;
    ok &= hipMalloc(&B->d_fuptr, sizeof(double*) * n) == hipSuccess;
    if (!ok) return ETD_ERR_HIP;
    for (int i = 0; i < n; ++i) B->fgb.h_tab[i] = geom_inst(B->inst[i]);
    HIP_TRY(geom_batch_prefix(B->fgb));
    B->f_alloc = true;
  }
  HIP_TRY(hipStreamSynchronize(B->stream));
  for (int i = 0; i < n; ++i) {
    B->fgb.h_tab[i].rho = rho[i];
    B->flsb.h_inst[i] = levelset_inst(B->inst[i], rho[i], u[i]);
  }
  B->flsb.device_sized = true;
  HIP_TRY(levelset_upload(B->flsb, B->stream));
  HIP_TRY(geom_upload(B->fgb, B->stream));
  const int mode = job_of(scheme);
  std::vector<KrylovDev> params(n);
  std::vector<int> blk(B->capacity);
  bool coop = false;
  const int blocks = batch_schedule(B, 0, mode, h, params.data(), blk.data(), &coop);
  HIP_TRY(hipStreamSynchronize(B->stream));
  HIP_TRY(hipMemcpy(B->d_fparams, params.data(), sizeof(KrylovDev) * n, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(B->d_fblk, blk.data(), sizeof(int) * blocks, hipMemcpyHostToDevice));
  std::vector<const double*> up(u, u + n);
  HIP_TRY(hipMemcpy(B->d_fuptr, up.data(), sizeof(double*) * n, hipMemcpyHostToDevice));
  if (!B->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = B->cap_stream;
  for (int r = 0; r < 2; ++r) {
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = levelset_begin(B->flsb, h, r, cs);
    if (e == hipSuccess) e = levelset_end(B->flsb, cs);
    if (e == hipSuccess) e = launch_geometry(B->fgb, GEOM_RADII, cs, true);
    if (e == hipSuccess) e = launch_gather_batch(B->fgb, B->d_fuptr, V_X0, cs);
    if (e == hipSuccess) e = launch_krylov_group(KB_LARGE, B->dim, B->d_fparams, n, B->d_fblk, blocks, false, cs);
    if (e == hipSuccess) e = launch_scatter_batch(B->fgb, (double* const*)B->d_fuptr, V_U, cs);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      fgraph_drop(B);
      return ETD_ERR_HIP;
    }
    B->fgraph[r] = g;
    if (hipGraphInstantiate(&B->fgexec[r], g, nullptr, nullptr, 0) != hipSuccess) {
      fgraph_drop(B);
      return ETD_ERR_HIP;
    }
  }
  B->f_scheme = scheme;
  B->f_h = h;
  B->f_limit = B->group_limit;
  B->f_stage = B->stage_min;
  B->f_u.assign(u, u + n);
  B->f_rho.assign(rho, rho + n);
  return ETD_OK;
}

// After replayed free-boundary steps: the host's copies of every instance's
// counters (active tiles, list sizes) from the device.
int refresh_host(etd_batch* B) {
  if (!B->host_stale) return ETD_OK;
  for (etd_ctx* c : B->inst)
    HIP_TRY(hipMemcpyAsync(c->h_counters, c->counters, NCOUNTERS * sizeof(int), hipMemcpyDeviceToHost, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  for (etd_ctx* c : B->inst) {
    c->n_active_host = c->h_counters[0];
    for (int q = 0; q <= LS_C_MAX; ++q) c->ncum_c[q] = c->h_counters[LS_CNT_C + q];
    for (int q = 0; q <= LS_V_MAX; ++q) c->ncum_v[q] = c->h_counters[LS_CNT_V + q];
    c->nu_host = c->h_counters[LS_CNT_U];
    choose_launch(c);
  }
  B->host_stale = false;
  return ETD_OK;
}

}  // namespace

extern "C" {

int etd_batch_create(int32_t count, const etd_grid* grids, const etd_physics* phys,
                     const etd_krylov_opts* opts, void* hip_stream, etd_batch** out) {
  if (!out) return ETD_ERR_INVALID;
  *out = nullptr;
  if (count < 1 || !grids || !phys) return ETD_ERR_INVALID;
  for (int i = 1; i < count; ++i)
    if (grids[i].dim != grids[0].dim) return ETD_ERR_INVALID;
  etd_batch* B = new etd_batch();
  B->count = count;
  B->dim = grids[0].dim;
  B->stream = (hipStream_t)hip_stream;
  B->inst.assign(count, nullptr);
  for (int i = 0; i < count; ++i) {
    const int r = etd_ctx_create(&grids[i], &phys[i], opts, hip_stream, &B->inst[i]);
    if (r) {
      batch_free(B);
      delete B;
      return r;
    }
  }
  B->capacity = B->inst[0]->max_grid_kb[KB_LARGE];   // batches run the 1024-thread build
  B->nchunks = (count + B->capacity - 1) / B->capacity;
  bool ok = true;
  ok &= hipMalloc(&B->d_params, sizeof(KrylovDev) * count) == hipSuccess;
  ok &= hipHostMalloc(&B->h_params, sizeof(KrylovDev) * count) == hipSuccess;
  ok &= hipMalloc(&B->d_blk, sizeof(int) * (size_t)B->capacity * B->nchunks) == hipSuccess;
  ok &= hipHostMalloc(&B->h_blk, sizeof(int) * (size_t)B->capacity * B->nchunks) == hipSuccess;
  ok &= hipEventCreate(&B->staged) == hipSuccess;
  ok &= levelset_batch_alloc(B->lsb, count, B->dim) == hipSuccess;
  ok &= hipHostMalloc(&B->h_uptr, sizeof(double*) * 2 * count) == hipSuccess;
  ok &= hipMalloc(&B->d_uptr, sizeof(double*) * 2 * count) == hipSuccess;
  ok &= hipEventCreateWithFlags(&B->uptr_done, hipEventDisableTiming) == hipSuccess;
  ok &= geom_batch_alloc(B->gb, count, NCOUNTERS) == hipSuccess;
  ok &= hipMalloc(&B->d_gparams, sizeof(KrylovDev) * count) == hipSuccess;
  ok &= hipMalloc(&B->d_gblk, sizeof(int) * (size_t)B->capacity) == hipSuccess;
  ok &= hipMalloc(&B->d_guptr, sizeof(double*) * count) == hipSuccess;
  if (ok) {
    for (int i = 0; i < count; ++i) B->gb.h_tab[i] = geom_inst(B->inst[i]);
    ok &= geom_batch_prefix(B->gb) == hipSuccess;
  }
  if (!ok) {
    batch_free(B);
    delete B;
    return ETD_ERR_HIP;
  }
  *out = B;
  return ETD_OK;
}

int etd_batch_destroy(etd_batch* B) {
  if (!B) return ETD_ERR_INVALID;
  (void)hipStreamSynchronize(B->stream);
  batch_free(B);
  delete B;
  return ETD_OK;
}

int etd_batch_set_stream(etd_batch* B, void* s) {
  if (!B) return ETD_ERR_INVALID;
  B->stream = (hipStream_t)s;
  for (etd_ctx* c : B->inst) c->stream = (hipStream_t)s;
  return ETD_OK;
}

int etd_batch_set_group_limit(etd_batch* B, int32_t max_blocks) {
  if (!B || max_blocks < 0) return ETD_ERR_INVALID;
  B->group_limit = max_blocks;
  return ETD_OK;
}

int etd_batch_set_stage_min(etd_batch* B, int32_t min_tiles) {
  if (!B || min_tiles < -1) return ETD_ERR_INVALID;
  B->stage_min = min_tiles;
  return ETD_OK;
}

int etd_batch_geometry_build(etd_batch* B, const double* const* rho) {
  if (!B || !rho) return ETD_ERR_INVALID;
  for (int i = 0; i < B->count; ++i)
    if (!rho[i]) return ETD_ERR_INVALID;
  B->host_stale = false;   // the build refreshes the host's counters
  // the table upload reads pinned memory: the previous build has been
  // synchronised, so it may be rewritten
  for (int i = 0; i < B->count; ++i) B->gb.h_tab[i].rho = rho[i];
  HIP_TRY(timer_begin(B->profiling, B->stream, B->t_geometry));
  HIP_TRY(launch_geometry(B->gb, GEOM_RADII, B->stream));
  HIP_TRY(timer_end(B->profiling, B->stream, B->t_geometry));
  HIP_TRY(hipStreamSynchronize(B->stream));
  ++B->geom_gen;
  int first = ETD_OK;
  for (int i = 0; i < B->count; ++i) {
    const int r = geometry_finish(B->inst[i], B->gb.h_cnt + (size_t)i * NCOUNTERS);
    if (r && !first) first = r;
  }
  return first;
}

// Upload the box pointers of this step (u, and f when not NULL) from pinned
// memory once the previous upload has been read.
static int upload_ptrs(etd_batch* B, double* const* u, double* const* f) {
  if (B->uptr_pending) {
    HIP_TRY(hipEventSynchronize(B->uptr_done));
    B->uptr_pending = false;
  }
  const int n = B->count;
  for (int i = 0; i < n; ++i) B->h_uptr[i] = u[i];
  if (f)
    for (int i = 0; i < n; ++i) B->h_uptr[n + i] = f[i];
  HIP_TRY(hipMemcpyAsync(B->d_uptr, B->h_uptr, sizeof(double*) * (f ? 2 * n : n), hipMemcpyHostToDevice,
                         B->stream));
  HIP_TRY(hipEventRecord(B->uptr_done, B->stream));
  B->uptr_pending = true;
  return ETD_OK;
}

// Level-set Steps 1-2a of every instance in shared launches (one
// synchronisation), then the geometry of the moved boundaries.
static int batch_levelset(etd_batch* B, double h, double* const* u, double* const* rho, int32_t reinit,
                          double* const* f = nullptr) {
  for (int i = 0; i < B->count; ++i)
    B->lsb.h_inst[i] = levelset_inst(B->inst[i], rho[i], u[i], f ? f[i] : nullptr);
  HIP_TRY(timer_begin(B->profiling, B->stream, B->t_levelset));
  HIP_TRY(levelset_begin(B->lsb, h, reinit, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  if (front_too_fast(B->lsb)) return ETD_ERR_FRONT;
  HIP_TRY(levelset_end(B->lsb, B->stream));
  HIP_TRY(timer_end(B->profiling, B->stream, B->t_levelset));
  return etd_batch_geometry_build(B, rho);
}

static int batch_stats(etd_batch* B, etd_stats* stats) {
  for (int i = 0; i < B->count; ++i) {
    int r = fill_stats(B->inst[i], &stats[i]);
    if (r) return r;
  }
  return etd_batch_sync(B);
}

int etd_batch_step(etd_batch* B, int32_t scheme, double h, double* const* u, double* const* rho,
                   int32_t reinit, etd_stats* stats) {
  if (!B || !u || !(h >= 0.0) || !isfinite(h)) return ETD_ERR_INVALID;
  if (scheme < ETD_SCHEME_ETD1 || scheme > ETD_SCHEME_ETD4RK_SIMUL) return ETD_ERR_INVALID;
  for (int i = 0; i < B->count; ++i) {
    if (!u[i]) return ETD_ERR_INVALID;
    if (rho && !rho[i]) return ETD_ERR_INVALID;
  }
  int r;
  if ((r = refresh_host(B))) return r;
  if (rho) {
    bool all = true;
    for (etd_ctx* c : B->inst) all &= c->have_geometry;
    if (!all && (r = etd_batch_geometry_build(B, rho))) return r;
    if ((r = batch_levelset(B, h, u, rho, reinit))) return r;
  }
  for (etd_ctx* c : B->inst)
    if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  if ((r = upload_ptrs(B, u, nullptr))) return r;
  HIP_TRY(launch_gather_batch(B->gb, B->d_uptr, V_X0, B->stream));
  if ((r = batch_run_krylov(B, job_of(scheme), h))) return r;
  HIP_TRY(launch_scatter_batch(B->gb, (double* const*)B->d_uptr, V_U, B->stream));
  return stats ? batch_stats(B, stats) : ETD_OK;
}

int etd_batch_multistep_step(etd_batch* B, double h, double* const* u, double* const* f_prev, int32_t first,
                             double* const* rho, int32_t reinit, etd_stats* stats) {
  if (!B || !u || !f_prev || !(h >= 0.0) || !isfinite(h)) return ETD_ERR_INVALID;
  for (int i = 0; i < B->count; ++i) {
    if (!u[i] || !f_prev[i] || f_prev[i] == u[i]) return ETD_ERR_INVALID;
    if (rho && (!rho[i] || f_prev[i] == rho[i])) return ETD_ERR_INVALID;
  }
  int r;
  if ((r = refresh_host(B))) return r;
  if (rho) {
    bool all = true;
    for (etd_ctx* c : B->inst) all &= c->have_geometry;
    if (!all && (r = etd_batch_geometry_build(B, rho))) return r;
    // F_{n-1} of every instance extended with its u from the computational
    // points of its current rho, in the same launches
    if ((r = batch_levelset(B, h, u, rho, reinit, first ? nullptr : f_prev))) return r;
  }
  for (etd_ctx* c : B->inst)
    if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  if ((r = upload_ptrs(B, u, f_prev))) return r;
  HIP_TRY(launch_gather_batch(B->gb, B->d_uptr, V_X0, B->stream));
  if (!first) HIP_TRY(launch_gather_batch(B->gb, B->d_uptr + B->count, V_G, B->stream));
  B->ms_first = first ? 1 : 0;
  r = batch_run_krylov(B, JOB_ETD2, h);
  B->ms_first = 0;
  if (r) return r;
  HIP_TRY(launch_scatter_batch(B->gb, (double* const*)B->d_uptr, V_U, B->stream));
  HIP_TRY(launch_scatter_batch(B->gb, (double* const*)B->d_uptr + B->count, V_G, B->stream));
  return stats ? batch_stats(B, stats) : ETD_OK;
}

int etd_batch_graph_steps(etd_batch* B, int32_t scheme, double h, double* const* u, int32_t nsteps) {
  if (!B || !u || nsteps < 0 || !(h >= 0.0) || !isfinite(h)) return ETD_ERR_INVALID;
  if (scheme < ETD_SCHEME_ETD1 || scheme > ETD_SCHEME_ETD4RK_SIMUL) return ETD_ERR_INVALID;
  for (int i = 0; i < B->count; ++i)
    if (!u[i]) return ETD_ERR_INVALID;
  for (etd_ctx* c : B->inst)
    if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  if (B->nchunks != 1) return ETD_ERR_INVALID;
  int rr = refresh_host(B);
  if (rr) return rr;
  bool same = B->gexec && B->g_scheme == scheme && B->g_h == h && B->g_geom == B->geom_gen &&
              B->g_limit == B->group_limit && B->g_stage == B->stage_min && (int)B->g_u.size() == B->count;
  for (int i = 0; same && i < B->count; ++i) same = B->g_u[i] == u[i];
  if (!same) {
    const int r = graph_record(B, scheme, h, u);
    if (r) return r;
  }
  HIP_TRY(timer_begin(B->profiling, B->stream, B->t_krylov));
  for (int k = 0; k < nsteps; ++k) HIP_TRY(hipGraphLaunch(B->gexec, B->stream));
  HIP_TRY(timer_end(B->profiling, B->stream, B->t_krylov));
  return ETD_OK;
}

int etd_batch_graph_free_steps(etd_batch* B, int32_t scheme, double h, double* const* u, double* const* rho,
                               int32_t reinit_every, int32_t step0, int32_t nsteps) {
  if (!B || !u || !rho || nsteps < 0 || step0 < 0 || reinit_every < 0 || !(h >= 0.0) || !isfinite(h))
    return ETD_ERR_INVALID;
  if (scheme < ETD_SCHEME_ETD1 || scheme > ETD_SCHEME_ETD4RK_SIMUL) return ETD_ERR_INVALID;
  for (int i = 0; i < B->count; ++i)
    if (!u[i] || !rho[i] || u[i] == rho[i]) return ETD_ERR_INVALID;
  if (B->nchunks != 1) return ETD_ERR_INVALID;
  int r = refresh_host(B);
  if (r) return r;
  bool all = true;
  for (etd_ctx* c : B->inst) all &= c->have_geometry;
  if (!all && (r = etd_batch_geometry_build(B, rho))) return r;
  bool same = B->fgexec[0] && B->fgexec[1] && B->f_scheme == scheme && B->f_h == h &&
              B->f_limit == B->group_limit && B->f_stage == B->stage_min && (int)B->f_u.size() == B->count;
  for (int i = 0; same && i < B->count; ++i) same = B->f_u[i] == u[i] && B->f_rho[i] == rho[i];
  if (!same) {
    const bool prof = B->profiling;
    B->profiling = false;
    r = graph_free_record(B, scheme, h, u, rho);
    B->profiling = prof;
    if (r) return r;
  }
  HIP_TRY(timer_begin(B->profiling, B->stream, B->t_krylov));
  for (int k = 0; k < nsteps; ++k) {
    const int reinit = (reinit_every > 0 && (step0 + k + 1) % reinit_every == 0) ? 1 : 0;
    HIP_TRY(hipGraphLaunch(B->fgexec[reinit], B->stream));
  }
  HIP_TRY(timer_end(B->profiling, B->stream, B->t_krylov));
  if (nsteps > 0) {
    B->host_stale = true;
    ++B->geom_gen;
  }
  return ETD_OK;
}

int etd_batch_autotune(etd_batch* B, int32_t scheme, double h, double* const* u, int32_t trials,
                       int32_t* limit_out, int32_t* stage_out, double* ms_out) {
  if (!B || !u || trials < 1 || !(h >= 0.0) || !isfinite(h)) return ETD_ERR_INVALID;
  if (scheme < ETD_SCHEME_ETD1 || scheme > ETD_SCHEME_ETD4RK_SIMUL) return ETD_ERR_INVALID;
  for (int i = 0; i < B->count; ++i)
    if (!u[i]) return ETD_ERR_INVALID;
  int rr = refresh_host(B);
  if (rr) return rr;
  for (etd_ctx* c : B->inst)
    if (!c->have_geometry) return ETD_ERR_NO_GEOMETRY;
  const int mode = job_of(scheme);
  const int n = B->count;
  // inputs into the workspaces (as a frozen step would gather them)
  HIP_TRY(hipStreamSynchronize(B->stream));
  B->uptr_pending = false;
  for (int i = 0; i < n; ++i) B->h_uptr[i] = u[i];
  HIP_TRY(hipMemcpy(B->d_uptr, B->h_uptr, sizeof(double*) * n, hipMemcpyHostToDevice));
  HIP_TRY(launch_gather_batch(B->gb, B->d_uptr, V_X0, B->stream));
  // the adaptive state before the trials, restored before each run
  KrylovStateDev* save = nullptr;
  HIP_TRY(hipMalloc(&save, sizeof(KrylovStateDev) * n));
  auto restore = [&](bool to_save) -> hipError_t {
    for (int i = 0; i < n; ++i) {
      hipError_t e = to_save ? hipMemcpyAsync(save + i, B->inst[i]->st, sizeof(KrylovStateDev),
                                              hipMemcpyDeviceToDevice, B->stream)
                             : hipMemcpyAsync(B->inst[i]->st, save + i, sizeof(KrylovStateDev),
                                              hipMemcpyDeviceToDevice, B->stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int result = ETD_OK;
  const bool prof = B->profiling;
  const int old_limit = B->group_limit, old_stage = B->stage_min;
  static const int cand[6] = {1, 2, 4, 8, 16, 0};
  static const int stage_cand[3] = {0, STAGE_MIN_TILES, INT32_MAX};
  double best = 1e300;
  int best_limit = old_limit, best_stage = old_stage;
  B->profiling = false;
  if (restore(true) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    result = ETD_ERR_HIP;
  }
  for (int q = 0; q < ETD_AUTOTUNE_CANDIDATES && result == ETD_OK; ++q) {
    B->group_limit = cand[q / 3];
    B->stage_min = stage_cand[q % 3];
    double sum = 0.0;
    for (int rep = 0; rep <= trials && result == ETD_OK; ++rep) {
      float ms = 0.0f;
      if (restore(false) != hipSuccess || hipEventRecord(e0, B->stream) != hipSuccess) { result = ETD_ERR_HIP; break; }
      const int r = batch_run_krylov(B, mode, h);
      if (r) { result = r; break; }
      if (hipEventRecord(e1, B->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { result = ETD_ERR_HIP; break; }
      if (rep > 0) sum += ms;
    }
    const double mean = sum / trials;
    if (ms_out) ms_out[q] = mean;
    if (result == ETD_OK && mean < best) {
      best = mean;
      best_limit = B->group_limit;
      best_stage = B->stage_min;
    }
  }
  B->group_limit = result == ETD_OK ? best_limit : old_limit;
  B->stage_min = result == ETD_OK ? best_stage : old_stage;
  B->profiling = prof;
  if (restore(false) != hipSuccess && result == ETD_OK) result = ETD_ERR_HIP;
  if (hipStreamSynchronize(B->stream) != hipSuccess && result == ETD_OK) result = ETD_ERR_HIP;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(save);
  if (result == ETD_OK) result = etd_batch_sync(B);   // a device error in a trial
  if (limit_out) *limit_out = B->group_limit;
  if (stage_out) *stage_out = B->stage_min;
  return result;
}

int etd_batch_sync(etd_batch* B) {
  if (!B) return ETD_ERR_INVALID;
  for (etd_ctx* c : B->inst)
    HIP_TRY(hipMemcpyAsync(c->h_counters, c->counters, 4 * sizeof(int), hipMemcpyDeviceToHost, B->stream));
  HIP_TRY(hipStreamSynchronize(B->stream));
  int first = ETD_OK;
  for (etd_ctx* c : B->inst) {
    const int st = c->h_counters[1];
    if (st != 0) {
      if (!first) first = st;
      int zero = 0;
      HIP_TRY(hipMemcpyAsync(c->counters + 1, &zero, sizeof(int), hipMemcpyHostToDevice, B->stream));
    }
  }
  HIP_TRY(hipStreamSynchronize(B->stream));
  return first;
}

int etd_batch_stats(etd_batch* B, int32_t i, etd_stats* s) {
  if (!B || !s || i < 0 || i >= B->count) return ETD_ERR_INVALID;
  return fill_stats(B->inst[i], s);
}

int etd_batch_profile_enable(etd_batch* B, int32_t enable) {
  if (!B) return ETD_ERR_INVALID;
  B->profiling = enable != 0;
  return ETD_OK;
}

int etd_batch_profile_read(etd_batch* B, etd_profile* out, int32_t reset) {
  if (!B || !out) return ETD_ERR_INVALID;
  for (etd_ctx* c : B->inst) {
    HIP_TRY(hipMemcpyAsync(c->h_state, c->st, sizeof(KrylovStateDev), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipMemcpyAsync(c->h_counters, c->counters, NCOUNTERS * sizeof(int), hipMemcpyDeviceToHost, B->stream));
  }
  HIP_TRY(hipStreamSynchronize(B->stream));
  HIP_TRY(timer_collect(B->t_krylov));
  HIP_TRY(timer_collect(B->t_levelset));
  HIP_TRY(timer_collect(B->t_geometry));
  out->krylov_ms = B->t_krylov.ms;
  out->levelset_ms = B->t_levelset.ms;
  out->geometry_ms = B->t_geometry.ms;
  out->krylov_launches = B->t_krylov.count;
  out->levelset_calls = B->t_levelset.count;
  out->geometry_calls = B->t_geometry.count;
  double bytes = 0.0;
  long unknowns = 0;
  for (etd_ctx* c : B->inst) {
    bytes += c->h_state->alg_bytes_total;
    unknowns += c->h_counters[4];
  }
  out->alg_bytes = bytes;
  out->n_unknowns = (int32_t)unknowns;
  // the instances run concurrently in one launch: report instance 0's clock
  const etd_ctx* c0 = B->inst[0];
  out->krylov_device_ms = c0->h_state->ticks_total / c0->clock_khz;
  out->krylov_sync_ms = c0->h_state->ticks_sync / c0->clock_khz;
  out->krylov_expm_ms = c0->h_state->ticks_expm / c0->clock_khz;
  out->krylov_pass_ms = c0->h_state->ticks_pass / c0->clock_khz;
  out->krylov_prologue_ms = c0->h_state->ticks_pro / c0->clock_khz;
  out->krylov_gap_ms = c0->h_state->ticks_gap / c0->clock_khz;
  out->krylov_syncs = c0->h_state->syncs;
  out->krylov_expms = c0->h_state->expm_calls;
  if (reset) {
    B->t_krylov.ms = B->t_levelset.ms = B->t_geometry.ms = 0.0;
    B->t_krylov.count = B->t_levelset.count = B->t_geometry.count = 0;
    for (etd_ctx* c : B->inst) HIP_TRY(reset_counters(c->st, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
  }
  return ETD_OK;
}

}  // extern "C"

// ------------------------------------------------- allocation-free entry
//
// phi_combination_apply_static: the context's buffers (workspace vectors,
// geometry tables, barrier flags, Krylov state, counters) all carved from
// one file-scope device array.  Its device address is taken once per device
// with hipGetSymbolAddress; host code never uses the array's name otherwise.

namespace {

constexpr int ST_TILES = ETD_STATIC_MAX_TILES;              // box tiles at most
constexpr size_t ST_LD = (size_t)ST_TILES * TILE_PTS;        // doubles per vector
constexpr int ST_GMAX = (ST_TILES + KB_TILES[KB_LARGE] - 1) / KB_TILES[KB_LARGE];   // blocks of the persistent launch at most (1024-thread build)

// Byte offsets of the carved buffers (256-byte aligned).
struct StaticLayout {
  size_t ws, cdiag, comp_bits, irr_bits, nbr, slot_tile, tile_map, tile_flag, tile_vb, band_tmp, band_list, mask,
      counters, part, flags, bar, st, tab, pre, cnt, total;
};

constexpr size_t al256(size_t x) { return (x + 255) / 256 * 256; }

constexpr StaticLayout static_layout() {
  StaticLayout L{};
  size_t o = 0;
  auto take = [&o](size_t bytes) { const size_t at = o; o = al256(o + bytes); return at; };
  L.ws = take(sizeof(double) * ST_LD * NVEC);
  L.cdiag = take(sizeof(double) * ST_LD);
  L.comp_bits = take(sizeof(uint64_t) * 4 * ST_TILES);
  L.irr_bits = take(sizeof(uint64_t) * 4 * ST_TILES);
  L.nbr = take(sizeof(int) * NBR_STRIDE * ST_TILES);
  L.slot_tile = take(sizeof(int) * ST_TILES);
  L.tile_map = take(sizeof(int) * ST_TILES);
  L.tile_flag = take(sizeof(int) * ST_TILES);
  L.tile_vb = take(sizeof(int) * ST_TILES);
  L.band_tmp = take(sizeof(int) * 2 * ST_TILES);
  L.band_list = take(sizeof(int) * LS_NLISTS * ST_TILES);
  L.mask = take(ST_LD);
  L.counters = take(sizeof(int) * NCOUNTERS);
  L.part = take(sizeof(double) * 2 * ST_GMAX * PART_STRIDE);
  L.flags = take(sizeof(unsigned) * ST_GMAX);
  L.bar = take(sizeof(BarrierDev));
  L.st = take(sizeof(KrylovStateDev));
  L.tab = take(sizeof(GeomInst));
  L.pre = take(sizeof(int) * GEOM_NPRE * 2);
  L.cnt = take(sizeof(int) * NCOUNTERS);
  L.total = o;
  return L;
}

constexpr StaticLayout SL = static_layout();
static_assert(SL.total <= ETD_STATIC_SCRATCH_BYTES, "the carved buffers exceed the static scratch array");

}  // namespace

static __device__ __align__(256) unsigned char scratch[ETD_STATIC_SCRATCH_BYTES];

namespace {

constexpr int ST_MAX_DEVICES = 64;
std::mutex g_static_mu;
void* g_static_ptr[ST_MAX_DEVICES] = {};   // device address of `scratch` per device
int g_static_grid[ST_MAX_DEVICES] = {};    // co-resident blocks of the Krylov kernel per device

// Address of this device's scratch array (device current), taken once.
int static_scratch(int dev, char** out, int* max_grid) {
  if (dev < 0 || dev >= ST_MAX_DEVICES) return ETD_ERR_NO_DEVICE;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return ETD_ERR_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return ETD_ERR_NO_DEVICE;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ETD_ERR_HIP;
    g_static_grid[dev] = krylov_max_blocks_per_cu(KB_LARGE, 2) * prop.multiProcessorCount;
    g_static_ptr[dev] = p;
  }
  *out = (char*)g_static_ptr[dev];
  *max_grid = g_static_grid[dev];
  return ETD_OK;
}

// Fresh state for a call: counters and the barrier cleared, the adaptive
// Krylov state at its defaults (a kernel, no memset).
__global__ void static_init_kernel(int* counters, BarrierDev* bar, KrylovStateDev* st, int m_min) {
  const int i = threadIdx.x;
  if (i < NCOUNTERS) counters[i] = 0;
  if (i == 0) {
    *bar = BarrierDev{};
    KrylovStateDev s{};
    for (int k = 0; k <= PMAX; ++k) {
      s.m_guess[k] = m_min;
      s.tau_frac[k] = 1.0;
    }
    *st = s;
  }
}

}  // namespace

extern "C" int phi_combination_apply_static(const etd_grid* grid, double beta, const double* rho, double t,
                                            int32_t p, const double* const* b, double* out,
                                            const etd_krylov_opts* opts, void* hip_stream) {
  if (!grid || !rho || !b || !out || p < 0 || p > PMAX || !(t >= 0.0) || !isfinite(t)) return ETD_ERR_INVALID;
  if (!(beta > 0.0) || !isfinite(beta)) return ETD_ERR_INVALID;
  for (int k = 0; k <= p; ++k)
    if (!b[k] || b[k] == out) return ETD_ERR_INVALID;
  if (grid->dim != 2 && grid->dim != 3) return ETD_ERR_INVALID;
  for (int d = 0; d < grid->dim; ++d)
    if (grid->n[d] < 5 || !(grid->hi[d] > grid->lo[d])) return ETD_ERR_INVALID;
  const double dx = (grid->hi[0] - grid->lo[0]) / (grid->n[0] - 1);
  for (int d = 1; d < grid->dim; ++d)
    if (fabs((grid->hi[d] - grid->lo[d]) / (grid->n[d] - 1) - dx) > 1e-12 * dx) return ETD_ERR_INVALID;
  etd_krylov_opts o{1e-10, 8, 64, 4, 64};
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.m_min < 1 || o.m_max > MMAX_LIMIT || o.m_min > o.m_max || o.m_step < 1 ||
      o.max_substeps < 1)
    return ETD_ERR_INVALID;
  // the box and its tiles
  etd_ctx c;
  BoxHost& bx = c.box;
  bx.dim = grid->dim;
  bx.nx = grid->n[0];
  bx.ny = grid->n[1];
  bx.nz = grid->dim == 3 ? grid->n[2] : 1;
  if (bx.dim == 2) { bx.tx = 32; bx.ty = 8; bx.tz = 1; } else { bx.tx = 16; bx.ty = 4; bx.tz = 4; }
  bx.ntx = (bx.nx + bx.tx - 1) / bx.tx;
  bx.nty = (bx.ny + bx.ty - 1) / bx.ty;
  bx.ntz = (bx.nz + bx.tz - 1) / bx.tz;
  for (int d = 0; d < 3; ++d) bx.lo[d] = d < grid->dim ? grid->lo[d] : 0.0;
  bx.dx = dx;
  if ((long)bx.ntx * bx.nty * bx.ntz > ST_TILES) return ETD_ERR_INVALID;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ETD_ERR_NO_DEVICE;
  char* base = nullptr;
  int max_grid = 0;
  int r = static_scratch(dev, &base, &max_grid);
  if (r) return r;
  // a context whose buffers are the carved pieces of the array
  c.device = dev;
  c.stream = (hipStream_t)hip_stream;
  c.grid = *grid;
  c.phys = etd_physics{beta, 0.0, 0.0, 0.0};
  c.opts = o;
  c.ntiles = bx.ntx * bx.nty * bx.ntz;
  c.nodes = (size_t)bx.nx * bx.ny * bx.nz;
  c.ld = ST_LD;
  c.ws = (double*)(base + SL.ws);
  c.cdiag = (double*)(base + SL.cdiag);
  c.comp_bits = (uint64_t*)(base + SL.comp_bits);
  c.irr_bits = (uint64_t*)(base + SL.irr_bits);
  c.nbr = (int*)(base + SL.nbr);
  c.slot_tile = (int*)(base + SL.slot_tile);
  c.tile_map = (int*)(base + SL.tile_map);
  c.tile_flag = (int*)(base + SL.tile_flag);
  c.tile_vb = (int*)(base + SL.tile_vb);
  c.band_tmp = (int*)(base + SL.band_tmp);
  c.band_list = (int*)(base + SL.band_list);
  c.mask = (uint8_t*)(base + SL.mask);
  c.counters = (int*)(base + SL.counters);
  c.part = (double*)(base + SL.part);
  c.flags = (unsigned*)(base + SL.flags);
  c.bar = (BarrierDev*)(base + SL.bar);
  c.st = (KrylovStateDev*)(base + SL.st);
  c.max_grid = max_grid < ST_GMAX ? max_grid : ST_GMAX;
  c.max_grid_kb[KB_LARGE] = c.max_grid;
  c.kb_fixed = KB_LARGE;
  // host-side mirrors on this call's stack (pageable: every copy into or
  // out of them is complete at the synchronisations below)
  int h_counters[NCOUNTERS] = {};
  GeomInst tab{};
  int h_pre[GEOM_NPRE * 2] = {};
  int h_cnt[NCOUNTERS] = {};
  c.h_counters = h_counters;
  c.gb.count = 1;
  c.gb.ncnt = NCOUNTERS;
  c.gb.h_tab = &tab;
  c.gb.d_tab = (GeomInst*)(base + SL.tab);
  c.gb.h_pre = h_pre;
  c.gb.d_pre = (int*)(base + SL.pre);
  c.gb.h_cnt = h_cnt;
  c.gb.d_cnt = (int*)(base + SL.cnt);
  tab = geom_inst(&c);
  int result = ETD_OK;
  do {
    // block prefixes: computed on the host, copied into the array
    {
      for (int q = 0; q < GEOM_NPRE; ++q) {
        const int per = geom_blocks_per(q, c.nodes, c.ntiles);
        h_pre[q * 2] = 0;
        h_pre[q * 2 + 1] = per;
        c.gb.blocks[q] = per;
      }
      if (hipMemcpyAsync(c.gb.d_pre, h_pre, sizeof(h_pre), hipMemcpyHostToDevice, c.stream) != hipSuccess) {
        result = ETD_ERR_HIP;
        break;
      }
    }
    hipLaunchKernelGGL(static_init_kernel, dim3(1), dim3(NCOUNTERS), 0, c.stream, c.counters, c.bar, c.st, o.m_min);
    if (hipGetLastError() != hipSuccess) { result = ETD_ERR_HIP; break; }
    if ((result = geometry_enqueue(&c, rho))) break;
    if (hipStreamSynchronize(c.stream) != hipSuccess) { result = ETD_ERR_HIP; break; }
    if ((result = geometry_finish(&c, h_cnt))) break;
    for (int k = 0; k <= p && !result; ++k) result = gather_to(&c, b[k], V_B0 + k);
    if (result) break;
    KrylovDev P = krylov_params(&c, JOB_PHI);
    P.p = p;
    P.t = t;
    if ((result = run_krylov(&c, P))) break;
    if ((result = scatter_from(&c, V_U, out))) break;
    result = latched_status(&c);
  } while (false);
  // nothing may still read the stack mirrors
  if (hipStreamSynchronize(c.stream) != hipSuccess && result == ETD_OK) result = ETD_ERR_HIP;
  c.h_counters = nullptr;
  return result;
}
