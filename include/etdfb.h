/*
 * libetdfb -- exponential time differencing on embedded-boundary domains
 * with a level-set free boundary, for AMD Instinct MI355X (gfx950), FP64.
 *
 * Method: S. Liu and X. Liu, "Integration factor combined with level set
 * method for reaction-diffusion systems with free boundary in high spatial
 * dimensions", arXiv 2209.15095.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays are DEVICE pointers to float64 in box layout [nz][ny][nx]
 *   (x fastest; 2D: nz = 1).  Node (i,j,k) sits at lo + (i,j,k) * h with
 *   h = (hi[0] - lo[0]) / (n[0] - 1), equal on every axis (Section 2,
 *   eq. 2.3).  The caller owns every array; the library never frees or
 *   reallocates them.  Arrays passed to one call must not overlap unless a
 *   parameter says so.
 * - The domain is where the level-set function rho < 0 (Section 4.3).
 *   Computational points are inside points whose 2d face neighbours are all
 *   inside; the other inside points are interior ghost points (Section 2).
 *   Unknowns live on computational points only: vectors are READ only there
 *   and WRITTEN as 0 at every other node.
 * - Calls are asynchronous on the context's HIP stream and return a status
 *   code (0 = ETD_OK, negative = error).  Argument errors are detected on
 *   the host and returned at once.  Errors found on the device (Krylov
 *   failure, non-finite data, domain at the box edge, barrier time-out) are
 *   latched in the context and returned by etd_ctx_sync() and by the next
 *   call that synchronises (any call given a non-NULL stats pointer).
 * - One context serves one stream at a time; calls on one context must not
 *   overlap.  Contexts are independent of each other.
 */
#ifndef ETDFB_H
#define ETDFB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  ETD_OK = 0,
  ETD_ERR_INVALID = -1,      /* bad argument (host check) */
  ETD_ERR_HIP = -2,          /* a HIP runtime call failed */
  ETD_ERR_NO_DEVICE = -3,    /* no gfx950 device visible */
  ETD_ERR_KRYLOV = -4,       /* Krylov method did not reach the tolerance */
  ETD_ERR_NONFINITE = -5,    /* NaN/Inf met in a reduction */
  ETD_ERR_DOMAIN = -6,       /* computational point within 2 layers of the box edge */
  ETD_ERR_BARRIER = -7,      /* grid barrier timed out (kernel drained and exited) */
  ETD_ERR_NO_GEOMETRY = -8,  /* no geometry built on this context yet */
  ETD_ERR_FRONT = -9         /* boundary beyond the reach of the level-set sweeps (front speed, reads) */
};

/* ETD1 (Section 3.1), ETD2RK, ETD3RK and ETD4RK (Section 3.2; the phi_3 of
 * the paper's ETD3RK and ETD4RK formulas is 2 phi_3 in the standard
 * normalisation phi_k(0) = 1/k! used by phi_combination_apply).  The
 * _SIMUL variants compute the same schemes with the simultaneous output of
 * Section 3.3 (as in phipm_simul_iom2): the ODE y' = A y + F_n, y(0) = U_n
 * is integrated once over h, its value at h/2 (stage a, from the Krylov
 * basis of the substep that holds h/2) and at h (the phi_0, phi_1 part of
 * the last stage) come from that one integration, and the other stages are
 * combinations with b_0 = 0 added to those values. */
enum {
  ETD_SCHEME_ETD1 = 1,
  ETD_SCHEME_ETD2RK = 2,
  ETD_SCHEME_ETD3RK = 3,
  ETD_SCHEME_ETD4RK = 4,
  ETD_SCHEME_ETD3RK_SIMUL = 5,
  ETD_SCHEME_ETD4RK_SIMUL = 6
};

/* Box grid: dim 2 or 3, n[d] nodes on [lo[d], hi[d]] per axis, equal spacing. */
typedef struct {
  int32_t dim;
  int32_t n[3];
  double lo[3];
  double hi[3];
} etd_grid;

/* u_t = div(beta grad u) + u (a - b u) in the domain; boundary speed
 * mu |grad u| along the outward normal (Section 1, eq. 1.1; Section 4.3). */
typedef struct {
  double beta;
  double a;
  double b;
  double mu;
} etd_physics;

/* Multi-species systems (Section 3, eq. 3.1 with u in R^m): m <= 4
 * components share the diffusion operator and react pointwise,
 * f_s(u) = u_s (a[s] - sum_j b[s*ETD_MAX_SPECIES + j] u_j) (the logistic
 * reaction of etd_physics for m = 1). */
#define ETD_MAX_SPECIES 4
typedef struct {
  int32_t m;
  double a[ETD_MAX_SPECIES];
  double b[ETD_MAX_SPECIES * ETD_MAX_SPECIES];
} etd_species;

/* Adaptive Krylov options.  tol: local error per unit time relative to the
 * solution norm (the paper's experiments use tolerance-driven adaptivity,
 * Section 3.3).  m_min <= m <= m_max <= 64 Krylov dimensions, grown in steps
 * of m_step; at most max_substeps time substeps per combination. */
typedef struct {
  double tol;
  int32_t m_min;
  int32_t m_max;
  int32_t m_step;
  int32_t max_substeps;
} etd_krylov_opts;

/* Statistics of the last device job of a context. */
typedef struct {
  int32_t substeps;
  int32_t rejected;
  int32_t matvecs;
  int32_t m_last;
  int32_t expms;
  int32_t n_active_tiles;
  int32_t n_unknowns;
  int32_t status;
  double err_est;
  double t_done;
} etd_stats;

/* Accumulated device timings (milliseconds, HIP events on the context's
 * stream) and algorithmic traffic, for measurement. */
typedef struct {
  double krylov_ms;          /* persistent phi-combination / ETD launches */
  double levelset_ms;        /* level-set sweep sequences */
  double geometry_ms;        /* geometry builds */
  double alg_bytes;          /* algorithmic HBM bytes of the Krylov launches */
  int32_t krylov_launches;
  int32_t levelset_calls;
  int32_t geometry_calls;
  int32_t n_unknowns;        /* computational points of the current geometry */
  /* inside the Krylov launches, from the device clock of block 0: whole
   * launches, grid synchronisations (waiting included), small exponentials,
   * passes over the tiles (from the start of a tile loop until every wave
   * of the block has finished it and the block has reduced its partials),
   * launch prologue (tile metadata into LDS), and from the end of each grid
   * synchronisation to the start of the next pass or exponential
   * (krylov_gap_ms); the rest is the control that follows passes and
   * exponentials without a synchronisation */
  double krylov_device_ms;
  double krylov_sync_ms;
  double krylov_expm_ms;
  double krylov_pass_ms;
  double krylov_prologue_ms;
  int32_t krylov_syncs;
  int32_t krylov_expms;
  double krylov_gap_ms;
} etd_profile;

typedef struct etd_ctx etd_ctx;

/* Create a context for one grid.  hip_stream: a hipStream_t (NULL = the
 * default stream).  opts may be NULL (tol 1e-10, m 8..64 step 4, 64
 * substeps).  Allocates all device workspaces for the worst case (every
 * tile of the box active).  *out receives the context; returns ETD_OK,
 * ETD_ERR_INVALID, ETD_ERR_NO_DEVICE or ETD_ERR_HIP. */
int etd_ctx_create(const etd_grid* grid, const etd_physics* phys, const etd_krylov_opts* opts,
                   void* hip_stream, etd_ctx** out);

/* Create a context for m species (etd_species; Section 3, eq. 3.1):
 * phys gives beta (shared by the species) and mu; its a and b are not used.
 * The discretised system is C = I_m (x) A, one Krylov space for all
 * species (its inner products sum over them).  Workspaces are m times those
 * of etd_ctx_create.  Such a context serves etd_geometry_build (frozen
 * domains), etd_step_species, sync, stats and profiling; every other call
 * returns ETD_ERR_INVALID.  ETD_ERR_INVALID for m outside 1..4 or
 * non-finite coefficients. */
int etd_ctx_create_species(const etd_grid* grid, const etd_physics* phys, const etd_species* species,
                           const etd_krylov_opts* opts, void* hip_stream, etd_ctx** out);

/* One step of size h of the m-species system u_t = A u + f(u) (ETD1,
 * ETD2RK, ETD3RK or ETD4RK as in etd_step, Section 3, every stage one
 * combination on all species) on the frozen domain of the last geometry
 * build.  u: host array of m device box arrays (distinct), updated in
 * place. */
int etd_step_species(etd_ctx* ctx, int32_t scheme, double h, double* const* u, etd_stats* stats);

/* Free a context and its workspaces (synchronises its stream first). */
int etd_ctx_destroy(etd_ctx* ctx);

/* Switch the stream later calls are enqueued on. */
int etd_ctx_set_stream(etd_ctx* ctx, void* hip_stream);

/* Replace beta (the operator is beta times the beta = 1 operator, Section 2
 * with constant beta); takes effect for later calls. */
int etd_ctx_set_beta(etd_ctx* ctx, double beta);

/* Classify the nodes of rho < 0 and build the operator coefficients
 * (Section 2, Cases 1-3; eq. 2.4 and eqs. 2.5-2.6).  rho: device array of
 * the box, read only.  Synchronises once to size the persistent launch.
 * Returns ETD_ERR_DOMAIN when a computational point lies in the two outer
 * box layers. */
int etd_geometry_build(etd_ctx* ctx, const double* rho);

/* Variable beta(x) (Section 2, eq. 2.4 with beta at the face midpoints; the
 * Case 2/3 closures as for etd_geometry_build): classify rho and build the
 * operator with face coefficients, and the boundary taps of non-homogeneous
 * Dirichlet data.  beta_face: host array of dim device pointers; entry d is
 * a box array whose value at node x is beta(x + h/2 e_d) (the midpoint of
 * the face between the node and its +e_d neighbour; read only at faces of
 * computational points).  Later calls use this operator (A is no longer
 * beta times a fixed matrix: etd_ctx_set_beta and etd_adjoint_step return
 * ETD_ERR_INVALID) until the next etd_geometry_build; free-boundary calls
 * (rho != NULL) return ETD_ERR_INVALID meanwhile.  Synchronises.  Device
 * buffers for the face coefficients and taps are allocated on the first
 * call.  Errors as etd_geometry_build. */
int etd_geometry_build_var(etd_ctx* ctx, const double* rho, const double* const* beta_face);

/* Boundary points of the Dirichlet data in the discretisation of the last
 * etd_geometry_build_var (Section 2: the interface crossing of each Case 2
 * face, the closest boundary points x_G1, x_G2 of each Case 3 face), in the
 * order etd_forcing_assemble reads their values.  *count receives their
 * number; points (host, may be NULL) receives dim coordinates per point
 * when capacity >= *count (else ETD_ERR_INVALID).  ETD_ERR_NO_GEOMETRY
 * without a variable-beta geometry. */
int etd_boundary_taps(etd_ctx* ctx, int32_t capacity, double* points, int32_t* count);

/* The forcing of u_t = A u + G: out = src + g, where g is the boundary term
 * of the Dirichlet data (Section 2, Cases 2 and 3: each tap's weight times
 * ub at that tap), at the computational points; 0 elsewhere.  ub: device
 * array of the data at the points of etd_boundary_taps (may be NULL when
 * there are none); src: device box array or NULL (0); out: device box
 * array, must not alias src or ub.  Asynchronous. */
int etd_forcing_assemble(etd_ctx* ctx, const double* ub, const double* src, double* out);

/* out = A v: the embedded-boundary discretisation of div(beta grad .) of
 * the last etd_geometry_build (Section 2: eq. 2.4 and the Case 2/3 ghost
 * closures with homogeneous boundary data).  v, out: device box arrays
 * (v read at computational points, out written everywhere, no aliasing). */
int etd_operator_apply(etd_ctx* ctx, const double* v, double* out);

/* out = sum_{k=0}^{p} phi_k(t A) b_k  (eq. 3.7 with A -> tA; standard
 * phi_k: phi_0 = exp, phi_k(z) = (phi_{k-1}(z) - 1/(k-1)!)/z), A the
 * operator of the last etd_geometry_build.  0 <= p <= 3, t >= 0.
 * b: host array of p+1 device pointers (box layout, read at computational
 * points).  out: device array (box), written everywhere; must not alias any
 * b_k.  stats: NULL, or receives the statistics (synchronises). */
int phi_combination_apply(etd_ctx* ctx, double t, int32_t p, const double* const* b, double* out,
                          etd_stats* stats);

/* The combination at two times from one integration (Section 3.3, the
 * simultaneous output of phipm_simul_iom2): out as phi_combination_apply
 * at t, and out_mid = y(t_mid) of the same ODE y' = A y + sum_k
 * s^{k-1}/(k-1)! b_k / t^k, y(0) = b_0, i.e.
 * sum_k phi_k(t_mid A) (t_mid/t)^k b_k, for 0 < t_mid <= t.  out_mid comes
 * from the Krylov basis of the substep that holds t_mid (one more small
 * exponential and one combine pass, its error estimate held to the same
 * tolerance).  out, out_mid: distinct device box arrays, not aliasing any
 * b_k. */
int phi_combination_apply_multi(etd_ctx* ctx, double t, int32_t p, const double* const* b, double t_mid,
                                double* out_mid, double* out, etd_stats* stats);

/* Steps 1 and 2a of the free-boundary algorithm (Section 4.3): extend u
 * from the computational points of rho by quadratic normal extrapolation,
 * Stefan speed mu |grad u| extended off the interface, HJ-WENO5/TVD-RK3
 * advection of rho over dt, reinitialisation if reinit != 0, then u is
 * restricted to the computational points of the new rho.  rho and u are
 * device box arrays updated in place.  Rebuilds the geometry for the new
 * rho.  The extrapolation serves fronts that move at most one node per
 * step: when the maximum extended speed V gives V * dt > h, nothing is
 * changed and ETD_ERR_FRONT is returned (take smaller steps). */
int levelset_advance(etd_ctx* ctx, double* rho, double* u, double dt, int32_t reinit);

/* One time step of size h of u_t = A u + f(u) (Section 3: ETD1, ETD2RK,
 * ETD3RK or ETD4RK; 1, 2, 3 or 4 phi-combinations in one persistent launch).
 * rho == NULL: frozen domain (geometry of the last build).  rho != NULL:
 * free boundary, levelset_advance(ctx, rho, u, h, reinit) first, then the
 * ETD step on the new domain.  u: device box array, updated in place. */
int etd_step(etd_ctx* ctx, int32_t scheme, double h, double* u, double* rho, int32_t reinit,
             etd_stats* stats);

/* One step of size h of u_t = A u + f(u) + G(t) on the frozen domain of the
 * last geometry build (Section 3 schemes as etd_step; G is the forcing of
 * a source and Dirichlet data, e.g. from etd_forcing_assemble, as in the
 * accuracy test of Section 4.2).  g: host array of 3 device box arrays,
 * G(t_n), G(t_n + h/2), G(t_n + h), read at computational points; ETD1
 * reads g[0], ETD2RK g[0] and g[2], ETD3RK and ETD4RK all three (unread
 * entries may be NULL).  u: device box array, updated in place; must not
 * alias a g entry read.  ETD_ERR_INVALID for a bad scheme, h, or a NULL
 * entry that is read; ETD_ERR_NO_GEOMETRY before any build. */
int etd_step_forced(etd_ctx* ctx, int32_t scheme, double h, double* u, const double* const* g, etd_stats* stats);

/* One ETD2 multistep step (Section 3.1, the ETD2 formula, eq. 3.6 with s = 2):
 * U_{n+1} = phi_0(hA) U_n + h phi_1(hA) F_n + h phi_2(hA) (F_n - F_{n-1}),
 * F_n = f(U_n), one phi-combination in one persistent launch.
 * f_prev: device box array owned by the caller.  On entry (first == 0) it
 * holds F_{n-1} = f(U_{n-1}) at the computational points of the domain
 * that U_n lives on (what the previous call left there); on return it holds
 * F_n at the computational points of the domain of this step and 0
 * elsewhere.  first != 0: f_prev is not read and the step is one ETD2RK step
 * (Section 3.2), which starts the two-step recursion.  rho == NULL: frozen
 * domain.  rho != NULL: free boundary as in etd_step; F_{n-1} is carried to
 * the points that join the domain by the quadratic normal extrapolation
 * from the old computational points that carries u (Section 4.3, Step 2,
 * the same sweeps, in the same launches as u's within the level-set step
 * of levelset_advance(ctx, rho, u, h, reinit); ETD_ERR_FRONT as there, with
 * rho, u and f_prev unchanged).  u: device box array, updated in place.  ETD_ERR_INVALID (nothing done) for a NULL ctx, u or
 * f_prev, f_prev aliasing u or rho, or h negative or not finite;
 * ETD_ERR_NO_GEOMETRY for a frozen step before any geometry build. */
int etd_multistep_step(etd_ctx* ctx, double h, double* u, double* f_prev, int32_t first, double* rho,
                       int32_t reinit, etd_stats* stats);

/* Discrete adjoint of one ETD2RK step (Section 3.2) on the frozen domain of
 * the last etd_geometry_build, for the loss gradient of a step-by-step
 * backward sweep.  A is symmetric (Section 2) and equals beta A_1 for the
 * constant beta.  u_n: the forward state U_n (device box array);
 * gbar_np1: dL/dU_{n+1} (device box array); both read at computational
 * points.  gbar_n: receives dL/dU_n (device box array, written everywhere;
 * may be the same array as gbar_np1, not u_n).  dL_dbeta: device scalar to
 * which this step's dL/dbeta is added (stream-ordered).  scheme must be
 * ETD_SCHEME_ETD2RK.  Six phi-combinations in one persistent launch. */
int etd_adjoint_step(etd_ctx* ctx, int32_t scheme, double h, const double* u_n, const double* gbar_np1,
                     double* gbar_n, double* dL_dbeta);

/* Wait for the context's stream; return the first latched device error
 * (and clear it), or ETD_OK. */
int etd_ctx_sync(etd_ctx* ctx);

/* Statistics of the last job (synchronises). */
int etd_ctx_stats(etd_ctx* ctx, etd_stats* stats);

/* Enable (1) or disable (0) event timing of the launches of a context. */
int etd_ctx_profile_enable(etd_ctx* ctx, int32_t enable);

/* Synchronise and read the accumulated timings; reset != 0 clears them. */
int etd_ctx_profile_read(etd_ctx* ctx, etd_profile* out, int32_t reset);

/* ------------------------------------------------------------------ batch
 * Many independent instances (each its own grid, domain, physics) advanced
 * together: the free-boundary sweeps of all instances share one host
 * synchronisation, and every ETD step of the batch is one persistent launch
 * in which each instance is worked on by its own group of blocks, sized by
 * its number of active tiles, synchronising only within the group.  The
 * method per instance is exactly that of etd_step (Sections 3 and 4.3). */
typedef struct etd_batch etd_batch;

/* count instances; grids[i], phys[i] describe instance i (all grids of one
 * dimension); opts as for etd_ctx_create (may be NULL, shared by all).
 * Workspaces per instance as for etd_ctx_create. */
int etd_batch_create(int32_t count, const etd_grid* grids, const etd_physics* phys,
                     const etd_krylov_opts* opts, void* hip_stream, etd_batch** out);
int etd_batch_destroy(etd_batch* batch);
int etd_batch_set_stream(etd_batch* batch, void* hip_stream);

/* At most max_blocks blocks per instance in the batched launch (0 = as many
 * as its active tiles can use); 1 makes every instance a single block. */
int etd_batch_set_group_limit(etd_batch* batch, int32_t max_blocks);

/* Tile schedule of the batched Krylov launch: an instance's Lanczos passes
 * stage each tile and its face halo in LDS when it has at least min_tiles
 * active tiles and its blocks take several loop trips (0: whenever they do;
 * INT32_MAX: never; -1: the library's default, 2048).  Results agree with
 * the unstaged passes to rounding (the same arithmetic per point). */
int etd_batch_set_stage_min(etd_batch* batch, int32_t min_tiles);

/* etd_geometry_build for every instance; rho: host array of count device
 * pointers.  One synchronisation for the whole batch.  ETD_ERR_DOMAIN if any
 * instance has a computational point in its two outer box layers. */
int etd_batch_geometry_build(etd_batch* batch, const double* const* rho);

/* etd_step for every instance with the same scheme, h and reinit flag.
 * u: host array of count device pointers (box arrays, updated in place).
 * rho: NULL (frozen domains) or host array of count device pointers.
 * stats: NULL, or an array of count etd_stats (synchronises). */
int etd_batch_step(etd_batch* batch, int32_t scheme, double h, double* const* u, double* const* rho,
                   int32_t reinit, etd_stats* stats);

/* etd_multistep_step for every instance with the same h, first and reinit
 * flags (Section 3.1, the ETD2 formula; Section 4.3 on moving domains): one
 * batched persistent launch of one ETD2 multistep step per instance.
 * u, f_prev: host arrays of count device pointers (box arrays; f_prev[i]
 * holds F(U_{n-1}) of instance i on entry unless first, F(U_n) on return;
 * f_prev[i] must not alias u[i] or rho[i]).  rho: NULL (frozen domains) or
 * host array of count device pointers.  stats: NULL, or an array of count
 * etd_stats (synchronises). */
int etd_batch_multistep_step(etd_batch* batch, double h, double* const* u, double* const* f_prev, int32_t first,
                             double* const* rho, int32_t reinit, etd_stats* stats);

/* Wait for the stream; first latched device error over the instances (all
 * cleared), or ETD_OK. */
int etd_batch_sync(etd_batch* batch);

/* Statistics of instance i's last job (synchronises). */
int etd_batch_stats(etd_batch* batch, int32_t i, etd_stats* stats);

/* Frozen-domain steps replayed from a HIP graph: nsteps etd_batch_step
 * calls with rho = NULL, each one graph launch (batched gather, the batched
 * persistent Krylov launch, batched scatter) with no host work between
 * steps.  The graph is recorded on the first call and kept while scheme, h,
 * the u pointers, the geometry and the group limit stay the same (any change
 * records it again).  Its parameters live in device buffers of the batch,
 * so eager calls in between do not alter it.  Results are those of
 * etd_batch_step with the same group limit (the same kernels and launch
 * shape).  The Krylov launch in the graph is an ordinary kernel node: its
 * blocks (at most the co-resident capacity) must all be resident, which
 * holds when no other work shares the GPU; otherwise the group barrier's
 * bounded wait ends the step with ETD_ERR_BARRIER (reported by
 * etd_batch_sync) rather than hanging.  Asynchronous; ETD_ERR_NO_GEOMETRY
 * before the first geometry build; ETD_ERR_INVALID if the batch needs more
 * than one launch per step (more instances than co-resident blocks). */
int etd_batch_graph_steps(etd_batch* batch, int32_t scheme, double h, double* const* u, int32_t nsteps);

/* nsteps free-boundary steps of every instance (the method of etd_batch_step
 * with rho: level set, Section 4.3; geometry, Section 2; the ETD step,
 * Section 3), each one replay of a recorded HIP graph with no host work
 * between steps.  Step k (0-based) is the global step step0 + k; it
 * reinitialises rho when reinit_every > 0 and (step0 + k + 1) is a multiple
 * of reinit_every (the schedule of eager steps with reinit = ((m + 1) %
 * reinit_every == 0)).  Launch sizes are found on the device: every
 * level-set launch loops over the tile lists that the step's geometry build
 * left in device memory, the most advection substeps the front guard allows
 * (4) are launched (each instance skips those beyond its own count), and
 * the Krylov block
 * schedule is the one of the active tiles when the graphs are recorded
 * (kept for later steps; blocks loop over any number of active tiles).
 * Two graphs (without and with the reinitialisation) are recorded on the
 * first call and kept while scheme, h, the u and rho pointers, the group
 * limit and the stage threshold stay the same.  Results are those of eager
 * steps up to the order of the Krylov reductions (the block schedule).
 * Errors are latched per instance and reported by etd_batch_sync; unlike
 * etd_batch_step, a step whose front would move farther than the guard of
 * the eager steps allows is not refused but latches ETD_ERR_FRONT, and the
 * instance's arrays are undefined from that step on.  The Krylov launch is
 * an ordinary kernel node (see etd_batch_graph_steps).  Asynchronous;
 * ETD_ERR_INVALID if the batch needs more than one launch per step or
 * u[i] == rho[i]. */
int etd_batch_graph_free_steps(etd_batch* batch, int32_t scheme, double h, double* const* u, double* const* rho,
                               int32_t reinit_every, int32_t step0, int32_t nsteps);

/* Autotuner of the Krylov block and tile schedule: times the batched
 * persistent launch of one frozen-domain step (scheme, h, the current u of
 * every instance) for the ETD_AUTOTUNE_CANDIDATES pairs of a group limit
 * (1, 2, 4, 8, 16, 0 = unlimited; see etd_batch_set_group_limit) and a
 * stage threshold (0, 2048, INT32_MAX; see etd_batch_set_stage_min), limit
 * major, trials timed runs each after one untimed run, and keeps the
 * fastest pair.  The Krylov adaptive state of every instance and the u
 * arrays are left as they were.  limit_out, stage_out (nullable): the
 * chosen pair; ms_out (nullable, ETD_AUTOTUNE_CANDIDATES doubles): mean ms
 * per launch of each candidate in the order above.  Synchronises. */
#define ETD_AUTOTUNE_CANDIDATES 18
int etd_batch_autotune(etd_batch* batch, int32_t scheme, double h, double* const* u, int32_t trials,
                       int32_t* limit_out, int32_t* stage_out, double* ms_out);

/* Event timing of the batch launches; profile_read sums the algorithmic
 * bytes and reports the unknowns over all instances. */
int etd_batch_profile_enable(etd_batch* batch, int32_t enable);
int etd_batch_profile_read(etd_batch* batch, etd_profile* out, int32_t reset);

/* ------------------------------------------------ allocation-free entry
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * phi_combination_apply without a context.  out = sum_{k=0}^{p} phi_k(t A) b_k
 * for the operator of the domain rho < 0 on `grid` with the constant beta
 * (the same kernels and arguments as etd_geometry_build followed by
 * phi_combination_apply; opts may be NULL for the defaults).  Every buffer
 * the kernels use lives in one static device array of
 * ETD_STATIC_SCRATCH_BYTES per GPU, held until the process ends; grids of at
 * most ETD_STATIC_MAX_TILES tiles (2D 32 x 8, 3D 16 x 4 x 4 nodes each, e.g.
 * 128 x 128 or 32 x 32 x 16 nodes) fit, larger ones return ETD_ERR_INVALID
 * before any device work.  Calls no allocating routine; the caller passes
 * inputs and outputs (device box arrays as for phi_combination_apply).
 * Synchronises the stream (twice: after the geometry, and at the end) and
 * returns the first device error of the call.  All calls on one GPU share
 * its array: calls that overlap on one GPU (several host threads or
 * streams) race and must not be made. */
#define ETD_STATIC_MAX_TILES 64
#define ETD_STATIC_SCRATCH_BYTES (12u << 20)
int phi_combination_apply_static(const etd_grid* grid, double beta, const double* rho, double t, int32_t p,
                                 const double* const* b, double* out, const etd_krylov_opts* opts,
                                 void* hip_stream);

/* Human-readable name of a status code (static string). */
const char* etd_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* ETDFB_H */
