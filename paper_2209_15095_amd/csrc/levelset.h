// Level-set sweeps of the free-boundary step (Section 4.3 of the paper,
// Algorithm Steps 1-2): host interface.
//
// The sweeps run on bands of tiles (the tile layout of the operator: 2D
// 32x8, 3D 16x4x4), built with the geometry from two L1 (Manhattan) tile
// distances: from the tiles holding a computational point (Dc) and from the
// tiles holding a node with |rho| < h (Dv); the distance between two tiles
// is a lower bound of the node distance between them.  A Jacobi sweep
// changes a node only where a face neighbour or its source is nonzero, so
// after s sweeps u_nn is exactly 0 beyond s nodes of the computational
// points, u_n beyond 25 + s, and the extended speed beyond s nodes of the
// |rho| < h nodes: those sweeps process only the tiles within that distance
// and give the whole-box values everywhere (the arrays are 0 elsewhere).
// The last stage, u, is kept exact where it is read (see the lists below).
// The advection changes rho only where the speed is nonzero and reads its
// WENO stencil 3 nodes further; the reinitialisation acts on a narrow band.
//
// One launch per sweep serves a whole batch: virtual block b works on tile
// b - off[i] of the list of instance i, off[] being the prefix sums of the
// list sizes; a launch's blocks loop over the virtual blocks of its row (the
// row total is read on the device), so a launch needs no size from the host.
#pragma once
#include <hip/hip_runtime.h>

#include "launch.h"

namespace etdfb {

// Iteration counts and pseudo-time steps of the sweeps (readings of the
// paper's unspecified parameters; identical in the CPU oracle).
constexpr int ASLAM_ITERS = 25;
// Largest front displacement per step (nodes) the extrapolation serves: with
// ASLAM_ITERS sweeps per stage it has converged to truncation error at every
// point that joins the domain when the boundary moves at most this far.  A
// step with max V * dt > LS_MAX_FRONT_NODES * h is refused on the host
// before rho or u change.
constexpr int LS_MAX_FRONT_NODES = 2;
// Advection substeps: max(1, ceil(max V dt / (h/2))), at most this many
// within the guard (graph replays launch this many and skip the rest on the
// device).
constexpr int LS_MAX_SUBSTEPS = 2 * LS_MAX_FRONT_NODES;
constexpr int VEL_ITERS = 20;
constexpr int REINIT_ITERS = 10;
// Narrow band of the reinitialisation (units of h): nodes with
// |rho_0| < REINIT_BAND h are updated, the others keep rho_0 in every RK
// stage.  The sweeps run on list R, which must hold every band node and the
// 3-node WENO reach around it (checked on the device at each
// reinitialisation, else ST_FRONT).
constexpr int REINIT_BAND = 12;
// Tile lists, built with the geometry: SC = tiles with Dc <= LS_C_MAX sorted
// by Dc, SV = tiles with Dv <= LS_V_MAX sorted by Dv (so the tiles within a
// radius r are a prefix, of cumulative count ncum_c[r] / ncum_v[r]), and
// U = SC or SV in any order.  A sweep of an extension stage takes the
// prefix its cone needs: the stages that grow from a known set (u_nn,
// u_n, the speed) process only the tiles their values can reach after that
// sweep (the arrays are 0 beyond, exactly as over the whole box); the last
// stage (u) is needed only where it is read (the |rho| < h band and the
// points that join the domain, within LS_READ_REACH nodes of the
// computational points), so sweep s processes the tiles within
// LS_READ_REACH + ASLAM_ITERS - s of them, and its values there equal the
// whole-box ones.  An L1 distance to the computational points (dilated one
// node per sweep of the u_nn stage, whose lists grow the same way) lets the
// reading kernels check that every value they read lies in that region
// (else ST_FRONT).  The reach covers the reads of the free-boundary
// workloads with margin (at most 13 nodes, where detached pieces of a noisy
// 3D domain form).
constexpr int LS_READ_REACH = 20;
constexpr int LS_C_MAX = 2 * ASLAM_ITERS + 1;   // the u_n stage's reach
constexpr int LS_V_MAX = VEL_ITERS + 4;         // the speed's reach plus the WENO stencil
enum LsList { LS_SC = 0, LS_SV = 1, LS_U = 2, LS_NLISTS = 3 };
// Launch rows: the prefix of SC within radius r, of SV within r, list U, the whole box.
enum LsRow {
  LS_ROW_C = 0,
  LS_ROW_V = LS_ROW_C + LS_C_MAX + 1,
  LS_ROW_U = LS_ROW_V + LS_V_MAX + 1,
  LS_ROW_FULL = LS_ROW_U + 1,
  LS_NROWS = LS_ROW_FULL + 1
};
constexpr int LS_DIST_CAP = 1000;   // distances are capped here (beyond every radius)
// geometry counters holding the cumulative list counts
constexpr int LS_CNT_C = 16;                          // ncum_c[0..LS_C_MAX]
constexpr int LS_CNT_V = LS_CNT_C + LS_C_MAX + 1;     // ncum_v[0..LS_V_MAX]
constexpr int LS_CNT_U = LS_CNT_V + LS_V_MAX + 1;     // size of U
constexpr int LS_NCOUNTERS = LS_CNT_U + 1;
// The maximum of the extended speed is gathered over this many slots per
// instance (one device-scope atomic per tile, spread over the slots by
// block, so that thousands of tiles do not queue on one address), then
// folded into the instance's maximum by one small launch; for short speed
// lists (below LS_VMAX_SLOT_MIN tiles in every instance) the atomics go to
// the maximum directly.
constexpr int LS_VMAX_SLOTS = 64;
// Below this many tiles in every instance's speed list the atomics go to
// the maximum itself (no queue to speak of, and no fold launch).
constexpr int LS_VMAX_SLOT_MIN = 512;

// Box-sized scratch arrays of one instance.  Between passes the extension
// arrays hold 0 and the distance 255 at every node (the whole-box values the
// sweeps on lists rely on): the restriction that ends a pass clears the
// tiles of list U, the only ones the pass writes.  A pass that does not
// reach its restriction (an error on the host between levelset_begin and
// levelset_end) leaves the scratch dirty, and the next pass clears the
// whole box first.
struct LevelsetScratch {
  size_t nodes = 0;
  double* buf = nullptr;      // 16 box arrays of doubles
  uint8_t* known = nullptr;   // bit 0: K0, bit 1: K1, bit 2: K2, bit 3: speed band, bit 4: reinit band
  uint8_t* dist = nullptr;    // L1 distance to the computational points, capped (LS_READ_REACH + 1 beyond)
  bool dirty = true;          // host flag: some node outside its list U may hold a nonzero value
};

// One instance as the kernels see it (device copy in LevelsetBatch).
struct LsInst {
  int dim, nx, ny, nz;
  int ntx, nty, ntz;
  int ncum_c[LS_C_MAX + 1];   // tiles of SC within each radius
  int ncum_v[LS_V_MAX + 1];   // tiles of SV within each radius
  int nu;                     // tiles of U
  double h, mu;
  double* rho;                // user arrays (updated in place)
  double* u;
  double* buf;                // LevelsetScratch::buf
  size_t nodes;
  uint8_t* known;
  const int* band;            // lists SC, SV, U, each a block of ntx*nty*ntz entries
  uint8_t* dist;              // LevelsetScratch::dist
  const int* tdist;           // packed tile distances of the lists (high 16 bits: Dv)
  int rr;                     // radius of list R (Dv <= rr)
  int* status;                // latched device error of the instance
  const int* cnt;             // the instance's geometry counters (list sizes, on the device)
  double* vmax;               // set by levelset_begin
  double* vslot;              // LS_VMAX_SLOTS partial maxima (0 between passes)
  int dirty;                  // set by levelset_begin (and levelset_upload): clear the whole box first
  bool* host_dirty;           // LevelsetScratch::dirty (host address, never read on the device)
  // A second box field extended with u in the same launches, or null:
  // F(U_{n-1}) of ETD2 multistep, known on the same computational points;
  // replaced by its extension within the reach of those points, 0 beyond.
  double* f;
};

// Instance table and launch offsets of a batch of `count` instances.
struct LevelsetBatch {
  int count = 0;
  int dim = 2;
  LsInst* d_inst = nullptr;   // count
  LsInst* h_inst = nullptr;   // pinned, count (caller fills before levelset_begin)
  int* d_off = nullptr;       // LS_NROWS * (count + 1): block offsets of each launch row
  int* h_off = nullptr;       // pinned
  double* d_vmax = nullptr;   // count maximum speeds
  double* d_vslot = nullptr;  // count * LS_VMAX_SLOTS partial maxima
  double* h_vmax = nullptr;   // pinned mirror
  int total[LS_NROWS] = {};
  double dt = 0.0;
  int reinit = 0;
  int uext = 0;               // scratch array holding u_ext after levelset_begin
  int nf = 1;                 // fields extended: 2 when some instance has f
  int vmax_tiles = 0;         // largest speed list of an instance (tiles of the last speed sweep)
  bool any_dirty = false;     // some instance's scratch is cleared over the whole box first
  // Device-sized mode (for graph capture): the launch rows come from the
  // geometry counters on the device, every launch has a fixed grid, the
  // front guard is checked on the device (ST_FRONT latched, the step goes
  // on), LS_MAX_SUBSTEPS advection substeps are launched, and nothing is
  // copied to or from the host.  The instance table must be on the device
  // (levelset_upload) before; the grids are sized from the lists then.
  bool device_sized = false;
};

hipError_t levelset_alloc(LevelsetScratch& s, size_t nodes);
void levelset_free(LevelsetScratch& s);
hipError_t levelset_batch_alloc(LevelsetBatch& b, int count, int dim);
void levelset_batch_free(LevelsetBatch& b);

// Steps 1 + 2a for every instance of b (h_inst filled by the caller; rho and
// u, and f where given, updated in place): levelset_begin enqueues
// everything up to the maximum speeds and their asynchronous copy to pinned
// memory; after the caller has synchronised the stream, levelset_end
// enqueues the advection substeps, the reinitialisation (if reinit) and the
// restriction of u (and of f).  Nothing the caller passed changes before
// levelset_end.
hipError_t levelset_begin(LevelsetBatch& b, double dt, int reinit, hipStream_t stream);
// Device-sized mode: copy the instance table (h_inst, with dirty flags
// taken as for a pass) to the device and clear every dirty scratch; the
// caller synchronises the stream before capturing levelset_begin/end.
hipError_t levelset_upload(LevelsetBatch& b, hipStream_t stream);
hipError_t levelset_end(LevelsetBatch& b, hipStream_t stream);

}  // namespace etdfb
