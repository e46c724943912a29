// Level-set sweeps of the free-boundary step (Section 4.3 of the paper,
// Algorithm Steps 1-2): host interface.
//
// The sweeps run on bands of tiles (the tile layout of the operator: 2D
// 32x8, 3D 16x4x4), built with the geometry from two L1 (Manhattan) tile
// distances: from the tiles holding a computational point (Dc) and from the
// tiles holding a node with |rho| < h (Dv); the distance between two tiles
// is a lower bound of the node distance between them.  A Jacobi sweep
// changes a node only where a face neighbour or its source is nonzero, so
// the extrapolated u_nn, u_n, u are exactly 0 beyond 25, 50 and 75 nodes of
// the computational points and the extended speed beyond 20 nodes of the
// |rho| < h nodes: each stage sweeps only the tiles within that distance
// plus one, and gives the whole-box values everywhere (the arrays are 0
// elsewhere).  The advection changes rho only where the speed is nonzero and
// reads its WENO stencil 3 nodes further.  Reinitialisation and the final
// restriction of u cover the whole box.
//
// One launch per sweep serves a whole batch: block b works on tile
// b - off[i] of the list of instance i, off[] being the prefix sums of the
// list sizes.
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
constexpr int VEL_ITERS = 20;
constexpr int REINIT_ITERS = 10;
// Narrow band of the reinitialisation (units of h): nodes with
// |rho_0| < REINIT_BAND h are updated, the others keep rho_0 in every RK
// stage.  The sweeps run on list R, which must hold every band node and the
// 3-node WENO reach around it (checked on the device at each
// reinitialisation, else ST_FRONT).
constexpr int REINIT_BAND = 12;
// Tile lists of a sweep (radii in nodes, see above).
enum LsList {
  LS_A1 = 0,    // Dc <= ASLAM_ITERS + 1: u_nn sweeps, known sets
  LS_A2 = 1,    // Dc <= 2 ASLAM_ITERS + 1: u_n sweeps
  LS_A3 = 2,    // Dc <= 3 ASLAM_ITERS + 1: u sweeps
  LS_V = 3,     // Dv <= VEL_ITERS + 1: speed and its extension
  LS_R = 4,     // Dv <= VEL_ITERS + 4: advection stages
  LS_U = 5,     // A3 or R: normals and initial values
  LS_NLIST = 6,
  LS_FULL = 6   // every tile of the box
};
constexpr int LS_DIST_CAP = 1000;   // distances are capped here (beyond every radius)

// Box-sized scratch arrays of one instance.
struct LevelsetScratch {
  size_t nodes = 0;
  double* buf = nullptr;      // 12 box arrays of doubles
  uint8_t* known = nullptr;   // bit 0: K0, bit 1: K1, bit 2: K2, bit 3: speed band
};

// One instance as the kernels see it (device copy in LevelsetBatch).
struct LsInst {
  int dim, nx, ny, nz;
  int ntx, nty, ntz;
  int nband[LS_NLIST];        // tiles per list
  double h, mu;
  double* rho;                // user arrays (updated in place)
  double* u;
  double* buf;                // LevelsetScratch::buf
  size_t nodes;
  uint8_t* known;
  const int* band;            // lists, LS_NLIST blocks of ntx*nty*ntz entries
  const int* tdist;           // packed tile distances of the lists (high 16 bits: Dv)
  int rr;                     // radius of list R (Dv <= rr)
  int* status;                // latched device error of the instance
  double* vmax;               // set by levelset_begin
};

// Instance table and launch offsets of a batch of `count` instances.
struct LevelsetBatch {
  int count = 0;
  int dim = 2;
  LsInst* d_inst = nullptr;   // count
  LsInst* h_inst = nullptr;   // pinned, count (caller fills before levelset_begin)
  int* d_off = nullptr;       // (LS_NLIST + 1) * (count + 1): list offsets, then whole-box offsets
  int* h_off = nullptr;       // pinned
  double* d_vmax = nullptr;   // count maximum speeds
  double* h_vmax = nullptr;   // pinned mirror
  int total[LS_NLIST + 1] = {};
  double dt = 0.0;
  int reinit = 0;
  int uext = 0;               // scratch array holding u_ext after levelset_begin
};

hipError_t levelset_alloc(LevelsetScratch& s, size_t nodes);
void levelset_free(LevelsetScratch& s);
hipError_t levelset_batch_alloc(LevelsetBatch& b, int count, int dim);
void levelset_batch_free(LevelsetBatch& b);

// Steps 1 + 2a for every instance of b (h_inst filled by the caller; rho and
// u updated in place): levelset_begin enqueues everything up to the maximum
// speeds and their asynchronous copy to pinned memory; after the caller has
// synchronised the stream, levelset_end enqueues the advection substeps, the
// reinitialisation (if reinit) and the restriction of u.
hipError_t levelset_begin(LevelsetBatch& b, double dt, int reinit, hipStream_t stream);
hipError_t levelset_end(LevelsetBatch& b, hipStream_t stream);
// The extrapolation of Step 2 alone (the same sweeps as for u): each
// instance's u (any box field known on the computational points of rho) is
// replaced, over the whole box, by its quadratic normal extrapolation from
// those points; rho is not changed.  The caller synchronises the stream
// before it refills h_inst.
hipError_t levelset_extend(LevelsetBatch& b, hipStream_t stream);

}  // namespace etdfb
