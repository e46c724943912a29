// Level-set sweeps of the free-boundary step (Section 4.3 of the paper,
// Algorithm Steps 1-2): host interface.
//
// The sweeps run on a narrow band of tiles (the tile layout of the operator:
// 2D 32x8, 3D 16x4x4), built with the geometry: every tile within 46 nodes
// (per axis) of a tile holding a computational point, or within 28 nodes of
// a tile holding a node with |rho| < h.  Outside that band the extrapolated
// u, its normal derivatives and the extended speed are exactly 0 (their
// supports grow by one node per Jacobi sweep from the computational points:
// 15 + 15 + 15 sweeps; the speed by 20 sweeps from |rho| < h), so the band
// sweeps give the full-box values everywhere; the advection leaves rho
// unchanged where the speed is 0.  Reinitialisation and the final
// restriction of u cover the whole box.
//
// One launch per sweep serves a whole batch: block b works on band tile
// b - off[i] of instance i, off[] being the prefix sums of the band sizes.
#pragma once
#include <hip/hip_runtime.h>

#include "launch.h"

namespace etdfb {

// Iteration counts and pseudo-time steps of the sweeps (readings of the
// paper's unspecified parameters; identical in the CPU oracle).
constexpr int ASLAM_ITERS = 15;
constexpr int VEL_ITERS = 20;
constexpr int REINIT_ITERS = 10;
// Band radii in nodes (see above): 3 * ASLAM_ITERS + 1 and VEL_ITERS + 3
// (WENO stencil) + 1, rounded up.
constexpr int BAND_ASLAM = 46;
constexpr int BAND_SPEED = 28;

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
  int nband;                  // band tiles
  double h, mu;
  double* rho;                // user arrays (updated in place)
  double* u;
  double* buf;                // LevelsetScratch::buf
  size_t nodes;
  uint8_t* known;
  const int* band;            // band tile indices (nband entries)
  double* vmax;               // set by levelset_begin
};

// Instance table and launch offsets of a batch of `count` instances.
struct LevelsetBatch {
  int count = 0;
  int dim = 2;
  LsInst* d_inst = nullptr;   // count
  LsInst* h_inst = nullptr;   // pinned, count (caller fills before levelset_begin)
  int* d_off = nullptr;       // 2 * (count + 1): band offsets, then whole-box offsets
  int* h_off = nullptr;       // pinned
  double* d_vmax = nullptr;   // count maximum speeds
  double* h_vmax = nullptr;   // pinned mirror
  int total_band = 0;
  int total_full = 0;
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

}  // namespace etdfb
