// Host-side launch wrappers of the HIP kernels (one per kernel file), used by
// the C-ABI layer.  All launches are asynchronous on the given stream.
#pragma once
#include <hip/hip_runtime.h>

#include "etdfb_internal.h"

namespace etdfb {

struct BoxHost {
  int dim, nx, ny, nz;
  int ntx, nty, ntz;
  int tx, ty, tz;
  double lo[3];
  double dx;
};

// geometry.hip
//
// The geometry build works on a table of instances (a single context is a
// table of one): per instance its box, level set and output arrays.
struct GeomInst {
  BoxHost b;
  const double* rho;     // level set (box layout), set per build
  uint8_t* mask;
  int* tile_flag;        // tiles with a computational point
  int* tile_vb;          // tiles with a node |rho| < h
  int* tile_map;
  int* slot_tile;
  uint64_t* comp_bits;
  uint64_t* irr_bits;
  double* cdiag;
  int* nbr;
  int* band_tmp;         // 2 * ntiles
  int* band_list;        // 3 * ntiles: level-set lists SC, SV, U
  int* counters;         // [0] active tiles, [1] status, [2..3] case counts, [4] unknowns, [5..6] species,
                         // then the level-set list counts (levelset.h)
  double* ws;            // workspace vectors (gather / scatter targets)
  size_t ld;
  size_t nodes;
  int ntiles;
  int pad;
  // variable beta (set for etd_geometry_build_var only): beta at the face
  // midpoints node + h/2 e_d (box arrays, d < dim); outputs: the 2d face
  // coefficients and the diagonal (vcoef, 2d+1 vectors of ld), and per
  // point up to TAPS_PER boundary taps (count, coefficient, point)
  const double* beta_face[3];
  double* vcoef;
  int* tap_n;
  double* tap_coef;
  double* tap_pt;
};

// Boundary taps per computational point: two per face (Case 3 has two
// boundary points, Case 2 one).
constexpr int TAPS_PER = 12;

// Block prefixes of the batched geometry launches: 256 nodes per block,
// 256 tiles per block, and blocks that loop over the active tiles (at most
// GEOM_SLOT_BLOCKS per instance).
enum { GEOM_PRE_NODE = 0, GEOM_PRE_T256 = 1, GEOM_PRE_TILE = 2, GEOM_NPRE = 3 };
constexpr int GEOM_SLOT_BLOCKS = 2048;
inline int geom_blocks_per(int q, size_t nodes, int ntiles) {
  if (q == GEOM_PRE_NODE) return (int)((nodes + 255) / 256);
  if (q == GEOM_PRE_T256) return (ntiles + 255) / 256;
  return ntiles < GEOM_SLOT_BLOCKS ? ntiles : GEOM_SLOT_BLOCKS;
}

struct GeomBatch {
  int count = 0;
  int ncnt = 0;                  // counters per instance
  GeomInst* h_tab = nullptr;     // pinned; uploaded by launch_geometry
  GeomInst* d_tab = nullptr;
  int* h_pre = nullptr;          // GEOM_NPRE block prefixes of count + 1 entries
  int* d_pre = nullptr;
  int blocks[GEOM_NPRE] = {};    // launch sizes
  int* h_cnt = nullptr;          // collected counters (pinned), ncnt per instance
  int* d_cnt = nullptr;
  // Eager builds of large tables run the level-set distance passes and
  // lists on a stream of their own beside the tile scan and coefficients
  // (both read only the classification); created on the first such build,
  // default priority.
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

hipError_t geom_batch_alloc(GeomBatch& gb, int count, int ncnt);
void geom_batch_free(GeomBatch& gb);
// After the table's sizes are filled in: block prefixes (synchronous).
hipError_t geom_batch_prefix(GeomBatch& gb);
// Whole build of every instance (classification, tile scan, Case 1-3
// coefficients and face neighbours, level-set tile distances and sorted
// lists: radii = {largest Dc, largest Dv, counter index of the cumulative
// Dc counts, of the Dv counts, of the size of U}), then the counters of all
// instances into gb.h_cnt
// (asynchronous: read after synchronising the stream).  The table's rho
// pointers must be set; the table is uploaded from pinned memory, so it
// must not change before the stream has passed this call.
hipError_t launch_geometry(GeomBatch& gb, const int* radii, hipStream_t s, bool device_sized = false);
// Device-sized builds (for graph capture) neither upload the table nor copy
// the counters back: geom_upload copies the table to the device beforehand
// (asynchronous, from pinned memory).
hipError_t geom_upload(GeomBatch& gb, hipStream_t s);
// After launch_geometry of a one-instance table whose beta_face, vcoef and
// tap arrays are set: the variable-beta coefficients and boundary taps.
hipError_t launch_geometry_var(GeomBatch& gb, hipStream_t s);
// After launch_geometry of a one-instance table: repeat the active tiles for
// m species (the face-neighbour slots of copy s point into copy s); the
// Krylov tile and unknown counts go to counters[5] and [6].
hipError_t launch_replicate_species(GeomBatch& gb, int m, hipStream_t s);
// out (box) = src + sum over the taps of coef * ub[tap_off[p] + k] at the
// computational points (src may be NULL), 0 elsewhere.
hipError_t launch_forcing(const BoxHost& b, const int* tile_map, const uint64_t* comp_bits, const int* tap_n,
                          const double* tap_coef, const int* tap_off, const double* ub, const double* src,
                          double* out, hipStream_t s);
// Batched box <-> workspace-vector transfers; d_boxes: device array of the
// instances' box pointers.
hipError_t launch_gather_batch(const GeomBatch& gb, const double* const* d_boxes, int vec, hipStream_t s);
hipError_t launch_scatter_batch(const GeomBatch& gb, double* const* d_boxes, int vec, hipStream_t s);
hipError_t launch_gather(const BoxHost& b, const double* box, const int* slot_tile,
                         const uint64_t* comp_bits, const int* n_active, double* vec, int grid,
                         hipStream_t s);
hipError_t launch_scatter(const BoxHost& b, const double* vec, const int* tile_map,
                          const uint64_t* comp_bits, double* box, hipStream_t s);
// The active tiles only (the other nodes of box are left as they are).
hipError_t launch_scatter_tiles(const BoxHost& b, const double* vec, const int* slot_tile,
                                const uint64_t* comp_bits, const int* n_active, double* box, int grid,
                                hipStream_t s);

// krylov.hip, one build per block size (KrylovBuild)
#define ETDFB_KRYLOV_DECLS                                                                              \
  hipError_t launch_krylov(int dim, const KrylovDev& P, int grid, hipStream_t s);                       \
  int krylov_max_blocks_per_cu(int dim, int tmax);                                                       \
  size_t krylov_dyn_lds(int dim, int tmax);                                                              \
  hipError_t launch_krylov_group(int dim, const KrylovDev* Ps, int count, const int* blk_inst, int blocks, \
                                 bool cooperative, hipStream_t s);
namespace kb1024 { ETDFB_KRYLOV_DECLS }
namespace kb512 { ETDFB_KRYLOV_DECLS }
#undef ETDFB_KRYLOV_DECLS

inline hipError_t launch_krylov(int kb, int dim, const KrylovDev& P, int grid, hipStream_t s) {
  return kb == KB_SMALL ? kb512::launch_krylov(dim, P, grid, s) : kb1024::launch_krylov(dim, P, grid, s);
}
inline int krylov_max_blocks_per_cu(int kb, int dim) {
  return kb == KB_SMALL ? kb512::krylov_max_blocks_per_cu(dim, 1) : kb1024::krylov_max_blocks_per_cu(dim, 1);
}
inline hipError_t launch_krylov_group(int kb, int dim, const KrylovDev* Ps, int count, const int* blk_inst,
                                      int blocks, bool cooperative, hipStream_t s) {
  return kb == KB_SMALL ? kb512::launch_krylov_group(dim, Ps, count, blk_inst, blocks, cooperative, s)
                        : kb1024::launch_krylov_group(dim, Ps, count, blk_inst, blocks, cooperative, s);
}

}  // namespace etdfb
