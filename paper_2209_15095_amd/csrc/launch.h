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
hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t s);
hipError_t launch_classify(const BoxHost& b, const double* rho, uint8_t* mask, int* tile_flag,
                           int* tile_vb, int* status, hipStream_t s);
// Level-set band: tiles within band_nodes_comp nodes (per axis) of a tile
// with a computational point or band_nodes_speed nodes of a tile with a node
// |rho| < h; list of their indices and count (device).
hipError_t launch_band(const BoxHost& b, const int* comp_flag, const int* vb_flag, int band_nodes_comp,
                       int band_nodes_speed, int* tmp0, int* tmp1, int* band_map, int* band_list, int* nband,
                       hipStream_t s);
hipError_t launch_scan_tiles(const int* tile_flag, int ntiles, int* tile_map, int* slot_tile,
                             int* n_active, hipStream_t s);
hipError_t launch_tile_coeff(const BoxHost& b, const double* rho, const uint8_t* mask,
                             const int* tile_map, uint64_t* comp_bits, uint64_t* irr_bits,
                             double* cdiag, int* nbr, int* counts, int ntiles, hipStream_t s);
hipError_t launch_gather(const BoxHost& b, const double* box, const int* slot_tile,
                         const uint64_t* comp_bits, const int* n_active, double* vec, int grid,
                         hipStream_t s);
hipError_t launch_scatter(const BoxHost& b, const double* vec, const int* tile_map,
                          const uint64_t* comp_bits, double* box, hipStream_t s);

// krylov.hip
hipError_t launch_krylov(int dim, const KrylovDev& P, int grid, hipStream_t s);
int krylov_max_blocks_per_cu(int dim, int tmax);
size_t krylov_dyn_lds(int dim, int tmax);
hipError_t launch_krylov_group(int dim, const KrylovDev* Ps, int count, const int* blk_inst, int blocks,
                               bool cooperative, hipStream_t s);

}  // namespace etdfb
