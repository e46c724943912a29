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
// Level-set tile lists: L1 tile distances from the tiles with a
// computational point and from those with a node |rho| < h, then the six
// lists (radii[0..2] on the first distance, radii[3..4] on the second, and
// the union of lists 2 and 4) into lists (6 * ntiles) and counts (6).
hipError_t launch_band(const BoxHost& b, const int* comp_flag, const int* vb_flag, const int* radii, int* tmp0,
                       int* tmp1, int* lists, int* counts, hipStream_t s);
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
