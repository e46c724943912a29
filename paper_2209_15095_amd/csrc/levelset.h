// Level-set sweeps of the free-boundary step (Section 4.3 of the paper,
// Algorithm Steps 1-2): host interface.
#pragma once
#include <hip/hip_runtime.h>

#include "launch.h"

namespace etdfb {

// Box-sized scratch arrays owned by a context.
struct LevelsetScratch {
  size_t nodes = 0;
  double* buf = nullptr;      // 12 box arrays of doubles
  uint8_t* known = nullptr;   // bit 0: K0, bit 1: K1, bit 2: K2, bit 3: velocity band
  double* vmax = nullptr;     // device scalar
  double* h_vmax = nullptr;   // pinned host mirror
};

struct LevelsetArgs {
  BoxHost box;
  double mu;
  double dt;
  int reinit;
  const uint8_t* mask;
  int* status;
};

// Iteration counts and pseudo-time steps of the sweeps (readings of the
// paper's unspecified parameters; identical in the CPU oracle).
constexpr int ASLAM_ITERS = 15;
constexpr int VEL_ITERS = 20;
constexpr int REINIT_ITERS = 10;

hipError_t levelset_alloc(LevelsetScratch& s, size_t nodes);
void levelset_free(LevelsetScratch& s);
// Steps 1 + 2a on rho and u (box arrays, updated in place): levelset_begin,
// a synchronisation of the stream, levelset_end.  The two halves let a batch
// share one synchronisation between many instances.
hipError_t levelset_run(const LevelsetArgs& a, LevelsetScratch& s, double* rho, double* u,
                        hipStream_t stream);
hipError_t levelset_begin(const LevelsetArgs& a, LevelsetScratch& s, double* rho, double* u,
                          hipStream_t stream);
hipError_t levelset_end(const LevelsetArgs& a, LevelsetScratch& s, double* rho, double* u,
                        hipStream_t stream);

}  // namespace etdfb
