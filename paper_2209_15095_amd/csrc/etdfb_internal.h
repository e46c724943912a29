// Structures shared by the host side (context management, launches) and the
// HIP kernels of libetdfb.  Plain data only; all pointers are device pointers.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace etdfb {

constexpr int TILE_PTS = 256;       // nodes per tile
constexpr int PART_STRIDE = 8;      // doubles per block in the partial-sum buffer
constexpr int MMAX_LIMIT = 64;      // largest Krylov dimension
constexpr int PMAX = 3;             // largest phi index in one combination
constexpr int EXPM_NMAX = MMAX_LIMIT + PMAX + 2;   // augmented matrix bound
// The persistent kernels are built twice (krylov.hip, namespaces kb1024 and
// kb512): blocks of 1024 threads for large instances and of 512 threads for
// small ones (more blocks on more CUs, twice the registers per thread).
enum KrylovBuild { KB_LARGE = 0, KB_SMALL = 1 };
constexpr int KB_THREADS[2] = {1024, 512};
constexpr int KB_TILES[2] = {1024 / TILE_PTS, 512 / TILE_PTS};   // tiles per block and loop trip
constexpr int NBR_STRIDE = 8;       // ints per slot in the face-neighbour table
constexpr double NOT_COMP = -1e300; // coefficient sentinel of non-computational points
constexpr int MAX_SPECIES = 4;      // components of u in a multi-species context

// Work vectors of the persistent kernel (indices into the workspace).
enum VecIndex {
  V_U = 0,     // running solution u(t_k) = W_0
  V_W1 = 1,    // W_1 .. W_3 (phipm-style stage vectors)
  V_W2 = 2,
  V_W3 = 3,
  V_B0 = 4,    // b_0 .. b_3 of a combination (compact layout)
  V_B1 = 5,
  V_B2 = 6,
  V_B3 = 7,
  V_X0 = 8,    // ETD: U_n
  V_F = 9,     // ETD: scratch
  V_T = 10,    // scratch
  V_Z0 = 11,   // A q_k (two buffers, alternating)
  V_Z1 = 12,
  V_G = 13,    // adjoint: dL/dU_{n+1}
  V_A = 14,    // adjoint: ETD2RK stage a
  V_AB = 15,   // adjoint: abar = f'(a) h phi_2(hA) g
  V_S = 16,    // adjoint: f'(U_n) s
  V_FG0 = 17,  // forced steps: G(t_n), G(t_n + h/2), G(t_n + h) (source + boundary forcing)
  V_FG1 = 18,
  V_FG2 = 19,
  V_Q0 = 20,   // Krylov basis q_0 .. q_MMAX
  NVEC = V_Q0 + MMAX_LIMIT + 1
};

struct BarrierDev {
  unsigned count;
  unsigned gen;               // last generation whose sums block 0 has released (single-reducer form)
  int abort;
  int pad;
};

struct GeomDev {
  int dim;
  int nx, ny, nz;
  int ntx, nty, ntz;
  int pad0;
  const int* tile_map;        // [ntz*nty*ntx] box tile -> slot, -1 inactive
  const int* slot_tile;       // [cap] slot -> box tile index
  const uint64_t* comp_bits;  // [cap*4]
  const uint64_t* irr_bits;   // [cap*4]
  const double* cdiag;        // [cap*256] diagonal weight sum c_p; NOT_COMP off the unknowns
  const int* nbr;             // [cap*NBR_STRIDE] face-neighbour slots (-x,+x,-y,+y,-z,+z), -1 none
  const int* n_active;        // device scalar: number of active tiles
  const int* n_unknowns;      // device scalar: number of computational points
  double coef;                // beta / h^2
  double dx;
  // variable beta (NULL for a constant beta): 2d face coefficients
  // beta_face / h^2 (-x,+x,-y,+y,-z,+z) and the diagonal, each a vector of
  // the workspace length: (A v)_p = sum_f w_f(p) v_{p+f} + dg(p) v_p
  const double* vcoef;
  size_t vld;
};

// Adaptive state carried across calls and the statistics of the last call.
struct KrylovStateDev {
  int m_guess[PMAX + 1];
  double tau_frac[PMAX + 1];
  int substeps, rejected, matvecs, m_last, expms, calls;
  double err_est;
  double t_done;
  double alg_bytes_per_unknown;   // algorithmic HBM bytes per unknown, last launch
  double alg_bytes_total;         // accumulated over launches: bytes/unknown * unknowns
  // device-clock ticks accumulated over launches (block 0 of the group):
  // whole launch, grid synchronisations, small exponentials, passes (tile
  // loops and block reductions), launch prologue
  double ticks_total, ticks_sync, ticks_expm, ticks_pass, ticks_pro, ticks_gap;
  int syncs, expm_calls;
};

enum JobMode {
  JOB_PHI = 0,        // out = sum_k phi_k(t A) b_k, b_k in V_B0..V_B3
  JOB_ETD1 = 1,       // one ETD1 step of V_X0
  JOB_ETD2RK = 2,     // one ETD2RK step of V_X0
  JOB_ETD2RK_STAGE = 3, // only the first stage a of ETD2RK
  JOB_APPLY = 4,        // V_U = A V_B0
  JOB_ADJ_ETD2RK = 5,   // adjoint of one ETD2RK step: V_U = dL/dU_n from V_G, V_X0; *dbeta += dL/dbeta
  JOB_ETD3RK = 6,       // one ETD3RK step of V_X0
  JOB_ETD4RK = 7,       // one ETD4RK step of V_X0
  JOB_ETD2 = 8,         // one ETD2 multistep step of V_X0; F(U_{n-1}) in V_G, replaced by F(U_n)
  JOB_ETD3RK_SIMUL = 9, // ETD3RK with stage a and the first-stage value at h from one integration
  JOB_ETD4RK_SIMUL = 10 // the same for ETD4RK
};

struct KrylovDev {
  GeomDev g;
  double* ws;                 // NVEC vectors of ld doubles
  size_t ld;
  double* part;               // 2 * gridDim * PART_STRIDE partial sums
  unsigned* flags;            // [gridDim] arrival generation of each block
  BarrierDev* bar;
  int tmax;                   // tiles per block cached in dynamic LDS
  int* status;                // first error code (0 = ok)
  KrylovStateDev* st;
  double tol;
  int m_min, m_max, m_step, max_substeps;
  double ra, rb;              // logistic reaction u (a - b u)
  int mode;
  int p;
  double t;                   // JOB_PHI: time t of phi_k(t A)
  double t_mid;               // JOB_PHI: 0, or the intermediate output time (into V_F)
  double beta;                // JOB_ADJ_ETD2RK: beta (A = beta A_1)
  double* dbeta;              // JOB_ADJ_ETD2RK: device scalar, dL/dbeta accumulated
  double h;                   // ETD step
  int g_first, g_size;        // blocks of this instance in the launch grid
  int stage_min;              // fewest active tiles for the LDS-staged Lanczos pass
  int sync_master_min;        // blocks (of the grid or group) from which block 0 alone reduces at a grid synchronisation
  int first;                  // JOB_ETD2: no F(U_{n-1}) yet, take one ETD2RK step
  int forced;                 // F(U, t) = f(U) + G(t), G of the stage times in V_FG0..V_FG2
  // m > 1 species: the active tiles are repeated m times (species s in
  // slots s*n .. s*n + n - 1 of the n base slots), f_s(u) = u_s (sa[s] -
  // sum_j sb[s][j] u_j)
  int species;
  double sa[MAX_SPECIES];
  double sb[MAX_SPECIES * MAX_SPECIES];
};

// Default of KrylovDev::stage_min: the LDS-staged Lanczos pass pays where
// the vectors outgrow the L2 (2048 active tiles, 4 MiB per vector); below,
// its two block barriers per loop trip cost more than the misses it saves.
constexpr int STAGE_MIN_TILES = 2048;

// Default of KrylovDev::sync_master_min.  At a grid synchronisation every
// block publishes its partial sums and an arrival flag.  Below this many
// blocks every block polls all flags and sums all partials itself (one
// memory round trip after the last arrival); from it on, block 0 alone does
// so and publishes the sums in one word the others poll: one round trip
// more, but without every block hammering the same few cache lines, which
// costs more once there are many blocks (ellipsoid192, about 150 blocks:
// 7.8 -> 5.8 us per synchronisation; star512, 24 blocks: 3.4 -> 3.6 us).
// The groups of a batched launch keep the all-to-all form.
constexpr int SYNC_MASTER_MIN_BLOCKS = 64;

// Status codes (mirror include/etdfb.h).
enum {
  ST_OK = 0,
  ST_INVALID = -1,
  ST_HIP = -2,
  ST_NO_DEVICE = -3,
  ST_KRYLOV = -4,
  ST_NONFINITE = -5,
  ST_DOMAIN = -6,
  ST_BARRIER = -7,
  ST_NO_GEOMETRY = -8,
  ST_FRONT = -9
};

}  // namespace etdfb
