// Persistent HIP kernel for sum_k phi_k(tA) b_k and the ETD steps built on it.
//
// What is computed (Section 3.3 of the paper, eq. 3.7 and its ODE form):
// out = sum_{k=0}^{p} phi_k(tA) b_k is the time-t value of
// u' = A u + sum_{k>=1} s^{k-1}/(k-1)! w_k, u(0) = b_0, w_k = b_k / t^k.
// The paper evaluates it with an adaptive Krylov method of the phipm family
// (incomplete orthogonalisation of length 2, which for the symmetric matrix
// of Section 2 is the Lanczos recurrence).  Design used here:
//
// * Substeps t_j -> t_j + tau.  With W_0 = u(t_j) and
//   W_k = A W_{k-1} + sum_{l=0}^{p-k} t_j^l/l! w_{k+l} (k = 1..p),
//   u(t_j + tau) = sum_{k<p} tau^k/k! W_k + tau^p phi_p(tau A) W_p, since
//   phi_k(z) = 1/k! + z phi_{k+1}(z).
// * phi_p(tau A) W_p ~ |W_p| V_m phi_p(tau T_m) e_1 from m Lanczos steps
//   started at W_p (basis kept unnormalised with its norms n_k).
// * One grid synchronisation per Lanczos step: pass k forms
//   q_k = (z_{k-1} - alpha_{k-1} q_{k-1}) / n_{k-1} - (n_{k-1}/n_{k-2}) q_{k-2}
//   pointwise (z_{k-1} = A q_{k-1} from the previous pass), also at the face
//   neighbours of each point, so z_k = A q_k follows in the same pass; its
//   reduction yields both |q_k|^2 and <z_k, q_k>.
// * phi_p(tau T) e_1 and phi_{p+1}(tau T) e_1 are columns of the exponential
//   of the (m+p+1)^2 augmented matrix [[tau T, e_1, 0], [0, 0, I], [0, 0, 0]],
//   computed in LDS by scaling, Taylor-Horner (X is sparse, so Horner is
//   O(N^2) per term) and squaring.
// * Error estimate |W_p| n_m tau^{p+1} |e_m^T phi_{p+1}(tau T) e_1|
//   (generalised residual); accept when it is below
//   tol * tau/t * max(|u(t_j)|, tau^p |W_p| / p!) and below
//   tol * tau/t * |u(t_j + tau)|.  Otherwise grow m in steps of m_step up to
//   m_max, then shrink tau.  A call starts at the dimension its previous
//   call accepted last (one lower when that passed below 1 % of the
//   tolerance), and at the fraction of t its last substep took after a
//   shrink.
//
// Everything after the launch is decided on the device: every block reduces
// the same per-block partials in the same order, so all blocks hold
// bit-identical scalars and take identical branches (no host round trip, no
// broadcast).  FP64 throughout; no matrix cores (nothing here is a dense
// contraction except the tiny in-LDS exponential).
#include <math.h>

#include "device_common.h"
#include "launch.h"

namespace etdfb {

// This file is compiled once per block size (KRYLOV_KBLOCK = 1024 or 512),
// each build in a namespace of its own.
#ifndef KRYLOV_KBLOCK
#define KRYLOV_KBLOCK 1024
#endif
#if KRYLOV_KBLOCK == 1024
#define KRYLOV_NS kb1024
#elif KRYLOV_KBLOCK == 512
#define KRYLOV_NS kb512
#else
#error "KRYLOV_KBLOCK must be 1024 or 512"
#endif
namespace KRYLOV_NS {

constexpr int KBLOCK = KRYLOV_KBLOCK;            // threads per block of the persistent kernels
constexpr int KTILES = KBLOCK / TILE_PTS;        // tiles a block works on per loop trip

constexpr int META_TRIPS = 128;         // loop trips whose tile metadata a block keeps in LDS
constexpr int NWAVE = KBLOCK / 64;

struct Ctl {
  // tile metadata of this block's first META_TRIPS loop trips (the same
  // tiles every pass): mask words per wave, face-neighbour slots per tile
  uint64_t mcw[META_TRIPS][NWAVE];
  uint64_t miw[META_TRIPS][NWAVE];
  int mnb[META_TRIPS][KTILES][8];   // face slots (-x,+x,-y,+y,-z,+z); 2D: then the diagonals
  // Lanczos data of the current substep (written by thread 0, read by all)
  double alpha[MMAX_LIMIT + 2];
  double nrm[MMAX_LIMIT + 2];
  double coef[MMAX_LIMIT + 1];
  double red[8];
  double scratch[(KBLOCK / 64) * 4];
  // adaptive state per p carried across calls (thread 0 writes)
  double tau_frac[PMAX + 1];
  int m_guess[PMAX + 1];
  // statistics of the launch, kept by thread 0 (out of the registers the
  // passes need): counters, the last accepted substep, algorithmic HBM
  // bytes per unknown moved so far (what the method must read and write per
  // computational point: vectors only; neighbour re-reads, masks and tile
  // padding are not counted), device-clock ticks of block 0 (passes, from
  // the start of a pass's tile loop until every wave of the block is done
  // and the block has reduced its partials; grid synchronisations; small
  // exponentials; the launch prologue; t_mark: start of the current pass)
  struct Stats {
    int substeps, rejected, matvecs, m_last, expms, n_sync;
    double err_est, ratio_last, t_done, bpu;   // ratio_last: error / tolerance of the last accepted substep
    // tk_gap: from the end of a synchronisation to the start of the next
    // timed region (pass or exponential); t_free: end of the last
    // synchronisation not yet followed by one (0: none)
    unsigned long long tk_sync, tk_expm, tk_pass, tk_pro, t_mark, tk_gap, t_free;
  } st;
  int abort;
};

// The loop of the 2D z-free staged Lanczos pass (Engine::lanczos_zf2), a
// function of its own so that its registers are allocated apart from the
// rest of the persistent kernel.  tb is the block's tile range within a
// trip (Engine::tile_block).  acc receives this thread's partial sums of
// |q_k|^2 and <A q_k, q_k>.
__device__ __attribute__((noinline)) void zf2_loop(gptr<const double> q1, gptr<const double> q2,
                                                   gptr<double> qk, gptr<const double> cdiag, double coef,
                                                   double alpha, double inv_n, double cm, int na, int G,
                                                   int tb, lptr<double> stage, lptr<const int> mnb,
                                                   double* acc) {
  constexpr int X = TileShape<2>::X, Y = TileShape<2>::Y;
  constexpr int W2 = X + 4, H2 = Y + 4;   // q_{k-1} box (2-node halo)
  constexpr int W1 = X + 2, H1 = Y + 2;   // q_{k-2}, c_p, q_k box (1-node halo)
  constexpr int N2 = W2 * H2, N1 = W1 * H1;
  constexpr int NH2 = 2 * 2 * (X + Y) + 4;   // two-node face halo and the diagonals
  constexpr int NH1 = 2 * (X + Y);           // one-node face halo
  constexpr int PER = N2 + N1 + 2 * N1;      // doubles per tile
  static_assert(NH2 <= TILE_PTS && NH1 <= TILE_PTS, "one halo node per thread");
  static_assert(KTILES * PER <= 2 * EXPM_NMAX * EXPM_NMAX, "staging exceeds the exponential buffers");
  // arguments arrive in vector registers: back to wave-uniform values
  q1 = uniform(q1);
  q2 = uniform(q2);
  qk = uniform(qk);
  cdiag = uniform(cdiag);
  coef = uniform(coef);
  alpha = uniform(alpha);
  inv_n = uniform(inv_n);
  cm = uniform(cm);
  na = __builtin_amdgcn_readfirstlane(na);
  G = __builtin_amdgcn_readfirstlane(G);
  tb = __builtin_amdgcn_readfirstlane(tb);
  double a0 = 0.0, a1 = 0.0;
    const int sub = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / TILE_PTS));
    const int l = (int)(threadIdx.x % TILE_PTS);
    const int lx = l % X, ly = l / X;
    const lptr<double> L1 = stage + (size_t)sub * PER;    // q_{k-1}
    const lptr<double> LC = L1 + N2;                        // c_p
    const lptr<double> LQ = LC + N1;                        // q_{k-2}, then q_k (two halves)
    const int o2 = (lx + 2) + W2 * (ly + 2);   // own point in the boxes
    const int o1 = (lx + 1) + W1 * (ly + 1);
    // two-node halo node of this thread: neighbour entry (0..3 faces,
    // 4..7 diagonals), index in that tile, position in the q_{k-1} box
    int h2n = -1, h2l = 0, h2p = 0;
    if (l < NH2) {
      int x, y, nx, ny;
      if (l < 4 * Y) {                 // x faces, depths 1 and 2
        const int side = l / (2 * Y), dd = 1 + (l / Y) % 2, row = l % Y;
        x = side ? X - 1 + dd : -dd;
        y = row;
        nx = side ? dd - 1 : X - dd;
        ny = row;
        h2n = side;
      } else if (l < 4 * Y + 4 * X) {  // y faces, depths 1 and 2
        const int q = l - 4 * Y;
        const int side = q / (2 * X), dd = 1 + (q / X) % 2, col = q % X;
        x = col;
        y = side ? Y - 1 + dd : -dd;
        nx = col;
        ny = side ? dd - 1 : Y - dd;
        h2n = 2 + side;
      } else {                         // diagonals -x-y, +x-y, -x+y, +x+y
        const int q = l - 4 * Y - 4 * X;
        const int sx = q & 1, sy = q >> 1;
        x = sx ? X : -1;
        y = sy ? Y : -1;
        nx = sx ? 0 : X - 1;
        ny = sy ? 0 : Y - 1;
        h2n = 4 + q;
      }
      h2l = nx + X * ny;
      h2p = (x + 2) + W2 * (y + 2);
    }
    // one-node face halo node of this thread
    int h1n = -1, h1l = 0, h1p1 = 0, h1p2 = 0;
    if (l < NH1) {
      int x, y, nx, ny;
      if (l < 2 * Y) {
        const int side = l / Y, row = l % Y;
        x = side ? X : -1;
        y = row;
        nx = side ? 0 : X - 1;
        ny = row;
        h1n = side;
      } else {
        const int q = l - 2 * Y;
        const int side = q / X, col = q % X;
        x = col;
        y = side ? Y : -1;
        nx = col;
        ny = side ? 0 : Y - 1;
        h1n = 2 + side;
      }
      h1l = nx + X * ny;
      h1p1 = (x + 1) + W1 * (y + 1);
      h1p2 = (x + 2) + W2 * (y + 2);
    }
    const int stride = G * KTILES;
    const int base0 = tb * KTILES;
    // loads of one trip (element 0 where there is nothing; selected after)
    double a_q1, a_q2, a_cd, a_h2, a_h1q, a_h1c;
    auto issue = [&](int r, int slot, bool valid) {
      int nb[8];
#pragma unroll
      for (int d = 0; d < 8; ++d) nb[d] = valid ? mnb[(r * KTILES + sub) * 8 + d] : -1;
      const unsigned i = valid ? (unsigned)slot * TILE_PTS + (unsigned)l : 0u;
      int s2 = -1, s1 = -1;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        s2 = h2n == d ? nb[d] : s2;
        s1 = h1n == d ? nb[d] : s1;
      }
      const bool ok2 = s2 >= 0, ok1 = s1 >= 0;
      const unsigned j2 = ok2 ? (unsigned)s2 * TILE_PTS + (unsigned)h2l : 0u;
      const unsigned j1 = ok1 ? (unsigned)s1 * TILE_PTS + (unsigned)h1l : 0u;
      const double v1 = at(q1, i), v2 = at(q2, i), vc = at(cdiag, i);
      const double w2 = at(q1, j2), w1q = at(q2, j1), w1c = at(cdiag, j1);
      a_q1 = valid ? v1 : 0.0;
      a_q2 = valid ? v2 : 0.0;
      a_cd = valid ? vc : NOT_COMP;
      a_h2 = ok2 ? w2 : 0.0;
      a_h1q = ok1 ? w1q : 0.0;
      a_h1c = ok1 ? w1c : NOT_COMP;
    };
    // q_k at one node of the face-halo box (position p1 there, p2 in the
    // q_{k-1} box), from the staged values
    auto qnode = [&](int p1, int p2, lptr<double> Q) -> double {
      const double cd = LC[p1];
      const double v = L1[p2];
      const double az = coef * (((L1[p2 - 1] + L1[p2 + 1]) + (L1[p2 - W2] + L1[p2 + W2])) - cd * v);
      const double q = (az - alpha * v) * inv_n - cm * Q[p1];
      return cd > -1e299 ? q : 0.0;   // NOT_COMP: not computational
    };
    if (base0 < na) {
      int slot = base0 + sub;
      bool valid = slot < na;
      issue(0, slot, valid);
      for (int r = 0;; ++r) {
        const lptr<double> Q = LQ + (r & 1) * N1;
        // stage (the previous trip's reads of this trip's buffers are behind
        // the last barrier of the previous trip; q_k's half alternates)
        L1[o2] = a_q1;
        Q[o1] = a_q2;
        LC[o1] = a_cd;
        if (h2n >= 0) L1[h2p] = a_h2;
        if (h1n >= 0) {
          Q[h1p1] = a_h1q;
          LC[h1p1] = a_h1c;
        }
        const int nslot = slot + stride;
        const bool more = base0 + (r + 1) * stride < na;
        const bool nvalid = nslot < na;
        __syncthreads();
        issue(r + 1 < META_TRIPS ? r + 1 : r, nslot, nvalid);
        // q_k at the own point and at this thread's halo node (in place of q_{k-2})
        const double cdo = LC[o1];
        const double qo = qnode(o1, o2, Q);
        const double qh = h1n >= 0 ? qnode(h1p1, h1p2, Q) : 0.0;
        Q[o1] = qo;
        if (h1n >= 0) Q[h1p1] = qh;
        __syncthreads();
        if (valid) {
          const bool comp = cdo > -1e299;
          const double z = comp ? coef * (((Q[o1 - 1] + Q[o1 + 1]) + (Q[o1 - W1] + Q[o1 + W1])) - cdo * qo) : 0.0;
          // streaming store: q_k is read back only in the next pass
          __builtin_nontemporal_store(qo, (gptr<double>)((gptr<char>)qk + ((unsigned)slot * TILE_PTS + (unsigned)l) * 8u));
          a0 += qo * qo;
          a1 += z * qo;
        }
        if (!more) break;
        slot = nslot;
        valid = nvalid;
      }
      __syncthreads();   // LDS free for the exponential
    }
  acc[0] = a0;
  acc[1] = a1;
}

// An instance is worked on by a group of G co-resident blocks (lb = this
// block's index in the group).  G == 1: the block synchronises only with
// itself; G > 1: the group synchronises with the flag barrier below, on the
// instance's own flags and partial sums, so groups of different instances
// never wait for each other.
template <int DIM>
struct Engine {
  const KrylovDev& P;
  Ctl& c;
  double* R;   // LDS EXPM_NMAX^2
  double* S;   // LDS EXPM_NMAX^2
  int nact;
  int pass_no;
  int lb, G;
  // control state: every thread of every block holds identical copies
  bool failed;
  int iu;   // vector holding u(t_j) = W_0 (V_U or V_T, ping-pong with the combine output)
  size_t sp_stride;   // index distance between the copies of one node in consecutive species
  double st_tmid;     // intermediate output of the current stage's combination (0: none)
  int st_midvec;      // and its vector

  // statistics (thread 0 only)
  __device__ __forceinline__ void count(int& f, int v) {
    if (threadIdx.x == 0) f += v;
  }
  __device__ __forceinline__ void add_bytes(double b) {
    if (threadIdx.x == 0) c.st.bpu += b;
  }
  // block 0, thread 0: a timed region starts at `now` (closes a pending gap)
  __device__ __forceinline__ void region_start(unsigned long long now) {
    if (c.st.t_free) c.st.tk_gap += now - c.st.t_free;
    c.st.t_free = 0;
  }

  __device__ __forceinline__ gptr<double> V(int i) const { return glb(P.ws) + (size_t)i * P.ld; }

  // Index of this block's range of KTILES tiles within a loop trip.  The
  // hardware hands consecutive workgroups to the 8 XCDs in turn; numbering
  // the ranges so that the blocks of one XCD take adjacent ranges keeps a
  // tile and its nearest neighbours in the compacted order (the rest of its
  // row, the neighbouring rows) under one L2.
  __device__ __forceinline__ int tile_block() const {
    if ((G & 7) != 0 || (P.g_first & 7) != 0) return lb;
    return (lb & 7) * (G >> 3) + (lb >> 3);
  }

  __device__ __forceinline__ void fail(int code) {
    if (threadIdx.x == 0 && lb == 0) atomicCAS(P.status, 0, code);
    failed = true;
  }

  // Grid synchronisation fused with the reduction of NR per-block partials.
  // Every wave waits for its own stores; lane 0 writes the block's partials,
  // one agent-scope release publishes them with the pass's stores, then it
  // writes its arrival generation into its own flag.  Below
  // P.sync_master_min blocks, wave 0 of every block polls every flag (no
  // contended atomic), acquires, and sums the partials in block order; from
  // it on, block 0 alone does so, writes the sums and the abort state into
  // its own row of the partial buffer (entries 4..6, past every block's
  // partials) and releases them with the generation word of the barrier,
  // which the other blocks poll before they acquire and read the sums.
  // Either way every block obtains the same bits (one summation order), and
  // the release/acquire chain through block 0 orders every block's stores
  // before the next pass.  Polls are bounded: past SPIN_LIMIT the abort flag
  // goes up and every block leaves.
  template <int NR>
  __device__ __forceinline__ bool grid_sync(const double (&acc)[NR], double (&out)[NR]) {
    static_assert(NR <= 4 && PART_STRIDE >= 7, "partials, sums and abort state share block 0's row");
    const unsigned long long t_in = wall_clock64();
    ++pass_no;
    const unsigned gen = (unsigned)pass_no;
    gptr<double> part = glb(P.part) + (size_t)(gen & 1u) * G * PART_STRIDE;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      if (lane == 0) {
        for (int k = 0; k < NR; ++k) part[(size_t)lb * PART_STRIDE + k] = acc[k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&P.flags[lb], gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const bool master = G >= P.sync_master_min;
      int ab = 0;
      if (!master || lb == 0) {
        long spins = 0;
        // a lane's flags and partials (b = lane + 64 q) are loaded four at a
        // time, all in flight before the first is used
        while (true) {
          bool mine = true;
          for (int b0 = lane; b0 < G; b0 += 256) {
            unsigned f[4];
  #pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int b = b0 + 64 * q;
              f[q] = (b < G) ? __hip_atomic_load(&P.flags[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : gen;
            }
  #pragma unroll
            for (int q = 0; q < 4; ++q) mine &= f[q] >= gen;
          }
          if (__ballot(!mine) == 0ull) break;
          __builtin_amdgcn_s_sleep(1);
          if ((++spins & 255) == 0) {
            ab = __hip_atomic_load(&P.bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ab) break;
            if (spins > SPIN_LIMIT) {
              if (lane == 0) __hip_atomic_store(&P.bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ab = 1;
              break;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        double t[NR];
  #pragma unroll
        for (int k = 0; k < NR; ++k) t[k] = 0.0;
        for (int b0 = lane; b0 < G; b0 += 256) {
          double v[4][NR];
  #pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int b = b0 + 64 * q;
  #pragma unroll
            for (int k = 0; k < NR; ++k) v[q][k] = (b < G) ? part[(size_t)b * PART_STRIDE + k] : 0.0;
          }
          // fixed order: every block sums the same values the same way
  #pragma unroll
          for (int k = 0; k < NR; ++k) t[k] += ((v[0][k] + v[1][k]) + v[2][k]) + v[3][k];
        }
  #pragma unroll
        for (int k = 0; k < NR; ++k) {
          const double r = wave_sum_lane0(t[k]);
          if (lane == 0) c.red[k] = r;
        }
        if (master && lane == 0) {
          // publish the sums and the abort state for the other blocks
          gptr<double> res = part + 4;
          for (int k = 0; k < NR; ++k) res[k] = c.red[k];
          res[2] = ab ? 1.0 : 0.0;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_store(&P.bar->gen, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      } else {
        // wait for block 0's sums
        long spins = 0;
        while (true) {
          if (__hip_atomic_load(&P.bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= gen) break;
          __builtin_amdgcn_s_sleep(1);
          if ((++spins & 255) == 0) {
            ab = __hip_atomic_load(&P.bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ab) break;
            if (spins > SPIN_LIMIT) {
              if (lane == 0) __hip_atomic_store(&P.bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ab = 1;
              break;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (lane == 0 && !ab) {
          gptr<const double> res = part + 4;
          for (int k = 0; k < NR; ++k) c.red[k] = res[k];
          ab = res[2] != 0.0 ? 1 : 0;
        }
      }
      if (lane == 0) c.abort = ab;
    }
    __syncthreads();
    for (int k = 0; k < NR; ++k) out[k] = c.red[k];
    const int ab = c.abort;
    __syncthreads();
    if (threadIdx.x == 0 && lb == 0) {
      const unsigned long long t_out = wall_clock64();
      c.st.tk_sync += t_out - t_in;
      c.st.t_free = t_out;
      ++c.st.n_sync;
    }
    return ab == 0;
  }

  // Close a pass: block sum of NR partials, then (grid mode) the grid
  // synchronisation with the fixed-order grid reduction into out[].
  // Returns false on a barrier time-out or a non-finite sum (status set; every
  // block takes the same exit).
  template <int NR>
  __device__ __forceinline__ bool finish(double (&acc)[NR], double (&out)[NR]) {
    block_sum<NR>(acc, c.scratch);
    if (threadIdx.x == 0 && lb == 0) c.st.tk_pass += wall_clock64() - c.st.t_mark;
    if (G == 1) {
      for (int k = 0; k < NR; ++k) out[k] = acc[k];
      if (threadIdx.x == 0 && lb == 0) c.st.t_free = wall_clock64();
    } else if (!grid_sync<NR>(acc, out)) {
      if (threadIdx.x == 0) atomicCAS(P.status, 0, ST_BARRIER);
      failed = true;
      return false;
    }
    for (int k = 0; k < NR; ++k)
      if (!isfinite(out[k])) {
        fail(ST_NONFINITE);
        return false;
      }
    return true;
  }

  __device__ __forceinline__ bool barrier() {
    __syncthreads();
    if (threadIdx.x == 0 && lb == 0) {
      c.st.tk_pass += wall_clock64() - c.st.t_mark;
      if (G == 1) c.st.t_free = wall_clock64();
    }
    if (G == 1) return true;
    double a[1] = {0.0}, o[1];
    if (!grid_sync<1>(a, o)) {
      if (threadIdx.x == 0) atomicCAS(P.status, 0, ST_BARRIER);
      failed = true;
      return false;
    }
    return true;
  }

  // One point of a loop trip: its tile slot and index, masks, and the
  // indices of its 2d face neighbours (the point's own index where a
  // neighbour does not exist, ok[] false), so that every load of a pass can
  // be issued without a branch and the trip costs one memory round trip.
  struct Tile {
    int slot, l;
    unsigned idx;
    bool comp, irr;
    unsigned ni[2 * DIM];
    bool ok[2 * DIM];
  };
  // Per-wave metadata of a trip (prefetched one trip ahead).
  struct Meta {
    uint64_t cw, iw;
    int nb[2 * DIM];
  };

  __device__ __forceinline__ void load_meta(Meta& m, int slot, int wt) const {
    m.cw = glb(P.g.comp_bits)[(size_t)slot * 4 + wt];
    m.iw = glb(P.g.irr_bits)[(size_t)slot * 4 + wt];
    gptr<const int> nbp = glb(P.g.nbr) + (size_t)slot * NBR_STRIDE;
#pragma unroll
    for (int d = 0; d < 2 * DIM; ++d) m.nb[d] = nbp[d];
  }

  __device__ __forceinline__ void make_tile(Tile& t, int slot, int l, const Meta& m) const {
    constexpr int X = TileShape<DIM>::X, Y = TileShape<DIM>::Y, Z = TileShape<DIM>::Z;
    t.slot = slot;
    t.l = l;
    t.idx = (unsigned)slot * TILE_PTS + l;
    t.comp = (m.cw >> (l & 63)) & 1ull;
    t.irr = t.comp && ((m.iw >> (l & 63)) & 1ull);
    const int lc[3] = {l % X, (l / X) % Y, l / (X * Y)};
    const int ext[3] = {X, Y, Z};
    const int str[3] = {1, X, X * Y};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      // -e_d: inside the tile, or the last layer of the neighbour tile
      const bool in_lo = lc[d] > 0;
      const int nlo = m.nb[2 * d];
      t.ok[2 * d] = in_lo || nlo >= 0;
      t.ni[2 * d] = in_lo ? t.idx - str[d]
                          : (nlo >= 0 ? (unsigned)nlo * TILE_PTS + l + str[d] * (ext[d] - 1) : t.idx);
      // +e_d: inside the tile, or the first layer of the neighbour tile
      const bool in_hi = lc[d] < ext[d] - 1;
      const int nhi = m.nb[2 * d + 1];
      t.ok[2 * d + 1] = in_hi || nhi >= 0;
      t.ni[2 * d + 1] = in_hi ? t.idx + str[d]
                              : (nhi >= 0 ? (unsigned)nhi * TILE_PTS + l - str[d] * (ext[d] - 1) : t.idx);
    }
  }

  // Metadata of loop trip r at `slot` for wave w (tile sub of the block):
  // from LDS for the first META_TRIPS trips, else from global memory.
  __device__ __forceinline__ void trip_meta(Meta& m, int r, int slot, int sub, int w) const {
    if (r < META_TRIPS) {
      m.cw = c.mcw[r][w];
      m.iw = c.miw[r][w];
#pragma unroll
      for (int d = 0; d < 2 * DIM; ++d) m.nb[d] = c.mnb[r][sub][d];
    } else {
      load_meta(m, slot, w & 3);
    }
  }

  // Fill the LDS metadata of this block's trips (once per launch).
  __device__ __forceinline__ void cache_meta() {
    const int stride = G * KTILES;
    const int sub = (int)(threadIdx.x / TILE_PTS);
    const int l = (int)(threadIdx.x % TILE_PTS);
    const int w = (int)(threadIdx.x >> 6);
    const int tb = tile_block();
    for (int r = 0; r < META_TRIPS; ++r) {
      const int slot = tb * KTILES + sub + r * stride;
      if (slot >= nact) break;
      if ((l & 63) == 0) {
        c.mcw[r][w] = glb(P.g.comp_bits)[(size_t)slot * 4 + (l >> 6)];
        c.miw[r][w] = glb(P.g.irr_bits)[(size_t)slot * 4 + (l >> 6)];
      }
      if (l < 2 * DIM) c.mnb[r][sub][l] = glb(P.g.nbr)[(size_t)slot * NBR_STRIDE + l];
      if (DIM == 2 && l >= 4 && l < 8) {
        // diagonal tile (-x-y, +x-y, -x+y, +x+y) through an existing face
        // neighbour (it matters only where one of them exists)
        const int fx = (l - 4) & 1, fy = 2 + ((l - 4) >> 1);
        const int nx = glb(P.g.nbr)[(size_t)slot * NBR_STRIDE + fx];
        const int ny = glb(P.g.nbr)[(size_t)slot * NBR_STRIDE + fy];
        int d = -1;
        if (nx >= 0) d = glb(P.g.nbr)[(size_t)nx * NBR_STRIDE + fy];
        else if (ny >= 0) d = glb(P.g.nbr)[(size_t)ny * NBR_STRIDE + fx];
        c.mnb[r][sub][l] = d;
      }
    }
    __syncthreads();
  }

  // Loop over the active tiles of this block (KTILES tiles per trip, one per
  // 256 threads); f(tile point).  Metadata comes from LDS or is prefetched a
  // trip ahead.  No block synchronisation inside: LDS is only read.
  template <class F>
  __device__ __forceinline__ void tiles(F&& f) {
    const int sub = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / TILE_PTS));
    const int l = (int)(threadIdx.x % TILE_PTS);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int stride = G * KTILES;
    int slot = tile_block() * KTILES + sub;
    if (threadIdx.x == 0 && lb == 0) { c.st.t_mark = wall_clock64(); region_start(c.st.t_mark); }
    Meta m;
    if (slot < nact) trip_meta(m, 0, slot, sub, w);
    for (int r = 0; slot < nact; ++r) {
      Tile t;
      make_tile(t, slot, l, m);
      const int next = slot + stride;
      if (next < nact) trip_meta(m, r + 1, next, sub, w);
      f(t);
      slot = next;
    }
  }

  // Variable beta: sum_f w_f v_f + dg v_p from the face values nv (order
  // -x,+x,-y,+y,-z,+z; a missing neighbour is a non-computational point,
  // whose value is 0) and the point's value vc.
  __device__ __forceinline__ double var_stencil(const Tile& t, const double (&nv)[2 * DIM], double vc) const {
    gptr<const double> w = glb(P.g.vcoef);
    double s = 0.0;
#pragma unroll
    for (int f = 0; f < 2 * DIM; ++f) s += t.ok[f] ? w[(size_t)f * P.g.vld + t.idx] * nv[f] : 0.0;
    return s + w[(size_t)(2 * DIM) * P.g.vld + t.idx] * vc;
  }

  // (A v) at the point: beta/h^2 (sum of neighbours - c_p v_p), 0 off the
  // computational points.
  __device__ __forceinline__ double Av(const Tile& t, gptr<const double> v) const {
    double nv[2 * DIM];
#pragma unroll
    for (int d = 0; d < 2 * DIM; ++d) nv[d] = v[t.ni[d]];
    const double vc = v[t.idx];
    if (P.g.vcoef) return t.comp ? var_stencil(t, nv, vc) : 0.0;
    const double cd = glb(P.g.cdiag)[t.irr ? t.idx : 0];
    __builtin_amdgcn_sched_barrier(0);
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 2 * DIM; ++d) s += t.ok[d] ? nv[d] : 0.0;
    const double cp = t.irr ? cd : (double)(2 * DIM);
    return t.comp ? P.g.coef * (s - cp * vc) : 0.0;
  }

  __device__ __forceinline__ double react(double u) const { return u * (P.ra - P.rb * u); }

  // F(U, t) at point i of state vector arr for stage time k (0: t_n,
  // 1: t_n + h/2, 2: t_n + h): the reaction, plus the caller's forcing G(t)
  // (source and Dirichlet boundary terms) in a forced step; with several
  // species the Lotka-Volterra reaction of the point's species, which reads
  // every species at the node (eq. 3.1 with u in R^m).
  __device__ __forceinline__ double Ft(gptr<const double> arr, size_t i, int k) const {
    const double u = arr[i];
    if (P.species > 1) {
      // species s of the point, and the same node in species 0
      const int s = (int)(i / sp_stride);
      const size_t base = i - (size_t)s * sp_stride;
      double acc = P.sa[s];
      for (int j = 0; j < P.species; ++j) acc -= P.sb[s * MAX_SPECIES + j] * arr[base + (size_t)j * sp_stride];
      return u * acc;
    }
    return P.forced ? react(u) + V(V_FG0 + k)[i] : react(u);
  }

  // ------------------------------------------------------------------ passes

  // W_k = A W_{k-1} + sum_l c_l b_{k+l}; at k == p also |W_p|^2 and |U|^2.
  __device__ __forceinline__ bool setup_pass(int k, int p, double tj, double tend, double (&out)[2]) {
    double cl[PMAX + 1];
    double fact = 1.0, tpow = 1.0;
#pragma unroll
    for (int l = 0; l <= PMAX; ++l) {
      if (l > 0) { fact *= l; tpow *= tj; }
      cl[l] = (l <= p - k) ? tpow / fact / pow(tend, (double)(k + l)) : 0.0;
    }
    gptr<const double> src = (k == 1) ? V(iu) : V(V_W1 + k - 2);
    gptr<double> dst = (k == p) ? V(V_Q0) : V(V_W1 + k - 1);
    double acc[2] = {0.0, 0.0};
    tiles([&](const Tile& t) {
      const bool comp = t.comp;
      const size_t i = t.idx;
      double w = 0.0;
      if (comp) {
        w = Av(t, src);
#pragma unroll
        for (int j = 0; j <= PMAX; ++j)
          if (j <= p - k) w += cl[j] * V(V_B0 + k + j)[i];
      }
      dst[i] = w;
      if (k == p) {
        const double u = V(iu)[i];
        acc[0] += w * w;
        acc[1] += u * u;
      }
    });
    add_bytes(24.0 + 8.0 * (p - k + 1));
    if (k == p) return finish<2>(acc, out);
    return barrier();
  }

  // p == 0: q_0 = U, norms.
  __device__ __forceinline__ bool copy_u_pass(double (&out)[2]) {
    double acc[2] = {0.0, 0.0};
    tiles([&](const Tile& t) {
      const bool comp = t.comp;
      const size_t i = t.idx;
      const double u = V(iu)[i];
      V(V_Q0)[i] = u;
      acc[0] += u * u;
      acc[1] += u * u;
    });
    add_bytes(16.0);
    return finish<2>(acc, out);
  }

  // Lanczos pass 0: z_0 = A q_0 into V_Z0; returns <z_0, q_0>.
  __device__ __forceinline__ bool lanczos_first(double& dot) {
    gptr<const double> q = V(V_Q0);
    gptr<double> z = V(V_Z0);
    double acc[1] = {0.0};
    tiles([&](const Tile& t) {
      const bool comp = t.comp;
      const size_t idx = t.idx;
      const double zz = Av(t, q);
      z[idx] = zz;
      acc[0] += zz * q[idx];
    });
    double out[1];
    if (!finish<1>(acc, out)) return false;
    dot = out[0];
    return true;
  }

  // Lanczos pass k >= 1: q_k from z_{k-1}, q_{k-1}, q_{k-2} (pointwise, also
  // at the face neighbours), written to V_Q0 + k; z_k = A q_k into
  // V_Z0 + (k & 1).  out = {|q_k|^2, <z_k, q_k>}.
  __device__ __forceinline__ bool lanczos_pass(int k, double (&out)[2]) {
    gptr<const double> zp = V(V_Z0 + ((k - 1) & 1));
    gptr<const double> q1 = V(V_Q0 + k - 1);
    gptr<const double> q2 = V(V_Q0 + (k >= 2 ? k - 2 : 0));
    gptr<double> qk = V(V_Q0 + k);
    gptr<double> zk = V(V_Z0 + (k & 1));
    const double alpha = c.alpha[k - 1];
    const double inv_n = 1.0 / c.nrm[k - 1];
    // k = 1: cm = 0 and q2 = q_0, so the last term is an exact 0 (no branch)
    const double cm = (k >= 2) ? c.nrm[k - 1] / c.nrm[k - 2] : 0.0;
    constexpr int NP = 2 * DIM + 1;   // the point (last) and its face neighbours
    double acc[2] = {0.0, 0.0};
    tiles([&](const Tile& t) {
      // every load of the point first (one memory round trip), then the math
      unsigned ix[NP];
#pragma unroll
      for (int d = 0; d < 2 * DIM; ++d) ix[d] = t.ni[d];
      ix[NP - 1] = t.idx;
      double a[NP], b[NP], e[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        a[j] = zp[ix[j]];
        b[j] = q1[ix[j]];
        e[j] = q2[ix[j]];
      }
      const double cd = glb(P.g.cdiag)[t.irr ? t.idx : 0];
      __builtin_amdgcn_sched_barrier(0);
      double qn[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j) qn[j] = (a[j] - alpha * b[j]) * inv_n - cm * e[j];
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < 2 * DIM; ++d) s += t.ok[d] ? qn[d] : 0.0;
      const double cp = t.irr ? cd : (double)(2 * DIM);
      const double q = t.comp ? qn[NP - 1] : 0.0;
      double z;
      if (P.g.vcoef) {
        double qf[2 * DIM];
#pragma unroll
        for (int d = 0; d < 2 * DIM; ++d) qf[d] = qn[d];
        z = t.comp ? var_stencil(t, qf, q) : 0.0;
      } else {
        z = t.comp ? P.g.coef * (s - cp * q) : 0.0;
      }
      qk[t.idx] = q;
      zk[t.idx] = z;
      acc[0] += q * q;
      acc[1] += z * q;
    });
    add_bytes(32.0);
    return finish<2>(acc, out);
  }

  // The same Lanczos pass with each tile and its face halo staged in LDS
  // (for blocks with several loop trips): every value of z_{k-1}, q_{k-1},
  // q_{k-2} in a tile is read from memory once per pass and its neighbours
  // from LDS, and the point values of the next trip are loaded one trip
  // ahead.  The staging buffers are the exponential's buffers (R, S; no
  // exponential runs during a pass).  Two block barriers per trip; every
  // block runs the same number of trips for all its tiles.
  __device__ __forceinline__ bool lanczos_lds(int k, double (&out)[2]) {
    constexpr int X = TileShape<DIM>::X, Y = TileShape<DIM>::Y, Z = TileShape<DIM>::Z;
    constexpr int EX = X + 2, EY = Y + 2, EZ = DIM == 3 ? Z + 2 : 1;
    constexpr int E = EX * EY * EZ;                       // staged box per array
    constexpr int NH = DIM == 2 ? 2 * (X + Y) : 2 * (X * Y + X * Z + Y * Z);   // face halo nodes
    constexpr int HR = (NH + TILE_PTS - 1) / TILE_PTS;   // halo nodes per thread
    constexpr int PS = DIM == 3 ? EX * EY : 0;            // z stride in the staged box
    static_assert(KTILES * 3 * E <= 2 * EXPM_NMAX * EXPM_NMAX, "staging exceeds the exponential buffers");
    // everything the loop reads from the parameters, hoisted (wave-uniform
    // registers; reads through the parameter reference in the loop would
    // wait for every load in flight)
    const gptr<const double> zp = uniform<const double>(V(V_Z0 + ((k - 1) & 1)));
    const gptr<const double> q1 = uniform<const double>(V(V_Q0 + k - 1));
    const gptr<const double> q2 = uniform<const double>(V(V_Q0 + (k >= 2 ? k - 2 : 0)));
    const gptr<double> qk = uniform<double>(V(V_Q0 + k));
    const gptr<double> zk = uniform<double>(V(V_Z0 + (k & 1)));
    const gptr<const double> cdiag = uniform<const double>(glb(P.g.cdiag));
    const double coef = uniform(P.g.coef);
    const double alpha = uniform(c.alpha[k - 1]);
    const double inv_n = uniform(1.0 / c.nrm[k - 1]);
    const double cm = uniform((k >= 2) ? c.nrm[k - 1] / c.nrm[k - 2] : 0.0);
    const int na = nact;
    const int sub = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / TILE_PTS));
    const int l = (int)(threadIdx.x % TILE_PTS);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lc[3] = {l % X, (l / X) % Y, l / (X * Y)};
    const lptr<double> Lz = lds(R) + (size_t)sub * 3 * E;
    const lptr<double> L1 = Lz + E;
    const lptr<double> L2 = L1 + E;
    const int pos = (lc[0] + 1) + EX * ((lc[1] + 1) + EY * (DIM == 3 ? lc[2] + 1 : 0));
    // this thread's halo nodes: face, index in the neighbour tile, staged position
    int hf[HR], hloc[HR], hpos[HR];
#pragma unroll
    for (int r = 0; r < HR; ++r) {
      int h = l + r * TILE_PTS;
      hf[r] = -1;
      hloc[r] = 0;
      hpos[r] = 0;
      if (h >= NH) continue;
      const int ext[3] = {X, Y, Z};
      int f = 0;
      for (; f < 2 * DIM; ++f) {
        const int d = f >> 1;
        const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
        const int cnt = ext[a] * (DIM == 3 ? ext[b] : 1);
        if (h < cnt) break;
        h -= cnt;
      }
      const int d = f >> 1;
      const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
      int cc[3] = {0, 0, 0};     // position in this tile's frame
      cc[a] = h % ext[a];
      cc[b] = DIM == 3 ? h / ext[a] : 0;
      cc[d] = (f & 1) ? ext[d] : -1;
      int nc[3] = {cc[0], cc[1], cc[2]};   // position in the neighbour tile
      nc[d] = (f & 1) ? 0 : ext[d] - 1;
      hf[r] = f;
      hloc[r] = nc[0] + X * (nc[1] + Y * nc[2]);
      hpos[r] = (cc[0] + 1) + EX * ((cc[1] + 1) + EY * (DIM == 3 ? cc[2] + 1 : 0));
    }
    const int stride = G * KTILES;
    const int base0 = tile_block() * KTILES;
    double acc[2] = {0.0, 0.0};
    if (threadIdx.x == 0 && lb == 0) { c.st.t_mark = wall_clock64(); region_start(c.st.t_mark); }
    // loads of trip r: the point and the halo nodes (0 where no tile)
    double pz, p1, p2, hz[HR], h1[HR], h2[HR];
    // metadata of trip r from the LDS cache (the caller uses this pass only
    // while every trip is cached)
    const lptr<const uint64_t> mcw = lds((const uint64_t*)&c.mcw[0][0]);
    const lptr<const uint64_t> miw = lds((const uint64_t*)&c.miw[0][0]);
    const lptr<const int> mnb = lds((const int*)&c.mnb[0][0][0]);
    auto meta = [&](Meta& m, int r, int) {
      m.cw = mcw[r * NWAVE + w];
      m.iw = miw[r * NWAVE + w];
#pragma unroll
      for (int d = 0; d < 2 * DIM; ++d) m.nb[d] = mnb[(r * KTILES + sub) * 8 + d];
    };
    // (every load is issued, at element 0 where there is nothing to read,
    // and the value selected afterwards: no branches, so the compiler can
    // count the loads in flight and wait only for the ones it needs)
    auto issue = [&](const Meta& m, int slot, bool valid) {
      const unsigned i = valid ? (unsigned)slot * TILE_PTS + (unsigned)l : 0u;
      const double a = at(zp, i), b = at(q1, i), e = at(q2, i);
      double ha[HR], hb[HR], he[HR];
      bool ok[HR];
#pragma unroll
      for (int r = 0; r < HR; ++r) {
        int ns = -1;
#pragma unroll
        for (int f = 0; f < 2 * DIM; ++f) ns = hf[r] == f ? m.nb[f] : ns;
        ok[r] = valid && hf[r] >= 0 && ns >= 0;
        const unsigned j = ok[r] ? (unsigned)ns * TILE_PTS + (unsigned)hloc[r] : 0u;
        ha[r] = at(zp, j);
        hb[r] = at(q1, j);
        he[r] = at(q2, j);
      }
      pz = valid ? a : 0.0;
      p1 = valid ? b : 0.0;
      p2 = valid ? e : 0.0;
#pragma unroll
      for (int r = 0; r < HR; ++r) {
        hz[r] = ok[r] ? ha[r] : 0.0;
        h1[r] = ok[r] ? hb[r] : 0.0;
        h2[r] = ok[r] ? he[r] : 0.0;
      }
    };
    if (base0 < na) {
      Meta m;
      int slot = base0 + sub;
      bool valid = slot < na;
      if (valid) meta(m, 0, slot);
      issue(m, slot, valid);
      for (int r = 0;; ++r) {
        // stage this trip's values
        __syncthreads();   // the previous trip's LDS reads are done
        Lz[pos] = pz;
        L1[pos] = p1;
        L2[pos] = p2;
#pragma unroll
        for (int q = 0; q < HR; ++q)
          if (hf[q] >= 0) {
            Lz[hpos[q]] = hz[q];
            L1[hpos[q]] = h1[q];
            L2[hpos[q]] = h2[q];
          }
        Tile t;
        if (valid) make_tile(t, slot, l, m);
        // the next trip's loads
        const int nslot = slot + stride;
        const bool more = base0 + (r + 1) * stride < na;
        const bool nvalid = nslot < na;
        Meta mn = m;
        if (nvalid) meta(mn, r + 1, nslot);
        // c_p: read at irregular points, element 0 elsewhere (no branch)
        const double cd = at(cdiag, (valid && t.irr) ? t.idx : 0u);
        issue(mn, nslot, nvalid);
        __syncthreads();
        if (valid) {
          constexpr int NS = 2 * DIM;
          const int off[6] = {-1, 1, -EX, EX, -PS, PS};
          double s = 0.0;
#pragma unroll
          for (int f = 0; f < NS; ++f) {
            const int pn = pos + off[f];
            s += (Lz[pn] - alpha * L1[pn]) * inv_n - cm * L2[pn];
          }
          const double qc = (Lz[pos] - alpha * L1[pos]) * inv_n - cm * L2[pos];
          const double cp = t.irr ? cd : (double)(2 * DIM);
          const double q = t.comp ? qc : 0.0;
          const double z = t.comp ? coef * (s - cp * q) : 0.0;
          put(qk, t.idx, q);
          put(zk, t.idx, z);
          acc[0] += q * q;
          acc[1] += z * q;
        }
        if (!more) break;
        slot = nslot;
        valid = nvalid;
        m = mn;
      }
      __syncthreads();   // LDS free for the exponential
    }
    add_bytes(32.0);
    return finish<2>(acc, out);
  }

  // 2D Lanczos pass without a stored A q, staged in LDS (large problems):
  // q_{k-1} is staged on the tile and a two-node halo (with the four
  // diagonal nodes), q_{k-2} and c_p on the tile and a one-node face halo;
  // A q_{k-1} and then q_k follow on the tile and its face halo, and
  // A q_k at the tile's points.  Reads q_{k-1}, q_{k-2}, c_p and writes q_k:
  // 32 B per unknown from memory, the count of the measurement plan (the
  // stored-A q pass moves 40 B).  c_p doubles as the computational mask
  // (NOT_COMP elsewhere).  The q_k buffer alternates between two LDS halves
  // by trip parity, so two block barriers per trip suffice.
  __device__ __forceinline__ bool lanczos_zf2(int k, double (&out)[2]) {
    if (threadIdx.x == 0 && lb == 0) { c.st.t_mark = wall_clock64(); region_start(c.st.t_mark); }
    double acc[2];
    zf2_loop(uniform<const double>(V(V_Q0 + k - 1)), uniform<const double>(V(V_Q0 + (k >= 2 ? k - 2 : 0))),
             uniform<double>(V(V_Q0 + k)), uniform<const double>(glb(P.g.cdiag)), P.g.coef, c.alpha[k - 1],
             1.0 / c.nrm[k - 1], (k >= 2) ? c.nrm[k - 1] / c.nrm[k - 2] : 0.0, nact, G, tile_block(), lds(R),
             lds((const int*)&c.mnb[0][0][0]), acc);
    add_bytes(32.0);
    return finish<2>(acc, out);
  }

  // out = sum_{k<p} tau^k/k! W_k + sum_i coef_i q_i into vector out_vec
  // (default: the buffer that is not iu); returns |out|^2 in nn.
  __device__ __forceinline__ bool combine_pass(int p, int m, double tau, double& nn, int out_vec = -1) {
    double ck[PMAX];
    double f = 1.0, tp = 1.0;
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      if (k > 0) { f *= k; tp *= tau; }
      ck[k] = tp / f;
    }
    const int io = out_vec >= 0 ? out_vec : ((iu == V_U) ? V_T : V_U);
    double acc[1] = {0.0};
    tiles([&](const Tile& t) {
      const bool comp = t.comp;
      const size_t idx = t.idx;
      double u = 0.0;
      if (comp) {
        if (p > 0) {
          u = V(iu)[idx];
#pragma unroll
          for (int k = 1; k < PMAX; ++k)
            if (k < p) u += ck[k] * V(V_W1 + k - 1)[idx];
        }
        // eight independent partial sums keep eight basis loads in flight
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, s5 = 0.0, s6 = 0.0, s7 = 0.0;
        int j = 0;
        for (; j + 8 <= m; j += 8) {
          s0 += c.coef[j] * V(V_Q0 + j)[idx];
          s1 += c.coef[j + 1] * V(V_Q0 + j + 1)[idx];
          s2 += c.coef[j + 2] * V(V_Q0 + j + 2)[idx];
          s3 += c.coef[j + 3] * V(V_Q0 + j + 3)[idx];
          s4 += c.coef[j + 4] * V(V_Q0 + j + 4)[idx];
          s5 += c.coef[j + 5] * V(V_Q0 + j + 5)[idx];
          s6 += c.coef[j + 6] * V(V_Q0 + j + 6)[idx];
          s7 += c.coef[j + 7] * V(V_Q0 + j + 7)[idx];
        }
        for (; j < m; ++j) s0 += c.coef[j] * V(V_Q0 + j)[idx];
        u += ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7));
      }
      V(io)[idx] = u;
      acc[0] += u * u;
    });
    add_bytes(8.0 * (m + p + 1));
    double out[1];
    if (!finish<1>(acc, out)) return false;
    nn = out[0];
    return true;
  }

  // --------------------------------------------------------- small expm

  // E = exp(X) in R, X the augmented matrix of size N = m + p + 1 built
  // from tau, alpha[0..m-1], nrm[1..m-1], by the whole block (one wave alone
  // was measured 2.5x slower: too few loads in flight per Horner step).
  __device__ __forceinline__ void expm_aug(int m, int p, double tau) {
    const unsigned long long t_in = wall_clock64();
    if (threadIdx.x == 0 && lb == 0) region_start(t_in);
    expm_run(m, p, tau, (int)threadIdx.x, (int)blockDim.x);
    __syncthreads();
    if (threadIdx.x == 0 && lb == 0) c.st.tk_expm += wall_clock64() - t_in;
  }

  // Scaling, Taylor-Horner and squaring by threads first, first + stride, ...
  __device__ __forceinline__ void expm_run(int m, int p, double tau, int first, int stride) {
    auto step_sync = [&]() { __syncthreads(); };
    const int N = m + p + 1;
    // 1-norm of X (column sums)
    if (first == 0) {
      double nx = 1.0;
      for (int j = 0; j < m; ++j) {
        double s = fabs(c.alpha[j]);
        if (j > 0) s += c.nrm[j];
        if (j < m - 1) s += c.nrm[j + 1];
        nx = fmax(nx, tau * s);
      }
      c.red[0] = nx;
    }
    step_sync();
    const double nx = c.red[0];
    int sq = 0;
    if (nx > 1.0) sq = (int)ceil(log2(nx));
    const double scale = ldexp(1.0, -sq);
    const int NN = N * N;
    for (int e = first; e < NN; e += stride) R[e] = ((e / N) == (e % N)) ? 1.0 : 0.0;
    step_sync();
    double* A = R;
    double* B = S;
    constexpr int K = 20;
    for (int k = K; k >= 1; --k) {
      const double f = scale / (double)k;
      for (int e = first; e < NN; e += stride) {
        const int i = e / N, j = e % N;
        double xr;
        if (i < m) {
          xr = c.alpha[i] * A[i * N + j];
          if (i > 0) xr += c.nrm[i] * A[(i - 1) * N + j];
          if (i < m - 1) xr += c.nrm[i + 1] * A[(i + 1) * N + j];
          xr *= tau;
          if (i == 0) xr += A[m * N + j];
        } else if (i < m + p) {
          xr = A[(i + 1) * N + j];
        } else {
          xr = 0.0;
        }
        B[e] = ((i == j) ? 1.0 : 0.0) + f * xr;
      }
      step_sync();
      double* t = A; A = B; B = t;
    }
    for (int s = 0; s < sq; ++s) {
      for (int e = first; e < NN; e += stride) {
        const int i = e / N, j = e % N;
        double acc = 0.0;
        // lower-left block (rows >= m, cols < m) of every power is zero
        const int l0 = (i >= m) ? m : 0;
        for (int l = l0; l < N; ++l) acc += A[i * N + l] * A[l * N + j];
        B[e] = acc;
      }
      step_sync();
      double* t = A; A = B; B = t;
    }
    if (A != R) {
      for (int e = first; e < NN; e += stride) R[e] = A[e];
      step_sync();
    }
  }

  // ------------------------------------------------------------ phi combo

  // V_U <- sum_{k=0}^{p} phi_k(tend A) b_k with b_0 in vector b0 (not
  // written) and b_k (k>=1) in V_B0 + k.  The substeps alternate between
  // V_U and V_T, starting with V_U, so a single substep needs no copy.
  // With 0 < t_mid <= tend, also the solution of the same ODE at t_mid,
  // y(t_mid) = sum_k phi_k(t_mid A) (t_mid/tend)^k b_k, into vector
  // mid_vec: from the Krylov basis of the substep that contains t_mid
  // (simultaneous output, no extra Lanczos passes: one more small
  // exponential at s = t_mid - t_j and one combine pass; the error
  // estimate at s must pass the same two tests).
  // Returns false on failure (status set).
  __device__ __forceinline__ bool phi_comb(int p, double tend, int b0, double t_mid = 0.0, int mid_vec = -1) {
    iu = b0;
    if (mid_vec < 0 || !(t_mid > 0.0)) t_mid = 0.0;
    if (tend == 0.0) {
      // phi_k(0) = 1/k!
      double f = 1.0;
      double ck[PMAX + 1];
#pragma unroll
      for (int k = 0; k <= PMAX; ++k) { if (k > 0) f *= k; ck[k] = 1.0 / f; }
      tiles([&](const Tile& t) {
        const size_t idx = t.idx;
        double u = V(iu)[idx];
#pragma unroll
        for (int k = 1; k <= PMAX; ++k)
          if (k <= p) u += ck[k] * V(V_B0 + k)[idx];
        V(V_U)[idx] = t.comp ? u : 0.0;
      });
      add_bytes(8.0 * (p + 2));
      iu = V_U;
      return barrier() && (t_mid == 0.0 || copy_pass(mid_vec, V_U));
    }
    const double tol = P.tol;
    double tj = 0.0;
    double tau = tend * c.tau_frac[p];
    int m_target = c.m_guess[p];
    int nsub = 0;
    bool shrunk_any = false;
    double fact_p = 1.0;
    for (int k = 2; k <= p; ++k) fact_p *= k;
    while (tj < tend) {
      if (nsub >= P.max_substeps) { fail(ST_KRYLOV); return false; }
      tau = fmin(tau, tend - tj);
      if (tend - tj - tau <= 1e-13 * tend) tau = tend - tj;
      // setup: W_1..W_p, q_0 = W_p, norms
      double nrm2[2];
      if (p == 0) {
        if (!copy_u_pass(nrm2)) return false;
      } else {
        for (int k = 1; k <= p; ++k) {
          double o[2];
          if (!setup_pass(k, p, tj, tend, o)) return false;
          if (k == p) { nrm2[0] = o[0]; nrm2[1] = o[1]; }
        }
        count(c.st.matvecs, p);
      }
      const double n0 = sqrt(nrm2[0]);
      const double unorm = sqrt(nrm2[1]);
      // this substep holds t_mid strictly inside: the output at s = t_mid - t_j
      const bool mid_in = t_mid > tj && t_mid < tj + tau - 1e-13 * tend;
      if (n0 == 0.0) {
        // W_p = 0: the Krylov term vanishes exactly.
        double nn;
        if (mid_in && !combine_pass(p, 0, t_mid - tj, nn, mid_vec)) return false;
        if (!combine_pass(p, 0, tau, nn)) return false;
        iu = (iu == V_U) ? V_T : V_U;
        if (t_mid > tj && !mid_in && t_mid <= tj + tau + 1e-13 * tend && !copy_pass(mid_vec, iu)) return false;
        tj += tau;
        ++nsub;
        continue;
      }
      if (threadIdx.x == 0) c.nrm[0] = n0;
      __syncthreads();
      int m = 0;
      bool started = false;   // Lanczos pass 0 done for this substep
      bool breakdown = false;
      double anorm = 0.0;
      bool shrunk = false;
      double err = 0.0, tol_loc = 0.0;
      // error estimate of the current (m, tau); fills R with exp(X)
      auto estimate = [&]() -> bool {
        expm_aug(m, p, tau);
        count(c.st.expms, 1);
        const int N = m + p + 1;
        const double phi_next_m = R[(m - 1) * N + (m + p)];
        double taup = 1.0;
        for (int k = 0; k < p; ++k) taup *= tau;
        err = breakdown ? 0.0 : n0 * c.nrm[m] * taup * tau * fabs(phi_next_m);
        const double ref = fmax(unorm, taup * n0 / fact_p);
        tol_loc = tol * (tau / tend) * fmax(ref, 1e-300);
        __syncthreads();
        if (!isfinite(err)) { fail(ST_NONFINITE); return false; }
        return true;
      };
      // tau^p |W_p| [phi_p(tau T) e_1]_j / n_j, from R = exp(X)
      auto set_coef = [&]() {
        const int N = m + p + 1;
        const int col = (p >= 1) ? (m + p - 1) : 0;
        double taup = 1.0;
        for (int k = 0; k < p; ++k) taup *= tau;
        if (threadIdx.x == 0)
          for (int j = 0; j < m; ++j) c.coef[j] = taup * n0 * R[j * N + col] / c.nrm[j];
        __syncthreads();
      };
      // Refine after a rejection with error ratio r > 1: more Krylov vectors
      // while m < m_max, else a smaller tau.  Returns false on failure.
      auto refine = [&](double r) -> bool {
        if (m < P.m_max && !breakdown) {
          count(c.st.rejected, 1);
          m_target = min(m + P.m_step, P.m_max);
          return true;
        }
        double fac = 0.9 * pow(r, -1.0 / (double)(m + 1));
        fac = fmin(0.9, fmax(0.1, fac));
        tau *= fac;
        shrunk = true;
        count(c.st.rejected, 1);
        if (tau < 1e-12 * tend) { fail(ST_KRYLOV); return false; }
        return true;
      };
      bool accept = false;
      int tries = 0;
      while (!accept) {
        if (++tries > 400) { fail(ST_KRYLOV); return false; }
        while (m < m_target && !breakdown) {
          if (m == 0 && !started) {
            double dot;
            if (!lanczos_first(dot)) return false;
            count(c.st.matvecs, 1);
            if (threadIdx.x == 0) c.alpha[0] = dot / (n0 * n0);
            __syncthreads();
            started = true;
          }
          double o[2];
          // large vectors, several loop trips per block, all with cached
          // metadata: the LDS-staged pass
          const bool staged = nact >= P.stage_min && nact > G * KTILES && nact <= G * KTILES * META_TRIPS &&
                              P.g.vcoef == nullptr;
          bool ok;
          if (staged && DIM == 2) ok = lanczos_zf2(m + 1, o);
          else if (staged) ok = lanczos_lds(m + 1, o);
          else ok = lanczos_pass(m + 1, o);
          if (!ok) return false;
          count(c.st.matvecs, 1);
          const double nb = sqrt(o[0]);
          const double alpha_next = (o[0] > 0.0) ? o[1] / o[0] : 0.0;
          anorm = fmax(anorm, fabs(c.alpha[m]) + nb + (m > 0 ? c.nrm[m] : 0.0));
          // entries m + 1 are read by no thread before the barrier below
          if (threadIdx.x == 0) {
            c.nrm[m + 1] = nb;
            c.alpha[m + 1] = alpha_next;
          }
          __syncthreads();
          ++m;
          if (nb <= 1e-13 * anorm) breakdown = true;
        }
        if (!estimate()) return false;
        // first test against the input scale (no pass needed)
        if (err > tol_loc) {
          if (!refine(err / tol_loc)) return false;
          continue;
        }
        // then against the norm of the candidate output
        set_coef();
        double nn_out;
        if (!combine_pass(p, m, tau, nn_out)) return false;
        const double tol_out = tol * (tau / tend) * fmax(sqrt(nn_out), 1e-300);
        if (err > tol_out) {
          if (!refine(err / tol_out)) return false;
          continue;
        }
        // (tau may have shrunk since the substep began)
        if (t_mid > tj && t_mid < tj + tau - 1e-13 * tend) {
          // the intermediate output from the same basis, with the same tests
          const double tau_full = tau, err_full = err;
          tau = t_mid - tj;
          if (!estimate()) return false;
          const double ratio_in = err / tol_loc;
          double ratio_out = 0.0;
          if (ratio_in <= 1.0) {
            set_coef();
            double nn_mid;
            if (!combine_pass(p, m, tau, nn_mid, mid_vec)) return false;
            ratio_out = err / (tol * (tau / tend) * fmax(sqrt(nn_mid), 1e-300));
          }
          tau = tau_full;
          err = err_full;
          const double ratio = fmax(ratio_in, ratio_out);
          if (ratio > 1.0) {
            if (!refine(ratio)) return false;
            continue;
          }
        }
        accept = true;
      }
      iu = (iu == V_U) ? V_T : V_U;
      // t_mid at the end of this substep: the output is the substep's result
      if (t_mid > tj && t_mid >= tj + tau - 1e-13 * tend && t_mid <= tj + tau + 1e-13 * tend &&
          !copy_pass(mid_vec, iu))
        return false;
      if (threadIdx.x == 0) {
        c.st.m_last = m;
        c.st.err_est = err;
        c.st.ratio_last = err / fmax(tol_loc, 1e-300);
      }
      tj += tau;
      ++nsub;
      shrunk_any |= shrunk;
      // next substep: keep tau after a shrink, else try the whole remainder
      if (!shrunk) tau = tend;
      m_target = max(P.m_min, m);
    }
    if (iu != V_U) {
      if (!copy_pass(V_U, iu)) return false;
      iu = V_U;
    }
    count(c.st.substeps, nsub);
    __syncthreads();
    if (threadIdx.x == 0) {
      // the next call starts at the dimension that passed, one lower when
      // it passed with a wide margin
      c.m_guess[p] = max(P.m_min, min(P.m_max, c.st.ratio_last < 1e-2 ? c.st.m_last - 1 : c.st.m_last));
      c.tau_frac[p] = shrunk_any ? fmin(1.0, 1.25 * tau / tend) : 1.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) c.st.t_done = tj;
    return true;
  }

  // ------------------------------------------------------------ jobs

  __device__ __forceinline__ bool copy_pass(int dst, int src) {
    tiles([&](const Tile& t) {
      const bool comp = t.comp;
      const size_t idx = t.idx;
      V(dst)[idx] = comp ? V(src)[idx] : 0.0;
    });
    add_bytes(16.0);
    return barrier();
  }

  __device__ __forceinline__ double dreact(double u) const { return P.ra - 2.0 * P.rb * u; }

  // Number of phi-combinations of a job.
  __device__ __forceinline__ int stages(int mode) const {
    switch (mode) {
      case JOB_ETD2RK: return 2;
      case JOB_ETD2: return P.first ? 2 : 1;
      case JOB_ETD3RK: return 3;
      case JOB_ETD4RK: return 4;
      case JOB_ETD3RK_SIMUL: return 3;
      case JOB_ETD4RK_SIMUL: return 4;
      case JOB_ADJ_ETD2RK: return 6;
      default: return 1;
    }
  }

  // Pointwise pass over the computational points: f(idx) at every point of
  // the active tiles (f sees comp), then a barrier.
  template <class F>
  __device__ __forceinline__ bool pointwise(double bytes, F&& f) {
    tiles([&](const Tile& t) { f(t.idx, t.comp); });
    add_bytes(bytes);
    return barrier();
  }

  // <V(vb), A V(va)> over the unknowns.
  __device__ __forceinline__ bool dot_A_pass(int va, int vb, double& out) {
    gptr<const double> a = V(va);
    gptr<const double> b = V(vb);
    double acc[1] = {0.0};
    tiles([&](const Tile& t) {
      const bool comp = t.comp;
      const size_t idx = t.idx;
      acc[0] += b[idx] * Av(t, a);
    });
    add_bytes(16.0);
    double o[1];
    if (!finish<1>(acc, o)) return false;
    out = o[0];
    return true;
  }

  // Inputs of stage `stage` of the job: b_0 in vector b0 and b_k = V_B0 + k
  // (k >= 1) of the combination sum_k phi_k(t A) b_k, its p and t.
  //
  // Adjoint of ETD2RK (A symmetric, A = beta A_1, g = dL/dU_{n+1},
  // F = f(U_n), a the stage, abar = f'(a) h phi_2 g):
  //   stage 0: a = phi_0 U_n + phi_1 hF                   -> V_A
  //   stage 1: phi_2 g                                    -> abar in V_AB
  //   stage 2: v_s = phi_0 U_n + phi_1 hF - phi_2 hF      -> <abar, A v_s>
  //   stage 3: v_f = phi_0 U_n + phi_1 hF + phi_2 (h(f(a)-F) - hF)
  //                  - phi_3 2h(f(a)-F)                   -> <g, A v_f>
  //   stage 4: s = phi_1 h(g + abar) - phi_2 hg           -> f'(U_n) s in V_S
  //   stage 5: phi_0 (g + abar); + V_S                    -> dL/dU_n in V_U
  // and dL/dbeta += (h/beta)(<g, A v_f> + <abar, A v_s>), from
  // d/dbeta phi_k(h beta A_1) = (h/beta) A (phi_k - k phi_{k+1})(hA).
  __device__ __forceinline__ bool assemble(int mode, int stage, int& p, double& t, int& b0) {
    st_tmid = 0.0;
    st_midvec = -1;
    if (mode == JOB_PHI) {
      // the gathered inputs are in place
      p = P.p;
      t = P.t;
      b0 = V_B0;
      if (P.t_mid > 0.0) {
        st_tmid = P.t_mid;
        st_midvec = V_F;
      }
      return true;
    }
    const double h = P.h;
    t = h;
    b0 = V_X0;
    gptr<double> U = V(V_U);
    gptr<double> T0 = V(V_T);
    gptr<double> B1 = V(V_B1);
    gptr<double> B2 = V(V_B2);
    gptr<double> B3 = V(V_B3);
    gptr<const double> X = V(V_X0);
    gptr<const double> G = V(V_G);
    gptr<const double> Aa = V(V_A);
    gptr<const double> AB = V(V_AB);
    if (mode == JOB_ADJ_ETD2RK) {
      // b_0 in V_T (stages 1, 4, 5) or U_n itself
      b0 = (stage == 1 || stage == 4 || stage == 5) ? V_T : V_X0;
      switch (stage) {
        case 0:
        case 2:
        case 3:
          p = (stage == 0) ? 1 : (stage == 2 ? 2 : 3);
          return pointwise(stage == 0 ? 16.0 : (stage == 2 ? 24.0 : 40.0), [&](size_t i, bool comp) {
            const double u = comp ? X[i] : 0.0;
            const double hF = comp ? h * react(u) : 0.0;
            B1[i] = hF;
            if (stage == 2) B2[i] = -hF;
            if (stage == 3) {
              const double d = comp ? h * (react(Aa[i]) - react(u)) : 0.0;
              B2[i] = d - hF;
              B3[i] = -2.0 * d;
            }
          });
        case 1:
          p = 2;
          return pointwise(32.0, [&](size_t i, bool comp) {
            T0[i] = 0.0;
            B1[i] = 0.0;
            B2[i] = comp ? G[i] : 0.0;
          });
        case 4:
          p = 2;
          return pointwise(40.0, [&](size_t i, bool comp) {
            const double g = comp ? G[i] : 0.0;
            T0[i] = 0.0;
            B1[i] = comp ? h * (g + AB[i]) : 0.0;
            B2[i] = -h * g;
          });
        default:
          p = 0;
          return pointwise(24.0, [&](size_t i, bool comp) { T0[i] = comp ? G[i] + AB[i] : 0.0; });
      }
    }
    if (mode == JOB_ETD3RK_SIMUL || mode == JOB_ETD4RK_SIMUL) {
      // The same schemes with the ODE y' = A y + F_n, y(0) = U_n integrated
      // once over h: its value at h/2 is stage a (simultaneous output from
      // the same Krylov basis) and its value e at h is the phi_0, phi_1 part
      // of the final combination; the remaining stages are combinations
      // with b_0 = 0 added to e or a (V_S holds the zero vector, V_F keeps e):
      //   ETD3RK: b = e + phi_1(hA) 2h (F(a) - F_n)
      //   ETD4RK: b = a + phi_1(hA/2) (h/2) (F(a) - F_n);  c as before
      //   final  = e + phi_2 h (...) + phi_3 2h (...)   (as in the standard form)
      const bool four = mode == JOB_ETD4RK_SIMUL;
      gptr<double> Zv = V(V_S);
      if (stage == 0) {
        p = 1;
        st_tmid = 0.5 * h;
        st_midvec = V_A;
        return pointwise(16.0, [&](size_t i, bool comp) { B1[i] = comp ? h * Ft(X, i, 0) : 0.0; });
      }
      if (stage == 1) {
        p = 1;
        b0 = V_S;
        const double sc = four ? 0.5 * h : 2.0 * h;
        if (four) t = 0.5 * h;
        return pointwise(24.0, [&](size_t i, bool comp) {
          Zv[i] = 0.0;
          B1[i] = comp ? sc * (Ft(Aa, i, 1) - Ft(X, i, 0)) : 0.0;
        });
      }
      if (four && stage == 2) {
        p = 1;
        t = 0.5 * h;
        b0 = V_A;
        return pointwise(24.0, [&](size_t i, bool comp) {
          B1[i] = comp ? 0.5 * h * (2.0 * Ft(AB, i, 1) - Ft(X, i, 0)) : 0.0;
        });
      }
      p = 3;
      b0 = V_S;
      if (!four) {
        return pointwise(48.0, [&](size_t i, bool comp) {
          const double fn = comp ? Ft(X, i, 0) : 0.0, fa = comp ? Ft(Aa, i, 1) : 0.0;
          const double fb = comp ? Ft(U, i, 2) : 0.0;
          B1[i] = 0.0;
          B2[i] = h * (-3.0 * fn + 4.0 * fa - fb);
          B3[i] = 2.0 * h * (2.0 * fn - 4.0 * fa + 2.0 * fb);
        });
      }
      return pointwise(56.0, [&](size_t i, bool comp) {
        const double fn = comp ? Ft(X, i, 0) : 0.0, fab = comp ? Ft(Aa, i, 1) + Ft(AB, i, 1) : 0.0;
        const double fc = comp ? Ft(U, i, 2) : 0.0;
        B1[i] = 0.0;
        B2[i] = h * (-3.0 * fn + 2.0 * fab - fc);
        B3[i] = 2.0 * h * (2.0 * fn - 2.0 * fab + 2.0 * fc);
      });
    }
    if (mode == JOB_ETD3RK || mode == JOB_ETD4RK) {
      // ETD3RK (F_n = F(U_n), stage results a, b (, c)):
      //   a = phi_0(h/2) U_n + phi_1(h/2) (h/2) F_n             -> V_A
      //   b = phi_0 U_n + phi_1 h (2 F(a) - F_n)                  (in V_U)
      //   U+ = phi_0 U_n + phi_1 h F_n + phi_2 h (-3F_n + 4F(a) - F(b))
      //        + phi_3 2h (2F_n - 4F(a) + 2F(b))
      // ETD4RK:
      //   a = phi_0(h/2) U_n + phi_1(h/2) (h/2) F_n             -> V_A
      //   b = phi_0(h/2) U_n + phi_1(h/2) (h/2) F(a)            -> V_AB
      //   c = phi_0(h/2) a + phi_1(h/2) (h/2) (2F(b) - F_n)       (in V_U)
      //   U+ = phi_0 U_n + phi_1 h F_n + phi_2 h (-3F_n + 2(F(a)+F(b)) - F(c))
      //        + phi_3 2h (2F_n - 2(F(a)+F(b)) + 2F(c))
      // (phi_3 standard; the paper's unnormalised phi_3 is 2 phi_3)
      const int last = stages(mode) - 1;
      if (stage < last) {
        p = 1;
        if (mode == JOB_ETD3RK && stage == 1) {
          return pointwise(24.0, [&](size_t i, bool comp) {
            B1[i] = comp ? h * (2.0 * Ft(Aa, i, 1) - Ft(X, i, 0)) : 0.0;
          });
        }
        t = 0.5 * h;
        if (stage == 0)
          return pointwise(16.0, [&](size_t i, bool comp) { B1[i] = comp ? 0.5 * h * Ft(X, i, 0) : 0.0; });
        if (stage == 1)
          return pointwise(16.0, [&](size_t i, bool comp) { B1[i] = comp ? 0.5 * h * Ft(Aa, i, 1) : 0.0; });
        b0 = V_A;   // ETD4RK c starts from a
        return pointwise(24.0, [&](size_t i, bool comp) {
          B1[i] = comp ? 0.5 * h * (2.0 * Ft(AB, i, 1) - Ft(X, i, 0)) : 0.0;
        });
      }
      p = 3;
      if (mode == JOB_ETD3RK) {
        return pointwise(48.0, [&](size_t i, bool comp) {
          const double fn = comp ? Ft(X, i, 0) : 0.0, fa = comp ? Ft(Aa, i, 1) : 0.0;
          const double fb = comp ? Ft(U, i, 2) : 0.0;
          B1[i] = h * fn;
          B2[i] = h * (-3.0 * fn + 4.0 * fa - fb);
          B3[i] = 2.0 * h * (2.0 * fn - 4.0 * fa + 2.0 * fb);
        });
      }
      return pointwise(56.0, [&](size_t i, bool comp) {
        const double fn = comp ? Ft(X, i, 0) : 0.0, fab = comp ? Ft(Aa, i, 1) + Ft(AB, i, 1) : 0.0;
        const double fc = comp ? Ft(U, i, 2) : 0.0;
        B1[i] = h * fn;
        B2[i] = h * (-3.0 * fn + 2.0 * fab - fc);
        B3[i] = 2.0 * h * (2.0 * fn - 2.0 * fab + 2.0 * fc);
      });
    }
    if (mode == JOB_ETD2 && stage == 0) {
      // ETD2 multistep: b_0 = U_n, b_1 = h F_n, b_2 = h (F_n - F_{n-1}),
      // F_{n-1} read from V_G, which then keeps F_n for the next step.  The
      // first step (no F_{n-1}) is an ETD2RK step; it stores F_n as well.
      gptr<double> Gw = V(V_G);
      const bool first = P.first != 0;
      p = first ? 1 : 2;
      return pointwise(first ? 24.0 : 40.0, [&](size_t i, bool comp) {
        const double fn = comp ? Ft(X, i, 0) : 0.0;
        B1[i] = h * fn;
        if (!first) B2[i] = h * (fn - (comp ? Gw[i] : 0.0));
        Gw[i] = fn;
      });
    }
    if (stage == 0) {
      // ETD1 / first ETD2RK stage: b_0 = U_n, b_1 = h F(U_n)
      p = 1;
      return pointwise(16.0, [&](size_t i, bool comp) { B1[i] = comp ? h * Ft(X, i, 0) : 0.0; });
    }
    // ETD2RK final stage: b_0 = U_n, b_1 = h F(U_n), b_2 = h (F(a) - F(U_n)),
    // a = the first stage (in V_U, overwritten once b_2 is formed)
    p = 2;
    return pointwise(24.0, [&](size_t i, bool comp) {
      B2[i] = comp ? h * (Ft(U, i, 2) - Ft(X, i, 0)) : 0.0;
    });
  }

  // What a stage leaves behind once its combination is in V_U.
  __device__ __forceinline__ bool post(int mode, int stage, double& dsum) {
    if (mode == JOB_ETD3RK_SIMUL || mode == JOB_ETD4RK_SIMUL) {
      const bool four = mode == JOB_ETD4RK_SIMUL;
      gptr<double> U = V(V_U);
      gptr<double> E = V(V_F);
      const int last = stages(mode) - 1;
      if (stage == 0) return pointwise(16.0, [&](size_t i, bool comp) { E[i] = U[i]; });   // e
      if (stage == 1 && !four) return pointwise(24.0, [&](size_t i, bool comp) { U[i] += E[i]; });   // b
      if (stage == 1) {
        gptr<const double> Aa = V(V_A);
        gptr<double> AB = V(V_AB);
        return pointwise(32.0, [&](size_t i, bool comp) {   // b = a + ..., kept for c and the final
          const double b = U[i] + Aa[i];
          U[i] = b;
          AB[i] = b;
        });
      }
      if (stage == last) return pointwise(24.0, [&](size_t i, bool comp) { U[i] += E[i]; });   // U_{n+1}
      return true;
    }
    if (mode == JOB_ETD3RK || mode == JOB_ETD4RK) {
      // keep a (and ETD4RK's b) for the later stages
      gptr<const double> U = V(V_U);
      if (stage == 0) {
        gptr<double> Aa = V(V_A);
        return pointwise(16.0, [&](size_t i, bool comp) { Aa[i] = U[i]; });
      }
      if (mode == JOB_ETD4RK && stage == 1) {
        gptr<double> AB = V(V_AB);
        return pointwise(16.0, [&](size_t i, bool comp) { AB[i] = U[i]; });
      }
      return true;
    }
    if (mode != JOB_ADJ_ETD2RK) return true;
    const double h = P.h;
    gptr<double> U = V(V_U);
    switch (stage) {
      case 0: {
        gptr<double> Aa = V(V_A);
        return pointwise(16.0, [&](size_t i, bool comp) { Aa[i] = U[i]; });
      }
      case 1: {
        gptr<double> AB = V(V_AB);
        gptr<const double> Aa = V(V_A);
        return pointwise(24.0, [&](size_t i, bool comp) { AB[i] = comp ? dreact(Aa[i]) * h * U[i] : 0.0; });
      }
      case 2:
      case 3: {
        double d = 0.0;
        if (!dot_A_pass(V_U, stage == 2 ? V_AB : V_G, d)) return false;
        dsum += d;
        return true;
      }
      case 4: {
        gptr<double> Sv = V(V_S);
        gptr<const double> X = V(V_X0);
        return pointwise(24.0, [&](size_t i, bool comp) { Sv[i] = comp ? dreact(X[i]) * U[i] : 0.0; });
      }
      default: {
        gptr<const double> Sv = V(V_S);
        return pointwise(24.0, [&](size_t i, bool comp) { U[i] = comp ? U[i] + Sv[i] : 0.0; });
      }
    }
  }

  __device__ __forceinline__ void run(unsigned long long t_start) {
    cache_meta();
    if (threadIdx.x == 0 && lb == 0) c.st.tk_pro = wall_clock64() - t_start;
    const int mode = P.mode;
    if (mode == JOB_APPLY) {
      tiles([&](const Tile& t) {
      const bool comp = t.comp;
        const size_t idx = t.idx;
        V(V_U)[idx] = Av(t, V(V_B0));
      });
      add_bytes(16.0);
      barrier();
      return;
    }
    if (mode != JOB_PHI && mode != JOB_ETD1 && mode != JOB_ETD2RK && mode != JOB_ETD2RK_STAGE &&
        mode != JOB_ADJ_ETD2RK && mode != JOB_ETD3RK && mode != JOB_ETD4RK && mode != JOB_ETD2 &&
        mode != JOB_ETD3RK_SIMUL && mode != JOB_ETD4RK_SIMUL) {
      if (threadIdx.x == 0 && lb == 0) atomicCAS(P.status, 0, ST_INVALID);
      return;
    }
    // one phi_comb call site for every job (keeps the engine inlined)
    const int nstage = stages(mode);
    double dsum = 0.0;
    for (int stage = 0; stage < nstage; ++stage) {
      int p = 0, b0 = V_U;
      double t = 0.0;
      if (!assemble(mode, stage, p, t, b0)) return;
      if (!phi_comb(p, t, b0, st_tmid, st_midvec)) return;
      if (!post(mode, stage, dsum)) return;
    }
    if (mode == JOB_ADJ_ETD2RK && threadIdx.x == 0 && lb == 0) *P.dbeta += (P.h / P.beta) * dsum;
  }
};

// One block of the persistent kernel (block lb of a group of G working on
// instance P); c, R and S are the block's LDS.
template <int DIM>
__device__ __forceinline__ void krylov_body(const KrylovDev& P, int lb, int G, Ctl& c, double* R, double* S) {
  const unsigned long long t_start = wall_clock64();
  Engine<DIM> e{P, c, R, S, *P.g.n_active, 0, lb, G};
  if (threadIdx.x == 0) {
    for (int k = 0; k <= PMAX; ++k) {
      c.m_guess[k] = P.st->m_guess[k];
      c.tau_frac[k] = P.st->tau_frac[k];
    }
    c.st = Ctl::Stats{};
  }
  e.failed = false;
  e.iu = V_U;
  e.sp_stride = (size_t)(e.nact / (P.species > 1 ? P.species : 1)) * TILE_PTS;
  __syncthreads();
  e.run(t_start);
  __syncthreads();
  if (threadIdx.x == 0 && lb == 0) {
    for (int k = 0; k <= PMAX; ++k) {
      P.st->m_guess[k] = c.m_guess[k];
      P.st->tau_frac[k] = c.tau_frac[k];
    }
    const Ctl::Stats& s = c.st;
    P.st->substeps = s.substeps;
    P.st->rejected = s.rejected;
    P.st->matvecs = s.matvecs;
    P.st->m_last = s.m_last;
    P.st->expms = s.expms;
    P.st->calls += 1;
    P.st->err_est = s.err_est;
    P.st->t_done = s.t_done;
    P.st->alg_bytes_per_unknown = s.bpu;
    P.st->alg_bytes_total += s.bpu * (double)(*P.g.n_unknowns);
    P.st->ticks_total += (double)(wall_clock64() - t_start);
    P.st->ticks_sync += (double)s.tk_sync;
    P.st->ticks_expm += (double)s.tk_expm;
    P.st->ticks_pass += (double)s.tk_pass;
    P.st->ticks_pro += (double)s.tk_pro;
    P.st->ticks_gap += (double)s.tk_gap;
    P.st->syncs += s.n_sync;
    P.st->expm_calls += s.expms;
  }
}

// One instance over the whole (cooperatively launched) grid.
template <int DIM>
__global__ __launch_bounds__(KBLOCK) void krylov_kernel(KrylovDev P) {
  __shared__ Ctl c;
  // the two exponential buffers, contiguous: between exponentials the
  // LDS-staged Lanczos pass uses them as its tile buffers
  __shared__ double RS[2 * EXPM_NMAX * EXPM_NMAX];
  double* R = RS;
  double* S = RS + EXPM_NMAX * EXPM_NMAX;
  // parameters in LDS: the engine refers to them by reference, and a
  // reference to a kernel argument would force a private-memory copy
  __shared__ KrylovDev sP;
  if (threadIdx.x == 0) sP = P;
  __syncthreads();
  krylov_body<DIM>(sP, (int)blockIdx.x, (int)gridDim.x, c, R, S);
}

// A batch of instances: block b belongs to instance blk_inst[b], whose
// group is blocks Ps[i].g_first .. Ps[i].g_first + Ps[i].g_size - 1.  The
// launch is cooperative whenever a group has more than one block.
template <int DIM>
__global__ __launch_bounds__(KBLOCK) void krylov_group_kernel(const KrylovDev* __restrict__ Ps,
                                                              const int* __restrict__ blk_inst) {
  __shared__ Ctl c;
  // the two exponential buffers, contiguous: between exponentials the
  // LDS-staged Lanczos pass uses them as its tile buffers
  __shared__ double RS[2 * EXPM_NMAX * EXPM_NMAX];
  double* R = RS;
  double* S = RS + EXPM_NMAX * EXPM_NMAX;
  const KrylovDev& P = Ps[blk_inst[blockIdx.x]];
  krylov_body<DIM>(P, (int)blockIdx.x - P.g_first, P.g_size, c, R, S);
}

// Reset the synchronisation state before a persistent launch (a kernel, not
// a memset, so the sequence can sit inside a captured graph).
__global__ void sync_reset_kernel(BarrierDev* b, unsigned* flags, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) flags[i] = 0u;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    b->count = 0;
    b->gen = 0;
    b->abort = 0;
  }
}

// Same for every instance of a batch (block i resets instance i).
__global__ void sync_reset_group_kernel(const KrylovDev* __restrict__ Ps, int count) {
  if ((int)blockIdx.x >= count) return;
  const KrylovDev& P = Ps[blockIdx.x];
  for (int i = threadIdx.x; i < P.g_size; i += blockDim.x) P.flags[i] = 0u;
  if (threadIdx.x == 0) {
    P.bar->count = 0;
    P.bar->gen = 0;
    P.bar->abort = 0;
  }
}

int krylov_max_blocks_per_cu(int dim, int /*tmax*/) {
  int nb = 0;
  hipError_t e = (dim == 2)
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, krylov_kernel<2>, KBLOCK, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, krylov_kernel<3>, KBLOCK, 0);
  if (e != hipSuccess) return 0;
  int ng = 0;
  e = (dim == 2) ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&ng, krylov_group_kernel<2>, KBLOCK, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&ng, krylov_group_kernel<3>, KBLOCK, 0);
  if (e != hipSuccess) return 0;
  return ng < nb ? ng : nb;
}

size_t krylov_dyn_lds(int /*dim*/, int /*tmax*/) { return 0; }

// A batch (Ps, blk_inst: device arrays of `count` parameter sets and
// `blocks` instance indices).  `cooperative` when some group has more than
// one block: the runtime then guarantees co-residency of the whole grid.
hipError_t launch_krylov_group(int dim, const KrylovDev* Ps, int count, const int* blk_inst, int blocks,
                               bool cooperative, hipStream_t s) {
  hipLaunchKernelGGL(sync_reset_group_kernel, dim3(count), dim3(256), 0, s, Ps, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!cooperative) {
    if (dim == 2)
      hipLaunchKernelGGL(krylov_group_kernel<2>, dim3(blocks), dim3(KBLOCK), 0, s, Ps, blk_inst);
    else
      hipLaunchKernelGGL(krylov_group_kernel<3>, dim3(blocks), dim3(KBLOCK), 0, s, Ps, blk_inst);
    return hipGetLastError();
  }
  const KrylovDev* a0 = Ps;
  const int* a1 = blk_inst;
  void* args[] = {&a0, &a1};
  const void* fn = (dim == 2) ? (const void*)krylov_group_kernel<2> : (const void*)krylov_group_kernel<3>;
  return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(KBLOCK), args, 0, s);
}

// Reset the barrier, then the cooperative launch (co-residency of all blocks
// is what makes the grid barrier safe).
hipError_t launch_krylov(int dim, const KrylovDev& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL(sync_reset_kernel, dim3(1), dim3(256), 0, s, P.bar, P.flags, grid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  KrylovDev arg = P;
  arg.g_first = 0;
  arg.g_size = grid;
  void* args[] = {&arg};
  const void* fn = (dim == 2) ? (const void*)krylov_kernel<2> : (const void*)krylov_kernel<3>;
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(KBLOCK), args, 0, s);
}

}  // namespace KRYLOV_NS
}  // namespace etdfb
