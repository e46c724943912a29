// Level-set sweeps that move the free boundary (Section 4.3 of the paper,
// Algorithm Steps 1-2).  Box layout, one thread per node, 256-node tiles
// (one tile per block), Jacobi updates (every node from the previous
// iterate, so the result does not depend on scheduling), nearest-node values
// beyond the box edge.  Band and whole-box launches: see levelset.h.
//
// Readings of the paper's unspecified details (shared with the CPU oracle):
// * normals n = grad rho / max(|grad rho|, 1e-12), central differences;
// * quadratic normal extrapolation of u (Aslam): known set K0 =
//   computational points; u_n = n.grad u where the central stencil is in K0
//   (K1), u_nn = n.grad u_n where it is in K1 (K2); then ASLAM_ITERS Jacobi
//   sweeps v <- v - dtau (n.grad v - src), first-order upwind along n,
//   dtau = h/2, for u_nn (src 0), u_n (src u_nn), u (src u_n), unknown values
//   starting at 0;
// * Stefan speed V = mu |grad u_ext| (central) where |rho| < h, extended
//   along sign(rho) n by VEL_ITERS sweeps, dtau = h/2;
// * rho_t + V |grad rho| = 0 with the Godunov Hamiltonian for V >= 0,
//   HJ-WENO5 (eps 1e-6), TVD-RK3, max(1, ceil(max V dt / (h/2))) substeps;
// * reinitialisation rho_t + S(rho_0)(|grad rho| - 1) = 0,
//   S = rho_0 / sqrt(rho_0^2 + h^2), REINIT_ITERS RK3 steps of h/2;
// * finally u = u_ext on the computational points of the new rho, else 0.
#include <math.h>

#include "device_common.h"
#include "levelset.h"

namespace etdfb {

namespace {

constexpr double WENO_EPS = 1e-6;

// box arrays of LevelsetScratch::buf; the second field's extension arrays
// (LsInst::f) sit FOFF after the first's (F0..F3 for E0..E3)
enum { A_NX = 0, A_NY = 1, A_NZ = 2, A_E0 = 3, A_E1 = 4, A_E2 = 5, A_E3 = 6, A_V = 7,
       A_R0 = 8, A_R1 = 9, A_R2 = 10, A_S = 11, A_F0 = 12, A_F1 = 13, A_F2 = 14, A_F3 = 15, A_COUNT = 16 };
constexpr int FOFF = A_F0 - A_E0;

struct Where {
  const LsInst* I;
  int local;     // tile index within the instance's list
  int i, j, k;
  size_t id;
  bool in;       // node inside the box
};

// Block -> instance (largest i with off[i] <= blockIdx.x, off the launch
// row's offsets) -> tile (row LS_ROW_C + r / LS_ROW_V + r: the prefix of the
// sorted list SC / SV within radius r; LS_ROW_U: list U; LS_ROW_FULL: every
// tile) -> node.
template <int DIM>
__device__ __forceinline__ Where locate_at(const LsInst* __restrict__ insts, const int* __restrict__ off, int count,
                                          int row, int b) {
  const int* o = off + (size_t)row * (count + 1);
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (o[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  Where w;
  w.I = insts + lo;
  w.local = b - o[lo];
  const LsInst& I = *w.I;
  const size_t nt = (size_t)I.ntx * I.nty * I.ntz;
  const int lst = row == LS_ROW_U ? LS_U : (row >= LS_ROW_V ? LS_SV : LS_SC);
  const int t = (row == LS_ROW_FULL) ? w.local : I.band[(size_t)lst * nt + w.local];
  constexpr int X = TileShape<DIM>::X, Y = TileShape<DIM>::Y;
  const int tx = t % I.ntx, ty = (t / I.ntx) % I.nty, tz = t / (I.ntx * I.nty);
  const int l = threadIdx.x;
  w.i = tx * X + l % X;
  w.j = ty * Y + (l / X) % Y;
  w.k = tz * TileShape<DIM>::Z + l / (X * Y);
  w.in = w.i < I.nx && w.j < I.ny && w.k < I.nz;
  w.id = ((size_t)w.k * I.ny + w.j) * I.nx + w.i;
  return w;
}

// Instance of virtual block b of a launch row (largest i with off[i] <= b).
__device__ __forceinline__ const LsInst& inst_at(const LsInst* __restrict__ insts, const int* __restrict__ off,
                                                 int count, int row, int b) {
  const int* o = off + (size_t)row * (count + 1);
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (o[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return insts[lo];
}

// Virtual blocks of a launch row (the row's total, read on the device); a
// launch's blocks loop over them, so any grid serves any list size.
__device__ __forceinline__ int row_total(const int* __restrict__ off, int count, int row) {
  return off[(size_t)row * (count + 1) + count];
}
#define FOR_VBLOCKS(ROW) \
  for (int vb_ = (int)blockIdx.x, tot_ = row_total(off, count, (ROW)); vb_ < tot_; vb_ += (int)gridDim.x)

__device__ __forceinline__ gptr<double> arr(const LsInst& I, int a) { return glb(I.buf) + (size_t)a * I.nodes; }

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// index of the node shifted by s along axis d, clamped to the box
__device__ __forceinline__ size_t shifted(const LsInst& I, const Where& w, int d, int s) {
  int i = w.i, j = w.j, k = w.k;
  if (d == 0) i = clampi(i + s, I.nx);
  else if (d == 1) j = clampi(j + s, I.ny);
  else k = clampi(k + s, I.nz);
  return ((size_t)k * I.ny + j) * I.nx + i;
}

// computational point of rho (inside, not on the box edge, 2d neighbours inside)
template <int DIM>
__device__ __forceinline__ bool comp_point(const LsInst& I, const Where& w, gptr<const double> rho) {
  bool c = rho[w.id] < 0.0;
  if (c) {
    if (w.i == 0 || w.i == I.nx - 1 || w.j == 0 || w.j == I.ny - 1) c = false;
    if (DIM == 3 && (w.k == 0 || w.k == I.nz - 1)) c = false;
  }
  for (int d = 0; d < DIM && c; ++d) c = rho[shifted(I, w, d, -1)] < 0.0 && rho[shifted(I, w, d, 1)] < 0.0;
  return c;
}

// ------------------------------------------------------------ Step 1: u_ext

// whole box of the instances with a dirty scratch: the extrapolation arrays,
// the speed and its ping-pong partner to 0, the distance to 255, and the
// instance's maximum speed to 0
template <int DIM>
__global__ __launch_bounds__(256) void zero_kernel(const LsInst* __restrict__ insts, const int* __restrict__ off,
                                                   int count) {
  FOR_VBLOCKS(LS_ROW_FULL) {
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_FULL, vb_);
    const LsInst& I = *w.I;
    if (!I.dirty) continue;
    if (w.local == 0 && threadIdx.x == 0) *glb(I.vmax) = 0.0;
    if (w.local == 0 && threadIdx.x < LS_VMAX_SLOTS) glb(I.vslot)[threadIdx.x] = 0.0;
    if (!w.in) continue;
    for (int a = A_E0; a <= A_V; ++a) arr(I, a)[w.id] = 0.0;
    arr(I, A_S)[w.id] = 0.0;
    for (int a = A_F0; a <= A_F3; ++a) arr(I, a)[w.id] = 0.0;
    glb(I.dist)[w.id] = 255;
  }
}

// list U: normals, K0 (bit 0, other bits cleared), E0 = K0 ? u : 0 (and
// F0 = K0 ? f : 0)
template <int DIM>
__global__ __launch_bounds__(256) void init_kernel(const LsInst* __restrict__ insts, const int* __restrict__ off,
                                                   int count) {
  FOR_VBLOCKS(LS_ROW_U) {
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_U, vb_);
    if (!w.in) continue;
    const LsInst& I = *w.I;
    gptr<const double> rho = glb((const double*)I.rho);
    double g[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < DIM; ++d) g[d] = (rho[shifted(I, w, d, 1)] - rho[shifted(I, w, d, -1)]) / (2.0 * I.h);
    double mag = 0.0;
    for (int d = 0; d < DIM; ++d) mag += g[d] * g[d];
    mag = fmax(sqrt(mag), 1e-12);
    for (int d = 0; d < DIM; ++d) arr(I, A_NX + d)[w.id] = g[d] / mag;
    const bool c = comp_point<DIM>(I, w, rho);
    glb(I.known)[w.id] = c ? 1 : 0;
    glb(I.dist)[w.id] = c ? 0 : 255;
    arr(I, A_E0)[w.id] = c ? glb((const double*)I.u)[w.id] : 0.0;
    if (I.f) arr(I, A_F0)[w.id] = c ? glb((const double*)I.f)[w.id] : 0.0;
  }
}

// every read of the extended u (velocity, restriction) must fall within
// LS_READ_REACH of the computational points, where it equals the whole-box
// extension (see levelset.h)
__device__ __forceinline__ bool in_reach(const LsInst& I, size_t id) {
  return glb((const uint8_t*)I.dist)[id] <= LS_READ_REACH;
}

// bit `src` at the node and its 2d (clamped) neighbours
template <int DIM>
__device__ __forceinline__ bool known_all(const LsInst& I, const Where& w, int src) {
  gptr<const uint8_t> kn = glb((const uint8_t*)I.known);
  bool c = (kn[w.id] >> src) & 1;
  for (int d = 0; d < DIM && c; ++d)
    c = ((kn[shifted(I, w, d, -1)] >> src) & 1) && ((kn[shifted(I, w, d, 1)] >> src) & 1);
  return c;
}

// n . (central gradient of a) at the node
template <int DIM>
__device__ __forceinline__ double dir_deriv(const LsInst& I, const Where& w, gptr<const double> a) {
  double v = 0.0;
  for (int d = 0; d < DIM; ++d)
    v += arr(I, A_NX + d)[w.id] * ((a[shifted(I, w, d, 1)] - a[shifted(I, w, d, -1)]) / (2.0 * I.h));
  return v;
}

// list A1: K1 (bit 1)
template <int DIM>
__global__ __launch_bounds__(256) void known1_kernel(const LsInst* __restrict__ insts, const int* __restrict__ off,
                                                     int count) {
  FOR_VBLOCKS(LS_ROW_C + ASLAM_ITERS + 1) {
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_C + ASLAM_ITERS + 1, vb_);
    if (!w.in) continue;
    const LsInst& I = *w.I;
    if (known_all<DIM>(I, w, 0)) glb(I.known)[w.id] |= (uint8_t)2;
  }
}

// list A1: K2 (bit 2) and E1 = K1 ? n . grad E0 : 0 (F1 likewise)
template <int DIM>
__global__ __launch_bounds__(256) void known2_un_kernel(const LsInst* __restrict__ insts,
                                                        const int* __restrict__ off, int count) {
  FOR_VBLOCKS(LS_ROW_C + ASLAM_ITERS + 1) {
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_C + ASLAM_ITERS + 1, vb_);
    if (!w.in) continue;
    const LsInst& I = *w.I;
    const bool k1 = (glb((const uint8_t*)I.known)[w.id] >> 1) & 1;
    if (known_all<DIM>(I, w, 1)) glb(I.known)[w.id] |= (uint8_t)4;
    arr(I, A_E1)[w.id] = k1 ? dir_deriv<DIM>(I, w, arr(I, A_E0)) : 0.0;
    if (I.f) arr(I, A_F1)[w.id] = k1 ? dir_deriv<DIM>(I, w, arr(I, A_F0)) : 0.0;
  }
}

// list A1: E2 = K2 ? n . grad E1 : 0 (F2 likewise)
template <int DIM>
__global__ __launch_bounds__(256) void unn_kernel(const LsInst* __restrict__ insts, const int* __restrict__ off,
                                                  int count) {
  FOR_VBLOCKS(LS_ROW_C + ASLAM_ITERS + 1) {
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_C + ASLAM_ITERS + 1, vb_);
    if (!w.in) continue;
    const LsInst& I = *w.I;
    const bool k2 = (glb((const uint8_t*)I.known)[w.id] >> 2) & 1;
    arr(I, A_E2)[w.id] = k2 ? dir_deriv<DIM>(I, w, arr(I, A_E1)) : 0.0;
    if (I.f) arr(I, A_F2)[w.id] = k2 ? dir_deriv<DIM>(I, w, arr(I, A_F1)) : 0.0;
  }
}

// Launch shape of the 3D sweeps: tiles per block, XCD-contiguous ranges.
#ifndef EXT_NPT
#define EXT_NPT 1
#endif
#ifndef EXT_XCD
#define EXT_XCD 1
#endif
// grid of an extend_kernel launch over `total` tiles
inline int ext_grid(int total) {
  const int nvb = (total + EXT_NPT - 1) / EXT_NPT;
  return EXT_XCD ? 8 * ((nvb + 7) / 8) : nvb;
}

// one Jacobi sweep on `list`: out = v - dtau (a.grad v - src) off the known set
// (bit), a = sgn * n, sgn = 1 or sign(rho) (speed extension); with
// do_max, also the maximum of out (non-negative values) into the instance's
// slots (vmax_fold_kernel takes their maximum).  With
// dil, the sweep also dilates the L1 distance to the computational points
// by one node, in place (a value only decreases, never below the true
// distance; after k such sweeps every node within k holds its exact
// distance).  With cone >= 0, only nodes within L1 distance cone of the
// computational points are swept (the others are neither read nor
// written): after the sweep's own dilation, or from the distance when it
// is already exact that far.  A block serves NPT consecutive tiles of the
// launch row (one node of each per thread); the loads of all of them are
// issued before the arithmetic (the update is computed everywhere and
// selected off the known set).  With NF == 2 the instances with a second
// field (LsInst::f) sweep it in the same launch, on the arrays FOFF after
// v, out and src, with the same normals, known set and cone.
template <int DIM, int NPT, int NF>
__global__ __launch_bounds__(256) void extend_kernel(const LsInst* __restrict__ insts, const int* __restrict__ off,
                                                     int count, int row, int v_arr, int out_arr, int src_arr,
                                                     int bit, int sign_rho, int do_max, int dil, int cone,
                                                     int nslot) {
  const int total = row_total(off, count, row);
  // XCD-contiguous ranges: workgroups go to the 8 XCDs in turn, so virtual
  // block v takes entry (v % 8) * chunk + v / 8 of the row (8 * chunk
  // virtual blocks; grids are multiples of 8, so v % 8 is the XCD of the
  // block that runs it) and each XCD walks a contiguous range of the list,
  // whose neighbouring tiles share halo lines in that XCD's L2.
  const int nvb = (total + NPT - 1) / NPT;
  const int chunk = EXT_XCD ? (nvb + 7) / 8 : 0;
  const int span = EXT_XCD ? 8 * chunk : nvb;
  for (int vx = (int)blockIdx.x; vx < span; vx += (int)gridDim.x) {
    const int bx = EXT_XCD ? (vx % 8) * chunk + vx / 8 : vx;
    Where w[NPT];
  #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int vb = bx * NPT + q;
      if (vb < total) {
        w[q] = locate_at<DIM>(insts, off, count, row, vb);
      } else {
        w[q].I = insts;
        w[q].in = false;
        w[q].id = 0;
        w[q].i = w[q].j = w[q].k = 0;
      }
    }
    size_t im[NPT][DIM], ip[NPT][DIM];
    int m[NPT];
    bool act[NPT];
  #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      act[q] = false;
      m[q] = 0;
      if (!w[q].in) continue;
      const LsInst& I = *w[q].I;
      for (int d = 0; d < DIM; ++d) {
        im[q][d] = shifted(I, w[q], d, -1);
        ip[q][d] = shifted(I, w[q], d, 1);
      }
      if (dil || cone >= 0) {
        gptr<const uint8_t> ds = glb((const uint8_t*)I.dist);
        m[q] = ds[w[q].id];
        if (dil) {
          int dn = 255;
          for (int d = 0; d < DIM; ++d) dn = min(dn, min((int)ds[im[q][d]], (int)ds[ip[q][d]]));
          m[q] = min(m[q], dn + 1);
        }
      }
      act[q] = cone < 0 || m[q] <= cone;
    }
    uint8_t kb[NPT];
    double vc[NF][NPT], vm[NF][NPT][DIM], vp[NF][NPT][DIM], nd[NPT][DIM], sr[NF][NPT], rr[NPT];
    bool two[NPT];
  #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      two[q] = false;
      if (!act[q]) continue;
      const LsInst& I = *w[q].I;
      two[q] = NF == 2 && I.f != nullptr;
      kb[q] = glb((const uint8_t*)I.known)[w[q].id];
      for (int d = 0; d < DIM; ++d) nd[q][d] = arr(I, A_NX + d)[w[q].id];
      rr[q] = sign_rho ? glb((const double*)I.rho)[w[q].id] : 1.0;
  #pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        if (fi == 1 && !two[q]) break;
        gptr<const double> v = arr(I, v_arr + fi * FOFF);
        vc[fi][q] = v[w[q].id];
        for (int d = 0; d < DIM; ++d) {
          vm[fi][q][d] = v[im[q][d]];
          vp[fi][q][d] = v[ip[q][d]];
        }
        sr[fi][q] = (src_arr >= 0) ? arr(I, src_arr + fi * FOFF)[w[q].id] : 0.0;
      }
    }
    double res[NF][NPT];
  #pragma unroll
    for (int q = 0; q < NPT; ++q) {
  #pragma unroll
      for (int fi = 0; fi < NF; ++fi) res[fi][q] = 0.0;
      if (!act[q]) continue;
      const LsInst& I = *w[q].I;
      const double sg = (rr[q] > 0.0) ? 1.0 : ((rr[q] < 0.0) ? -1.0 : 0.0);
  #pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        if (fi == 1 && !two[q]) break;
        double up = 0.0;
        for (int d = 0; d < DIM; ++d) {
          const double a = sg * nd[q][d];
          up += fmax(a, 0.0) * (vc[fi][q] - vm[fi][q][d]) + fmin(a, 0.0) * (vp[fi][q][d] - vc[fi][q]);
        }
        up = up / I.h;
        const double upd = vc[fi][q] - (0.5 * I.h) * (up - sr[fi][q]);
        res[fi][q] = ((kb[q] >> bit) & 1) ? vc[fi][q] : upd;
      }
    }
  #pragma unroll
    for (int q = 0; q < NPT; ++q) {
      if (!w[q].in) continue;
      const LsInst& I = *w[q].I;
      if (act[q]) {
        arr(I, out_arr)[w[q].id] = res[0][q];
        if (two[q]) arr(I, out_arr + FOFF)[w[q].id] = res[NF - 1][q];
      }
      if (dil) glb(I.dist)[w[q].id] = (uint8_t)min(m[q], 255);
    }
    if (do_max) {
      // per tile (each tile belongs to one instance)
      __shared__ double sm[256];
      for (int q = 0; q < NPT; ++q) {
        if (bx * NPT + q >= total) break;   // uniform over the block
        sm[threadIdx.x] = act[q] ? res[0][q] : 0.0;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
          if ((int)threadIdx.x < st) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + st]);
          __syncthreads();
        }
        // max of non-negative doubles: integer order equals value order
        if (threadIdx.x == 0)
          atomicMax((unsigned long long*)(nslot > 1 ? w[q].I->vslot + (vx & (nslot - 1)) : w[q].I->vmax),
                    (unsigned long long)__double_as_longlong(sm[0]));
        __syncthreads();
      }
    }
  }
}

// 2D only: SWEEP_GROUP Jacobi sweeps of extend_kernel in one launch.  The
// block stages its tile plus a halo of SWEEP_GROUP nodes in LDS (values,
// normals, source, known bit, sign of rho), sweeps there (the valid region
// shrinks by one node per sweep) and writes the tile.  Halo nodes outside the
// stage's list hold their whole-box values (0, see levelset.h), so the tile
// gets exactly the values of `nsweep` single sweeps.  With NF == 2 the
// instances with a second field sweep it alongside (arrays FOFF after v,
// out and src; the same normals, known set and signs).
constexpr int SWEEP_GROUP = 5;

template <int NF>
__global__ __launch_bounds__(256) void extend_group_kernel(const LsInst* __restrict__ insts,
                                                           const int* __restrict__ off, int count, int row,
                                                           int v_arr, int out_arr, int src_arr, int bit,
                                                           int sign_rho, int do_max, int nsweep, int dil,
                                                           int nslot) {
  constexpr int X = TileShape<2>::X, Y = TileShape<2>::Y, K = SWEEP_GROUP;
  constexpr int RW = X + 2 * K, RH = Y + 2 * K, RN = RW * RH;
  __shared__ double va[NF][RN], vb[NF][RN], ssrc[NF][RN], snx[RN], sny[RN];
  __shared__ uint8_t sfl[RN];   // bit 0: in the box, bit 1: known, bits 2-3: sign(rho) + 1
  __shared__ uint8_t sd[2][RN]; // dil: the distance to the computational points (dilated with the sweeps)
  __shared__ double sm[256];
  FOR_VBLOCKS(row) {
    const Where w = locate_at<2>(insts, off, count, row, vb_);
    const LsInst& I = *w.I;
    const int nf = (NF == 2 && I.f != nullptr) ? 2 : 1;   // uniform over the block
    const int ox = w.i - (int)(threadIdx.x % X), oy = w.j - (int)(threadIdx.x / X);   // tile origin
    gptr<const double> nxg = arr(I, A_NX);
    gptr<const double> nyg = arr(I, A_NY);
    gptr<const uint8_t> kn = glb((const uint8_t*)I.known);
    gptr<const double> rho = glb((const double*)I.rho);
    gptr<const double> vg[NF], sg_[NF];
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      vg[fi] = arr(I, v_arr + fi * FOFF);
      sg_[fi] = arr(I, (src_arr >= 0 ? src_arr : v_arr) + fi * FOFF);
    }
    for (int r = threadIdx.x; r < RN; r += blockDim.x) {
      const int gi = ox - K + r % RW, gj = oy - K + r / RW;
      uint8_t f = 0;
      double x[NF], sc[NF], a = 0.0, b = 0.0;
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) { x[fi] = 0.0; sc[fi] = 0.0; }
      if (gi >= 0 && gi < I.nx && gj >= 0 && gj < I.ny) {
        const size_t id = (size_t)gj * I.nx + gi;
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) {
          if (fi >= nf) break;
          x[fi] = vg[fi][id];
          sc[fi] = (src_arr >= 0) ? sg_[fi][id] : 0.0;
        }
        a = nxg[id];
        b = nyg[id];
        f = 1 | ((((kn[id] >> bit) & 1) != 0) ? 2 : 0);
        if (sign_rho) {
          const double rr = rho[id];
          f |= (uint8_t)(((rr > 0.0) ? 2 : ((rr < 0.0) ? 0 : 1)) << 2);
        } else {
          f |= (uint8_t)(2 << 2);
        }
      }
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        va[fi][r] = x[fi];
        ssrc[fi][r] = sc[fi];
      }
      snx[r] = a;
      sny[r] = b;
      sfl[r] = f;
      if (dil) sd[0][r] = (f & 1) ? glb((const uint8_t*)I.dist)[(size_t)gj * I.nx + gi] : (uint8_t)255;
    }
    __syncthreads();
    const double dt = 0.5 * I.h;
    double (*cur)[RN] = va;
    double (*nxt)[RN] = vb;
    for (int s = 0; s < nsweep; ++s) {
      for (int r = threadIdx.x; r < RN; r += blockDim.x) {
        const uint8_t f = sfl[r];
        const int x = r % RW, y = r / RW;
        const int gi = ox - K + x, gj = oy - K + y;
        // neighbours, clamped at the box edge; outside the region: the node itself
        // (such nodes are beyond the valid region of this sweep)
        const int rxm = (gi == 0 || x == 0) ? r : r - 1;
        const int rxp = (gi == I.nx - 1 || x == RW - 1) ? r : r + 1;
        const int rym = (gj == 0 || y == 0) ? r : r - RW;
        const int ryp = (gj == I.ny - 1 || y == RH - 1) ? r : r + RW;
        if (dil) {
          const uint8_t* dc = sd[s & 1];
          int m = dc[r];
          m = min(m, min(min((int)dc[rxm], (int)dc[rxp]), min((int)dc[rym], (int)dc[ryp])) + 1);
          sd[(s + 1) & 1][r] = (uint8_t)min(m, 255);
        }
#pragma unroll
        for (int fi = 0; fi < NF; ++fi) {
          if (fi >= nf) break;
          const double vc = cur[fi][r];
          double res = vc;
          if ((f & 1) && !(f & 2)) {
            const double sg = (double)((f >> 2) & 3) - 1.0;
            const double ax = sg * snx[r], ay = sg * sny[r];
            double up = fmax(ax, 0.0) * (vc - cur[fi][rxm]) + fmin(ax, 0.0) * (cur[fi][rxp] - vc);
            up += fmax(ay, 0.0) * (vc - cur[fi][rym]) + fmin(ay, 0.0) * (cur[fi][ryp] - vc);
            up = up / I.h;
            res = vc - dt * (up - ssrc[fi][r]);
          }
          nxt[fi][r] = res;
        }
      }
      __syncthreads();
      double (*t)[RN] = cur; cur = nxt; nxt = t;
    }
    const int l = threadIdx.x;
    const int rl = (l / X + K) * RW + (l % X + K);
    const double res = cur[0][rl];
    if (w.in) arr(I, out_arr)[w.id] = res;
    if (w.in && nf == 2) arr(I, out_arr + FOFF)[w.id] = cur[NF - 1][rl];
    if (w.in && dil) glb(I.dist)[w.id] = sd[nsweep & 1][rl];
    if (do_max) {
      sm[threadIdx.x] = w.in ? res : 0.0;
      __syncthreads();
      for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + st]);
        __syncthreads();
      }
      if (threadIdx.x == 0)
        atomicMax((unsigned long long*)(nslot > 1 ? I.vslot + (vb_ & (nslot - 1)) : I.vmax),
                  (unsigned long long)__double_as_longlong(sm[0]));
    }
    __syncthreads();   // LDS is restaged by the next virtual block
  }
}

// Whole box, before a reinitialisation: every node of the narrow band
// (|rho_0| < REINIT_BAND h) and its 3-node WENO reach along each axis must lie
// in tiles of list R (Dv <= rr), where the RK stages run; else ST_FRONT.
template <int DIM>
__global__ __launch_bounds__(256) void reinit_check_kernel(const LsInst* __restrict__ insts,
                                                           const int* __restrict__ off, int count) {
  FOR_VBLOCKS(LS_ROW_FULL) {
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_FULL, vb_);
    if (!w.in) continue;
    const LsInst& I = *w.I;
    if (!(fabs(glb((const double*)I.rho)[w.id]) < REINIT_BAND * I.h)) continue;
    constexpr int X = TileShape<DIM>::X, Y = TileShape<DIM>::Y, Z = TileShape<DIM>::Z;
    const int ext[3] = {X, Y, Z};
    const int n[3] = {I.nx, I.ny, I.nz};
    bool ok = true;
    for (int d = 0; d < DIM; ++d)
      for (int s = -3; s <= 3; s += 6) {
        int c[3] = {w.i, w.j, w.k};
        c[d] = clampi(c[d] + s, n[d]);
        const int t = ((c[2] / Z) * I.nty + c[1] / Y) * I.ntx + c[0] / X;
        ok = ok && (I.tdist[t] >> 16) <= I.rr;
        (void)ext;
      }
    if (!ok) atomicCAS(I.status, 0, ST_FRONT);
  }
}

// list V: V = (|rho| < h) ? mu |central grad u_ext| : 0; speed band into bit 3
template <int DIM>
__global__ __launch_bounds__(256) void velocity_kernel(const LsInst* __restrict__ insts,
                                                       const int* __restrict__ off, int count, int uext_arr) {
  FOR_VBLOCKS(LS_ROW_V + VEL_ITERS + 1) {
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_V + VEL_ITERS + 1, vb_);
    if (!w.in) continue;
    const LsInst& I = *w.I;
    gptr<const double> ue = arr(I, uext_arr);
    gptr<uint8_t> kn = glb(I.known);
    const bool band = fabs(glb((const double*)I.rho)[w.id]) < I.h;
    double v = 0.0;
    if (band) {
      double s = 0.0;
      bool reach = true;
      for (int d = 0; d < DIM; ++d) {
        const size_t ip = shifted(I, w, d, 1), im = shifted(I, w, d, -1);
        reach = reach && in_reach(I, ip) && in_reach(I, im);
        const double g = (ue[ip] - ue[im]) / (2.0 * I.h);
        s += g * g;
      }
      if (!reach) atomicCAS(I.status, 0, ST_FRONT);
      v = I.mu * sqrt(s);
      kn[w.id] |= (uint8_t)8;
    } else {
      kn[w.id] &= (uint8_t)~8u;
    }
    arr(I, A_V)[w.id] = v;
  }
}


// ------------------------------------------------------------ Step 2: WENO

// Fifth-order WENO derivative from the five differences v1..v5 (Jiang-Peng
// weights, eps 1e-6).  The nonlinear weights d_k / (eps + beta_k)^2 are
// normalised through their common denominator, so one division remains.
__device__ __forceinline__ double weno5(double v1, double v2, double v3, double v4, double v5) {
  constexpr double SIXTH = 1.0 / 6.0;
  const double p1 = (2.0 * v1 - 7.0 * v2 + 11.0 * v3) * SIXTH;
  const double p2 = (-v2 + 5.0 * v3 + 2.0 * v4) * SIXTH;
  const double p3 = (2.0 * v3 + 5.0 * v4 - v5) * SIXTH;
  const double t1 = v1 - 2.0 * v2 + v3, t1b = v1 - 4.0 * v2 + 3.0 * v3;
  const double t2 = v2 - 2.0 * v3 + v4, t2b = v2 - v4;
  const double t3 = v3 - 2.0 * v4 + v5, t3b = 3.0 * v3 - 4.0 * v4 + v5;
  const double s1 = 13.0 / 12.0 * (t1 * t1) + 0.25 * (t1b * t1b);
  const double s2 = 13.0 / 12.0 * (t2 * t2) + 0.25 * (t2b * t2b);
  const double s3 = 13.0 / 12.0 * (t3 * t3) + 0.25 * (t3b * t3b);
  const double e1 = s1 + WENO_EPS, e2 = s2 + WENO_EPS, e3 = s3 + WENO_EPS;
  const double q1 = e1 * e1, q2 = e2 * e2, q3 = e3 * e3;
  const double b1 = 0.1 * (q2 * q3), b2 = 0.6 * (q1 * q3), b3 = 0.3 * (q1 * q2);
  return (b1 * p1 + b2 * p2 + b3 * p3) / (b1 + b2 + b3);
}

// Godunov |grad phi| for speed sign sg (+1 / -1 / 0), HJ-WENO5 derivatives
template <int DIM>
__device__ double godunov(const LsInst& I, const Where& w, gptr<const double> phi, double sg) {
  double accp = 0.0, accn = 0.0;
  const double inv_h = 1.0 / I.h;
  for (int d = 0; d < DIM; ++d) {
    double f[7];
    for (int s = -3; s <= 3; ++s) f[s + 3] = phi[shifted(I, w, d, s)];
    double dd[6];
    for (int q = 0; q < 6; ++q) dd[q] = (f[q + 1] - f[q]) * inv_h;
    const double dm = weno5(dd[0], dd[1], dd[2], dd[3], dd[4]);
    const double dp = weno5(dd[5], dd[4], dd[3], dd[2], dd[1]);
    const double a = fmax(dm, 0.0), bb = fmin(dp, 0.0);
    accp += fmax(a * a, bb * bb);
    const double c = fmin(dm, 0.0), e = fmax(dp, 0.0);
    accn += fmax(c * c, e * e);
  }
  if (sg > 0.0) return sqrt(accp);
  if (sg < 0.0) return sqrt(accn);
  return 0.0;
}

// Substeps of the advection of an instance (the host takes the same
// formula on the same maximum speed).
__device__ __forceinline__ int substeps(const LsInst& I, double dt) {
  int n = (int)ceil(*glb((const double*)I.vmax) * dt / (0.5 * I.h));
  return n < 1 ? 1 : n;
}

// One TVD-RK3 stage (1, 2, 3): out = c0 * R0 + c1 * (in - dt * L(in)) with
// stage 1: in = rho, out = R1 (and R0 = rho); stage 2: in = R1, out = R2;
// stage 3: in = R2, out = rho; L = V G(in) (advection, list R, speed 0
// gives L = 0) or S (G_sign(S)(in) - 1) (reinitialisation, list R, only at
// nodes of the narrow band |rho_0| < REINIT_BAND h, the others keep rho_0 in
// every stage; first != 0 computes S and the band bit (known bit 4) from
// rho).  Advection substep q runs only for instances with more than q
// substeps.
template <int DIM>
__global__ __launch_bounds__(256) void rk_kernel(const LsInst* __restrict__ insts, const int* __restrict__ off,
                                                 int count, int reinit, int stage, int q, double dt, int first) {
  FOR_VBLOCKS(LS_ROW_V + LS_V_MAX) {
    double step;
    if (reinit) {
      step = 0.5 * inst_at(insts, off, count, LS_ROW_V + LS_V_MAX, vb_).h;
    } else {
      // substeps beyond the instance's count: nothing to do (checked before
      // the tile lookup)
      const LsInst& J = inst_at(insts, off, count, LS_ROW_V + LS_V_MAX, vb_);
      const int ns = substeps(J, dt);
      if (q >= ns) continue;
      step = dt / ns;
    }
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_V + LS_V_MAX, vb_);
    if (!w.in) continue;
    const LsInst& I = *w.I;
    gptr<double> rho = glb(I.rho);
    gptr<const double> in = (stage == 1) ? (gptr<const double>)rho : arr(I, stage == 2 ? A_R1 : A_R2);
    double L = 0.0;
    bool upd = true;
    if (reinit) {
      gptr<uint8_t> kn = glb(I.known);
      if (first) {
        const double r = rho[w.id];
        arr(I, A_S)[w.id] = r / sqrt(r * r + I.h * I.h);
        const bool inb = fabs(r) < REINIT_BAND * I.h;
        kn[w.id] = inb ? (uint8_t)(kn[w.id] | 16) : (uint8_t)(kn[w.id] & ~16u);
        upd = inb;
      } else {
        upd = (kn[w.id] >> 4) & 1;
      }
      if (upd) {
        const double s = arr(I, A_S)[w.id];
        const double sg = (s > 0.0) ? 1.0 : ((s < 0.0) ? -1.0 : 0.0);
        L = s * (godunov<DIM>(I, w, in, sg) - 1.0);
      }
    } else {
      const double V = arr(I, A_V)[w.id];
      L = (V != 0.0) ? V * godunov<DIM>(I, w, in, 1.0) : 0.0;
    }
    const double cur = in[w.id];
    const double st = cur - step * L;
    if (stage == 1) {
      arr(I, A_R0)[w.id] = cur;
      arr(I, A_R1)[w.id] = upd ? st : cur;
    } else if (stage == 2) {
      arr(I, A_R2)[w.id] = upd ? 0.75 * arr(I, A_R0)[w.id] + 0.25 * st : cur;
    } else if (upd) {
      rho[w.id] = (1.0 / 3.0) * arr(I, A_R0)[w.id] + (2.0 / 3.0) * st;
    }
  }
}

// whole box: u = comp(rho_new) ? u_ext : 0 (a computational point beyond
// the reach of the extension: ST_FRONT), and a second field f = f_ext
// within the reach of the extension and 0 beyond (what the step reads of
// it).  Outside list U (Dc > LS_C_MAX and Dv > LS_V_MAX) both are 0
// without a read: rho changes only on list R, inside U, so a tile outside U
// holds no computational point of the new rho, and no node within the
// reach.  Then the pass's own writes are cleared: on the tiles of U the
// extension arrays, the speed and its partner go to 0 and the distance to
// 255 (each thread reads and clears its own node only), and the maximum
// speed to 0.
template <int DIM>
__global__ __launch_bounds__(256) void restrict_kernel(const LsInst* __restrict__ insts,
                                                       const int* __restrict__ off, int count, int uext_arr) {
  FOR_VBLOCKS(LS_ROW_FULL) {
    const Where w = locate_at<DIM>(insts, off, count, LS_ROW_FULL, vb_);
    const LsInst& I = *w.I;
    if (w.local == 0 && threadIdx.x == 0) *glb(I.vmax) = 0.0;
    if (!w.in) continue;
    const int td = I.tdist[w.local];
    if ((td & 0xFFFF) > LS_C_MAX && (td >> 16) > LS_V_MAX) {
      glb(I.u)[w.id] = 0.0;
      if (I.f) glb(I.f)[w.id] = 0.0;
      continue;
    }
    const bool reach = in_reach(I, w.id);
    const bool c = comp_point<DIM>(I, w, glb((const double*)I.rho));
    if (c && !reach) atomicCAS(I.status, 0, ST_FRONT);
    glb(I.u)[w.id] = c ? arr(I, uext_arr)[w.id] : 0.0;
    for (int a = A_E0; a <= A_V; ++a) arr(I, a)[w.id] = 0.0;
    arr(I, A_S)[w.id] = 0.0;
    if (I.f) {
      glb(I.f)[w.id] = reach ? arr(I, uext_arr + FOFF)[w.id] : 0.0;
      for (int a = A_F0; a <= A_F3; ++a) arr(I, a)[w.id] = 0.0;
    }
    glb(I.dist)[w.id] = 255;
  }
}

// Device-sized mode: the launch rows' offsets from the geometry counters of
// every instance (thread q: row q).
__global__ void ls_rows_kernel(const LsInst* __restrict__ insts, int* __restrict__ off, int count) {
  const int q = (int)threadIdx.x;
  if (q >= LS_NROWS) return;
  int acc = 0;
  for (int i = 0; i < count; ++i) {
    const LsInst& I = insts[i];
    off[(size_t)q * (count + 1) + i] = acc;
    if (q == LS_ROW_FULL) acc += I.ntx * I.nty * I.ntz;
    else if (q == LS_ROW_U) acc += I.cnt[LS_CNT_U];
    else if (q >= LS_ROW_V) acc += I.cnt[LS_CNT_V + q - LS_ROW_V];
    else acc += I.cnt[LS_CNT_C + q - LS_ROW_C];
  }
  off[(size_t)q * (count + 1) + count] = acc;
}

// Device-sized mode: the front guard (max V dt <= LS_MAX_FRONT_NODES h, the
// host's test) per instance; a violation latches ST_FRONT.
__global__ void front_check_kernel(const LsInst* __restrict__ insts, int count, double dt) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= count) return;
  const LsInst& I = insts[i];
  if (!(*glb((const double*)I.vmax) * dt <= LS_MAX_FRONT_NODES * I.h)) atomicCAS(I.status, 0, ST_FRONT);
}

// The instance's maximum speed from its slots, which go back to 0 (block i:
// instance i; lane l: slot l).
__global__ __launch_bounds__(LS_VMAX_SLOTS) void vmax_fold_kernel(const LsInst* __restrict__ insts) {
  static_assert(LS_VMAX_SLOTS == 64, "one slot per lane of a wave");
  const LsInst& I = insts[blockIdx.x];
  const int l = (int)threadIdx.x;
  gptr<double> sl = glb(I.vslot);
  double m = sl[l];
  for (int o = LS_VMAX_SLOTS / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  sl[l] = 0.0;
  if (l == 0) *glb(I.vmax) = m;
}

// Fixed grid of a device-sized launch on `row` (a multiple of 8, see
// extend_kernel): the row's size when recorded (b.total, from the host
// counts of levelset_upload) with half again as headroom for a growing
// domain, at most LS_DEVICE_GRID (the blocks loop over any larger list).
constexpr int LS_DEVICE_GRID = 2048;
int device_grid(const LevelsetBatch& b, int row) {
  const int want = b.total[row] + b.total[row] / 2 + 8;
  const int g = 8 * ((want + 7) / 8);
  return g < LS_DEVICE_GRID ? g : LS_DEVICE_GRID;
}

// The restriction that clears every instance's list U is enqueued.
void mark_clean(LevelsetBatch& b) {
  for (int i = 0; i < b.count; ++i)
    if (b.h_inst[i].host_dirty) *b.h_inst[i].host_dirty = false;
}

template <int DIM>
hipError_t begin_dim(LevelsetBatch& b, hipStream_t st) {
  const int n = b.count;
  const LsInst* I = b.d_inst;
  const int* off = b.d_off;
  const dim3 B(256);
  // grid of a launch on `row`: its size (host counts), or the fixed grid
  const bool dev = b.device_sized;
  auto grid = [&](int row) { return dev ? device_grid(b, row) : b.total[row]; };
#define LL(row, kernel, ...)                                                                 \
  do {                                                                                       \
    if (grid(row) > 0) {                                                                     \
      hipLaunchKernelGGL(kernel<DIM>, dim3(grid(row)), B, 0, st, I, off, n, ##__VA_ARGS__);  \
      hipError_t _e = hipGetLastError();                                                     \
      if (_e != hipSuccess) return _e;                                                       \
    }                                                                                        \
  } while (0)
  if (b.any_dirty) LL(LS_ROW_FULL, zero_kernel);
  LL(LS_ROW_U, init_kernel);
  LL(LS_ROW_C + ASLAM_ITERS + 1, known1_kernel);
  LL(LS_ROW_C + ASLAM_ITERS + 1, known2_un_kernel);
  LL(LS_ROW_C + ASLAM_ITERS + 1, unn_kernel);
  // Aslam: u_nn (E2 <-> E3, result E3), u_n (E1 <-> E2, src u_nn, result E2),
  // u (E0 <-> E1, src u_n, result E1); each stage's array alternates once
  // per launch (2D: SWEEP_GROUP sweeps per launch, 3D: one), and the launch
  // counts per stage are odd.  row(s0, s1) gives the list prefix of a launch
  // of sweeps s0..s1 (1-based) from the stage's cone (see levelset.h):
  //   u_nn grows from K2:            radius s1
  //   u_n grows from u_nn's support: radius ASLAM_ITERS + s1
  //   u shrinks to the read region:  radius LS_READ_REACH + ASLAM_ITERS - s0 + 1
  //   the speed grows from |rho| < h: SV radius s1
  const int group = (DIM == 2) ? SWEEP_GROUP : 1;
  // the maximum speed through the slots (and a fold) where some speed list
  // is long, or its size is unknown when recorded
  const int nslot = (dev || b.vmax_tiles >= LS_VMAX_SLOT_MIN) ? LS_VMAX_SLOTS : 1;
  // nf: fields swept (2: also the second field of the instances that have
  // one, on the arrays FOFF after a0, a1, src)
  auto stage = [&](auto row, auto cone, int a0, int a1, int src, int bit, int sign_rho, int sweeps, int do_max,
                   int dil, int nf) -> int {
    int v = a0, t = a1;
    for (int done = 0; done < sweeps;) {
      const int ns = (sweeps - done < group) ? sweeps - done : group;
      const int mx = (do_max && done + ns == sweeps) ? 1 : 0;
      const int r = row(done + 1, done + ns);
      if (grid(r) > 0) {
        const dim3 g3(dev ? device_grid(b, r) : ext_grid(b.total[r]));
        if (DIM == 2 && nf == 2)
          hipLaunchKernelGGL(extend_group_kernel<2>, dim3(grid(r)), B, 0, st, I, off, n, r, v, t, src, bit, sign_rho,
                             mx, ns, dil, nslot);
        else if (DIM == 2)
          hipLaunchKernelGGL(extend_group_kernel<1>, dim3(grid(r)), B, 0, st, I, off, n, r, v, t, src, bit, sign_rho,
                             mx, ns, dil, nslot);
        else if (nf == 2)
          hipLaunchKernelGGL((extend_kernel<DIM, EXT_NPT, 2>), g3, B, 0, st, I, off, n, r, v, t, src, bit, sign_rho, mx,
                             dil, cone(done + 1), nslot);
        else
          hipLaunchKernelGGL((extend_kernel<DIM, EXT_NPT, 1>), g3, B, 0, st, I, off, n, r, v, t, src, bit, sign_rho, mx,
                             dil, cone(done + 1), nslot);
        if (hipGetLastError() != hipSuccess) return -1;
      }
      done += ns;
      const int x = v; v = t; t = x;
    }
    return v;
  };
  static_assert((ASLAM_ITERS + SWEEP_GROUP - 1) / SWEEP_GROUP % 2 == 1 && ASLAM_ITERS % 2 == 1,
                "the Aslam stages must end in the partner array");
  static_assert((VEL_ITERS + SWEEP_GROUP - 1) / SWEEP_GROUP % 2 == 0 && VEL_ITERS % 2 == 0,
                "the speed extension must end in V");
  static_assert(LS_READ_REACH + ASLAM_ITERS <= LS_C_MAX, "the u stage's cone must lie in list SC");
  static_assert(LS_READ_REACH <= ASLAM_ITERS, "the distance is dilated by the u_nn (and 3D: u_n) sweeps");
  // The u_nn stage (lists growing one node per sweep from the computational
  // points) also dilates the distance to them; in 3D so does the u_n stage,
  // and every 3D Aslam sweep skips the nodes beyond its node cone (u_nn
  // sweep s: distance <= s; u_n: ASLAM_ITERS + s; u: LS_READ_REACH +
  // ASLAM_ITERS - s + 1, where the distance is exact after the 2 *
  // ASLAM_ITERS dilations).  2D keeps the tile cones.
  auto cap = [](int r) { return r < LS_C_MAX ? r : LS_C_MAX; };
  const bool nc = DIM == 3;
  auto no_cone = [](int) { return -1; };
  const int nf = b.nf;
  const int unn = stage([&](int, int s1) { return LS_ROW_C + cap(s1); }, [&](int s) { return nc ? s : -1; }, A_E2, A_E3,
                        -1, 2, 0, ASLAM_ITERS, 0, 1, nf);
  const int un = stage([&](int, int s1) { return LS_ROW_C + cap(ASLAM_ITERS + s1); },
                       [&](int s) { return nc ? ASLAM_ITERS + s : -1; }, A_E1, A_E2, A_E3, 1, 0, ASLAM_ITERS, 0,
                       nc ? 1 : 0, nf);
  const int uext = stage([&](int s0, int) { return LS_ROW_C + cap(LS_READ_REACH + ASLAM_ITERS - s0 + 1); },
                         [&](int s) { return nc ? LS_READ_REACH + ASLAM_ITERS - s + 1 : -1; }, A_E0, A_E1, A_E2, 0, 0,
                         ASLAM_ITERS, 0, 0, nf);
  if (unn != A_E3 || un != A_E2 || uext != A_E1) return hipErrorUnknown;
  b.uext = uext;
  // Stefan speed, extension V <-> S (ends in V), maximum on the last sweep
  LL(LS_ROW_V + VEL_ITERS + 1, velocity_kernel, b.uext);
  auto vcap = [](int r) { return r < LS_V_MAX ? r : LS_V_MAX; };
  if (stage([&](int, int s1) { return LS_ROW_V + vcap(s1); }, no_cone, A_V, A_S, -1, 3, 1, VEL_ITERS, 1, 0, 1) != A_V)
    return hipErrorUnknown;
  if (nslot > 1) {
    hipLaunchKernelGGL(vmax_fold_kernel, dim3(n), dim3(LS_VMAX_SLOTS), 0, st, I);
    if (hipGetLastError() != hipSuccess) return hipErrorUnknown;
  }
#undef LL
  return hipSuccess;
}

template <int DIM>
hipError_t end_dim(LevelsetBatch& b, hipStream_t st) {
  const int n = b.count;
  const LsInst* I = b.d_inst;
  const int* off = b.d_off;
  const dim3 B(256);
  const bool dev = b.device_sized;
  auto grid = [&](int row) { return dev ? device_grid(b, row) : b.total[row]; };
  // advection substeps: from the maximum speeds on the host, or the most
  // the front guard allows (each instance skips those beyond its own count)
  int nsub = 1;
  if (dev) {
    nsub = LS_MAX_SUBSTEPS;
  } else {
    for (int i = 0; i < n; ++i) {
      int ns = (int)ceil(b.h_vmax[i] * b.dt / (0.5 * b.h_inst[i].h));
      if (ns < 1) ns = 1;
      if (ns > nsub) nsub = ns;
    }
  }
  hipError_t e;
  const int rrow = LS_ROW_V + LS_V_MAX;
  if (grid(rrow) > 0) {
    for (int q = 0; q < nsub; ++q)
      for (int s = 1; s <= 3; ++s) {
        hipLaunchKernelGGL(rk_kernel<DIM>, dim3(grid(rrow)), B, 0, st, I, off, n, 0, s, q, b.dt, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
  }
  if (b.reinit) {
    hipLaunchKernelGGL(reinit_check_kernel<DIM>, dim3(grid(LS_ROW_FULL)), B, 0, st, I, off, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (grid(rrow) > 0) {
      for (int it = 0; it < REINIT_ITERS; ++it)
        for (int s = 1; s <= 3; ++s) {
          hipLaunchKernelGGL(rk_kernel<DIM>, dim3(grid(rrow)), B, 0, st, I, off, n, 1, s, 0, 0.0,
                             (it == 0 && s == 1) ? 1 : 0);
          if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
  }
  hipLaunchKernelGGL(restrict_kernel<DIM>, dim3(grid(LS_ROW_FULL)), B, 0, st, I, off, n, b.uext);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  mark_clean(b);
  return hipSuccess;
}

// The whole-box clear of the dirty instances alone (exact grid).
template <int DIM>
hipError_t zero_only(LevelsetBatch& b, hipStream_t st) {
  if (b.total[LS_ROW_FULL] > 0)
    hipLaunchKernelGGL(zero_kernel<DIM>, dim3(b.total[LS_ROW_FULL]), dim3(256), 0, st, b.d_inst, b.d_off, b.count);
  return hipGetLastError();
}

}  // namespace

hipError_t levelset_alloc(LevelsetScratch& s, size_t nodes) {
  s.nodes = nodes;
  hipError_t e = hipMalloc(&s.buf, sizeof(double) * nodes * A_COUNT);
  if (e != hipSuccess) return e;
  // every array starts finite (sweeps may read arrays outside their lists)
  e = hipMemset(s.buf, 0, sizeof(double) * nodes * A_COUNT);
  if (e != hipSuccess) return e;
  e = hipMalloc(&s.known, nodes);
  if (e != hipSuccess) return e;
  e = hipMemset(s.known, 0, nodes);
  if (e != hipSuccess) return e;
  e = hipMalloc(&s.dist, nodes);
  if (e != hipSuccess) return e;
  e = hipMemset(s.dist, 255, nodes);
  s.dirty = e != hipSuccess;
  return e;
}

void levelset_free(LevelsetScratch& s) {
  if (s.buf) (void)hipFree(s.buf);
  if (s.known) (void)hipFree(s.known);
  if (s.dist) (void)hipFree(s.dist);
  s = LevelsetScratch{};
}

hipError_t levelset_batch_alloc(LevelsetBatch& b, int count, int dim) {
  b.count = count;
  b.dim = dim;
  hipError_t e;
  if ((e = hipMalloc(&b.d_inst, sizeof(LsInst) * count)) != hipSuccess) return e;
  if ((e = hipHostMalloc(&b.h_inst, sizeof(LsInst) * count)) != hipSuccess) return e;
  if ((e = hipMalloc(&b.d_off, sizeof(int) * LS_NROWS * (count + 1))) != hipSuccess) return e;
  if ((e = hipHostMalloc(&b.h_off, sizeof(int) * LS_NROWS * (count + 1))) != hipSuccess) return e;
  if ((e = hipMalloc(&b.d_vmax, sizeof(double) * count)) != hipSuccess) return e;
  if ((e = hipHostMalloc(&b.h_vmax, sizeof(double) * count)) != hipSuccess) return e;
  if ((e = hipMemset(b.d_vmax, 0, sizeof(double) * count)) != hipSuccess) return e;
  if ((e = hipMalloc(&b.d_vslot, sizeof(double) * LS_VMAX_SLOTS * count)) != hipSuccess) return e;
  if ((e = hipMemset(b.d_vslot, 0, sizeof(double) * LS_VMAX_SLOTS * count)) != hipSuccess) return e;
  for (int i = 0; i < count; ++i) b.h_inst[i] = LsInst{};
  return hipSuccess;
}

void levelset_batch_free(LevelsetBatch& b) {
  if (b.d_inst) (void)hipFree(b.d_inst);
  if (b.h_inst) (void)hipHostFree(b.h_inst);
  if (b.d_off) (void)hipFree(b.d_off);
  if (b.h_off) (void)hipHostFree(b.h_off);
  if (b.d_vmax) (void)hipFree(b.d_vmax);
  if (b.d_vslot) (void)hipFree(b.d_vslot);
  if (b.h_vmax) (void)hipHostFree(b.h_vmax);
  b = LevelsetBatch{};
}

namespace {

// Launch offsets of the lists and the device copy of the instance table.
hipError_t upload(LevelsetBatch& b, hipStream_t st) {
  const int n = b.count;
  for (int q = 0; q < LS_NROWS; ++q) {
    int acc = 0;
    for (int i = 0; i < n; ++i) {
      const LsInst& I = b.h_inst[i];
      b.h_off[q * (n + 1) + i] = acc;
      if (q == LS_ROW_FULL) acc += I.ntx * I.nty * I.ntz;
      else if (q == LS_ROW_U) acc += I.nu;
      else if (q >= LS_ROW_V) acc += I.ncum_v[q - LS_ROW_V];
      else acc += I.ncum_c[q - LS_ROW_C];
    }
    b.h_off[q * (n + 1) + n] = acc;
    b.total[q] = acc;
  }
  b.any_dirty = false;
  b.nf = 1;
  b.vmax_tiles = 0;
  for (int i = 0; i < n; ++i) {
    LsInst& I = b.h_inst[i];
    if (I.f) b.nf = 2;
    const int nv = I.ncum_v[VEL_ITERS < LS_V_MAX ? VEL_ITERS : LS_V_MAX];
    if (nv > b.vmax_tiles) b.vmax_tiles = nv;
    I.vmax = b.d_vmax + i;
    I.vslot = b.d_vslot + (size_t)LS_VMAX_SLOTS * i;
    // an instance without a host flag is always cleared first
    I.dirty = (!I.host_dirty || *I.host_dirty) ? 1 : 0;
    b.any_dirty = b.any_dirty || I.dirty;
    if (I.host_dirty) *I.host_dirty = true;   // until its restriction is enqueued
  }
  hipError_t e;
  if ((e = hipMemcpyAsync(b.d_inst, b.h_inst, sizeof(LsInst) * n, hipMemcpyHostToDevice, st)) != hipSuccess)
    return e;
  return hipMemcpyAsync(b.d_off, b.h_off, sizeof(int) * LS_NROWS * (n + 1), hipMemcpyHostToDevice, st);
}

}  // namespace

hipError_t levelset_begin(LevelsetBatch& b, double dt, int reinit, hipStream_t st) {
  b.dt = dt;
  b.reinit = reinit;
  hipError_t e;
  if (b.device_sized) {
    // the table is on the device (levelset_upload); the rows from the
    // geometry counters
    hipLaunchKernelGGL(ls_rows_kernel, dim3(1), dim3(128), 0, st, b.d_inst, b.d_off, b.count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  } else if ((e = upload(b, st)) != hipSuccess) {
    return e;
  }
  e = (b.dim == 2) ? begin_dim<2>(b, st) : begin_dim<3>(b, st);
  if (e != hipSuccess) return e;
  if (b.device_sized) {
    hipLaunchKernelGGL(front_check_kernel, dim3((b.count + 63) / 64), dim3(64), 0, st, b.d_inst, b.count, dt);
    return hipGetLastError();
  }
  return hipMemcpyAsync(b.h_vmax, b.d_vmax, sizeof(double) * b.count, hipMemcpyDeviceToHost, st);
}

hipError_t levelset_upload(LevelsetBatch& b, hipStream_t st) {
  const int n = b.count;
  hipError_t e = upload(b, st);   // table, dirty flags, offsets of the current lists
  if (e != hipSuccess) return e;
  if (b.any_dirty) {
    // clear the dirty scratch now, with exact grids: the captured passes
    // then start from clean arrays, and their restrictions keep them so
    const bool dev = b.device_sized;
    b.device_sized = false;
    e = (b.dim == 2) ? zero_only<2>(b, st) : zero_only<3>(b, st);
    b.device_sized = dev;
    if (e != hipSuccess) return e;
    for (int i = 0; i < n; ++i) {
      b.h_inst[i].dirty = 0;
      if (b.h_inst[i].host_dirty) *b.h_inst[i].host_dirty = false;
    }
    b.any_dirty = false;
    e = hipMemcpyAsync(b.d_inst, b.h_inst, sizeof(LsInst) * n, hipMemcpyHostToDevice, st);
  }
  return e;
}

hipError_t levelset_end(LevelsetBatch& b, hipStream_t st) {
  return (b.dim == 2) ? end_dim<2>(b, st) : end_dim<3>(b, st);
}

}  // namespace etdfb
