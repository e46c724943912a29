// Geometry build for the embedded-boundary operator (Section 2 of the paper)
// and the box <-> tile-layout transfers.
//
// classify_kernel     inside <=> rho < 0; computational <=> inside and all
//                     2d face neighbours inside (outer box layer never);
//                     marks tiles that hold a computational point; a
//                     computational point within 2 layers of the box edge is
//                     a domain error.
// scan_tiles_kernel   active tiles -> slots in lexicographic tile order.
// tile_coeff_kernel   per active tile: computational / irregular bit masks and,
//                     per point of the tile, the diagonal weight sum
//                     c_p = sum over faces of 1 (Case 1), h/s = 1/(1+theta)
//                     (Case 2), 1 - w_p (Case 3), so that
//                     (A v)_p = beta/h^2 (sum_q v_q - c_p v_p); NOT_COMP
//                     marks the other points of the tile.
//
// Case 3 weight (ghost q of p whose next node on the line is inside): the
// linear interpolant through p and the closest boundary points x_G1 of q and
// x_G2 of p.  w_p is the ratio of signed distances of q and p to the plane
// (2D: line) through x_G1, x_G2 whose normal is the averaged level-set
// normal made orthogonal to x_G2 - x_G1; closest points are one projection
// step x - rho g/|g|^2 with g the central-difference gradient.  Degenerate
// configurations use w_p = rho_q / rho_p.  In 2D this equals the paper's RBF
// interpolant with a linear tail (eqs. 2.5-2.6), whose radial part vanishes
// for three centres.
#include <math.h>
#include <string.h>

#include "device_common.h"
#include "launch.h"

namespace etdfb {

using BoxDev = BoxHost;   // plain box description, the same on both sides

// Batched launches: block b of a launch over the instances of a table works
// for instance i with pre[i] <= b < pre[i+1] on its block b - pre[i].
__device__ __forceinline__ int instance_of(const int* __restrict__ pre, int count, int b) {
  int lo = 0, hi = count;   // pre[lo] <= b < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ size_t node_index(const BoxDev& b, int i, int j, int k) {
  return ((size_t)k * b.ny + j) * b.nx + i;
}

__device__ __forceinline__ int tile_of(const BoxDev& b, int i, int j, int k) {
  return ((k / b.tz) * b.nty + (j / b.ty)) * b.ntx + (i / b.tx);
}

// Node coordinates of a box index: 32-bit divisions where the box has
// fewer than 2^32 nodes (a 64-bit division costs several times as many
// instructions, and the whole-box kernels do one per node).
__device__ __forceinline__ void node_coords(const BoxDev& b, size_t id, int& i, int& j, int& k) {
  if ((size_t)b.nx * b.ny * b.nz <= 0xFFFFFFFFull) {
    const unsigned u = (unsigned)id, nx = (unsigned)b.nx, ny = (unsigned)b.ny;
    const unsigned q = u / nx;
    i = (int)(u - q * nx);
    k = (int)(q / ny);
    j = (int)(q - (unsigned)k * ny);
  } else {
    i = (int)(id % b.nx);
    j = (int)((id / b.nx) % b.ny);
    k = (int)(id / ((size_t)b.nx * b.ny));
  }
}

// Tile of a node: the tile extents are the fixed shapes (powers of two).
__device__ __forceinline__ int tile_of_node(const BoxDev& b, int i, int j, int k) {
  if (b.dim == 2)
    return ((unsigned)j / TileShape<2>::Y) * b.ntx + (unsigned)i / TileShape<2>::X;
  return (((unsigned)k / TileShape<3>::Z) * b.nty + (unsigned)j / TileShape<3>::Y) * b.ntx +
         (unsigned)i / TileShape<3>::X;
}

// Index of a node within its tile (x fastest).
__device__ __forceinline__ int tile_local(const BoxDev& b, int i, int j, int k) {
  if (b.dim == 2) return ((unsigned)j % TileShape<2>::Y) * TileShape<2>::X + (unsigned)i % TileShape<2>::X;
  return (((unsigned)k % TileShape<3>::Z) * TileShape<3>::Y + (unsigned)j % TileShape<3>::Y) * TileShape<3>::X +
         (unsigned)i % TileShape<3>::X;
}

__device__ __forceinline__ void classify_node(const BoxDev& b, const double* __restrict__ rho,
                                              uint8_t* __restrict__ mask, int* __restrict__ tile_flag,
                                              int* __restrict__ tile_vb, int* __restrict__ status, size_t id) {
  int i, j, k;
  node_coords(b, id, i, j, k);
  const bool inside = rho[id] < 0.0;
  bool comp = inside;
  if (comp) {
    if (i == 0 || i == b.nx - 1 || j == 0 || j == b.ny - 1) comp = false;
    if (b.dim == 3 && (k == 0 || k == b.nz - 1)) comp = false;
  }
  if (comp) {
    comp = rho[id - 1] < 0.0 && rho[id + 1] < 0.0 && rho[id - b.nx] < 0.0 && rho[id + b.nx] < 0.0;
    if (b.dim == 3) {
      const size_t sz = (size_t)b.nx * b.ny;
      comp = comp && rho[id - sz] < 0.0 && rho[id + sz] < 0.0;
    }
  }
  mask[id] = comp ? 2 : (inside ? 1 : 0);
  if (fabs(rho[id]) < b.dx) tile_vb[tile_of_node(b, i, j, k)] = 1;   // a node of the speed band
  if (comp) {
    tile_flag[tile_of_node(b, i, j, k)] = 1;
    bool edge = i < 2 || i > b.nx - 3 || j < 2 || j > b.ny - 3;
    if (b.dim == 3) edge = edge || k < 2 || k > b.nz - 3;
    if (edge) atomicCAS(status, 0, ST_DOMAIN);
  }
}

// Zero the tile flags and the per-build counters ([2..4]) of every instance;
// blocks over ceil(ntiles / 256) per instance (prefix pre).
__global__ __launch_bounds__(256) void geom_zero_kernel(const GeomInst* __restrict__ tab,
                                                        const int* __restrict__ pre, int count) {
  const int inst = instance_of(pre, count, (int)blockIdx.x);
  const GeomInst& I = tab[inst];
  const int t = (int)(blockIdx.x - pre[inst]) * 256 + (int)threadIdx.x;
  if (t < I.ntiles) {
    I.tile_flag[t] = 0;
    I.tile_vb[t] = 0;
  }
  if (blockIdx.x == (unsigned)pre[inst] && threadIdx.x < 3) I.counters[2 + threadIdx.x] = 0;
}

// Classification, 256 nodes per block (prefix over ceil(nodes / 256)).
__global__ __launch_bounds__(256) void classify_kernel(const GeomInst* __restrict__ tab,
                                                       const int* __restrict__ pre, int count) {
  const int inst = instance_of(pre, count, (int)blockIdx.x);
  const GeomInst& I = tab[inst];
  const size_t id = (size_t)(blockIdx.x - pre[inst]) * 256 + threadIdx.x;
  if (id < I.nodes) classify_node(I.b, I.rho, I.mask, I.tile_flag, I.tile_vb, I.counters + 1, id);
}

// One block of 1024 threads per instance: exclusive scan of tile flags, in
// chunks of SCAN_CHUNK tiles: the chunk's flags are loaded coalesced into
// LDS (bytes), thread t counts the flags of its run of SCAN_CHUNK / 1024
// consecutive tiles there, one block scan gives each run its first slot,
// the runs write their slots into LDS, and the chunk's tile map is stored
// coalesced (the slot -> tile entries at the active tiles only).
constexpr int SCAN_CHUNK = 8192;

__global__ __launch_bounds__(1024) void scan_tiles_kernel(const GeomInst* __restrict__ tab) {
  constexpr int RUN = SCAN_CHUNK / 1024;
  const GeomInst& I = tab[blockIdx.x];
  const int* __restrict__ tile_flag = I.tile_flag;
  const int ntiles = I.ntiles;
  int* __restrict__ tile_map = I.tile_map;
  int* __restrict__ slot_tile = I.slot_tile;
  __shared__ uint8_t fl[SCAN_CHUNK];
  __shared__ int sl[SCAN_CHUNK];
  __shared__ int wave_tot[16];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int base = 0; base < ntiles; base += SCAN_CHUNK) {
    const int n = min(SCAN_CHUNK, ntiles - base);
#pragma unroll
    for (int k = threadIdx.x; k < SCAN_CHUNK; k += 1024) fl[k] = (k < n && tile_flag[base + k] != 0) ? 1 : 0;
    __syncthreads();
    const int r0 = (int)threadIdx.x * RUN;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < RUN; ++k) cnt += fl[r0 + k];
    int x = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wave_tot[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = carry;
      for (int q = 0; q < 16; ++q) { const int v = wave_tot[q]; wave_tot[q] = acc; acc += v; }
      carry = acc;
    }
    __syncthreads();
    int slot = wave_tot[w] + x - cnt;
#pragma unroll
    for (int k = 0; k < RUN; ++k) sl[r0 + k] = fl[r0 + k] ? slot++ : -1;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += 1024) {
      const int v = sl[k];
      tile_map[base + k] = v;
      if (v >= 0) slot_tile[v] = base + k;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) I.counters[0] = carry;   // active tiles
}

// L1 distances on the tile grid (level-set bands), one axis of a separable
// min-plus transform: the node gap between tiles k apart along an axis of
// tile extent t is (k-1) t + 1 (0 for k = 0).  Packed per tile: distance
// from a tile with a computational point in the low 16 bits, from a tile
// with a node |rho| < h in the high 16 bits; the first pass (axis 0) starts
// from the two flag arrays.
// Blocks over ceil(ntiles / 256) per instance (prefix pre); the pass of
// axis a reads band_tmp[(a+1) % 2] (axis 0: the flags) and writes
// band_tmp[a % 2], each half of the instance's 2 * ntiles scratch.  r: tile
// radius per axis (3 entries).
__global__ __launch_bounds__(256) void band_dist_kernel(const GeomInst* __restrict__ tab,
                                                        const int* __restrict__ pre, int count, int axis,
                                                        int r0, int r1, int r2, int cap) {
  const int inst = instance_of(pre, count, (int)blockIdx.x);
  const GeomInst& I = tab[inst];
  const BoxDev& b = I.b;
  const int ntiles = I.ntiles;
  const int* __restrict__ comp_flag = I.tile_flag;
  const int* __restrict__ vb_flag = I.tile_vb;
  const int* __restrict__ in = I.band_tmp + (size_t)((axis + 1) & 1) * ntiles;
  int* __restrict__ out = I.band_tmp + (size_t)(axis & 1) * ntiles;
  const int r = axis == 0 ? r0 : (axis == 1 ? r1 : r2);
  const int n[3] = {b.ntx, b.nty, b.ntz};
  const int text[3] = {b.tx, b.ty, b.tz};
  {
    const int t = (int)(blockIdx.x - pre[inst]) * 256 + (int)threadIdx.x;
    if (t >= ntiles) return;
    int c[3] = {t % b.ntx, (t / b.ntx) % b.nty, t / (b.ntx * b.nty)};
    const int c0 = c[axis];
    int dc = cap, dv = cap;
    for (int d = -r; d <= r; ++d) {
      const int x = c0 + d;
      if (x < 0 || x >= n[axis]) continue;
      c[axis] = x;
      const int tn = (c[2] * b.nty + c[1]) * b.ntx + c[0];
      int sc, sv;
      if (axis == 0) {
        sc = comp_flag[tn] != 0 ? 0 : cap;
        sv = vb_flag[tn] != 0 ? 0 : cap;
      } else {
        sc = in[tn] & 0xFFFF;
        sv = in[tn] >> 16;
      }
      const int k = d < 0 ? -d : d;
      const int gap = k == 0 ? 0 : (k - 1) * text[axis] + 1;
      dc = min(dc, sc + gap);
      dv = min(dv, sv + gap);
    }
    out[t] = min(dc, cap) | (min(dv, cap) << 16);
  }
}

// One block of 1024 threads per instance: the level-set tile lists from the
// packed distances.  SC: tiles with Dc <= cmax sorted by Dc; SV: tiles with
// Dv <= vmax sorted by Dv (counting sort; the order within one distance is
// that of the atomic cursors, which no result depends on); U: SC or SV.
// The cumulative counts of SC and SV per radius go to counters[cnt_c + r]
// and counters[cnt_v + r], the size of U to counters[cnt_u].
__global__ __launch_bounds__(1024) void band_lists_kernel(const GeomInst* __restrict__ tab, int last_axis, int cmax,
                                                          int vmax, int cnt_c, int cnt_v, int cnt_u) {
  constexpr int NB = 128;   // histogram bins (>= cmax + 1, vmax + 1)
  const GeomInst& I = tab[blockIdx.x];
  const int ntiles = I.ntiles;
  const int* __restrict__ dist = I.band_tmp + (size_t)(last_axis & 1) * ntiles;
  int* __restrict__ sc = I.band_list;
  int* __restrict__ sv = I.band_list + ntiles;
  int* __restrict__ su = I.band_list + 2 * (size_t)ntiles;
  __shared__ int hc[NB], hv[NB], nu;
  for (int q = threadIdx.x; q < NB; q += blockDim.x) { hc[q] = 0; hv[q] = 0; }
  if (threadIdx.x == 0) nu = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
    const int dc = dist[t] & 0xFFFF, dv = dist[t] >> 16;
    if (dc <= cmax) atomicAdd(&hc[dc], 1);
    if (dv <= vmax) atomicAdd(&hv[dv], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // cumulative counts out, histograms -> start offsets
    int a = 0;
    for (int q = 0; q <= cmax; ++q) { const int c = hc[q]; hc[q] = a; a += c; I.counters[cnt_c + q] = a; }
    a = 0;
    for (int q = 0; q <= vmax; ++q) { const int c = hv[q]; hv[q] = a; a += c; I.counters[cnt_v + q] = a; }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
    const int dc = dist[t] & 0xFFFF, dv = dist[t] >> 16;
    if (dc <= cmax) sc[atomicAdd(&hc[dc], 1)] = t;
    if (dv <= vmax) sv[atomicAdd(&hv[dv], 1)] = t;
    if (dc <= cmax || dv <= vmax) su[atomicAdd(&nu, 1)] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) I.counters[cnt_u] = nu;
}

__device__ __forceinline__ void central_grad(const BoxDev& b, const double* __restrict__ rho, int i,
                                             int j, int k, double g[3]) {
  const size_t id = node_index(b, i, j, k);
  const double inv = 1.0 / (2.0 * b.dx);
  g[0] = (rho[id + 1] - rho[id - 1]) * inv;
  g[1] = (rho[id + b.nx] - rho[id - b.nx]) * inv;
  g[2] = 0.0;
  if (b.dim == 3) {
    const size_t sz = (size_t)b.nx * b.ny;
    g[2] = (rho[id + sz] - rho[id - sz]) * inv;
  }
}

__device__ double case3_weight(const BoxDev& b, const double* __restrict__ rho, const int p[3],
                               const int q[3]) {
  const int D = b.dim;
  const double rp = rho[node_index(b, p[0], p[1], p[2])];
  const double rq = rho[node_index(b, q[0], q[1], q[2])];
  const double fallback = rq / rp;
  double gp[3], gq[3];
  central_grad(b, rho, p[0], p[1], p[2], gp);
  central_grad(b, rho, q[0], q[1], q[2], gq);
  double ggp = 0.0, ggq = 0.0;
  for (int d = 0; d < D; ++d) { ggp += gp[d] * gp[d]; ggq += gq[d] * gq[d]; }
  if (ggp < 1e-300 || ggq < 1e-300) return fallback;
  double xp[3], xq[3], g1[3], g2[3];
  for (int d = 0; d < D; ++d) {
    xp[d] = b.lo[d] + b.dx * p[d];
    xq[d] = b.lo[d] + b.dx * q[d];
    g1[d] = xq[d] - rq * gq[d] / ggq;
    g2[d] = xp[d] - rp * gp[d] / ggp;
  }
  const double np_ = sqrt(ggp), nq_ = sqrt(ggq);
  double ng[3] = {0.0, 0.0, 0.0};
  double nn = 0.0;
  for (int d = 0; d < D; ++d) { ng[d] = gq[d] / nq_ + gp[d] / np_; nn += ng[d] * ng[d]; }
  nn = sqrt(nn);
  if (nn < 1e-12) return fallback;
  double nbar[3];
  for (int d = 0; d < D; ++d) nbar[d] = ng[d] / nn;
  double t[3];
  double L = 0.0;
  for (int d = 0; d < D; ++d) { t[d] = g2[d] - g1[d]; L += t[d] * t[d]; }
  L = sqrt(L);
  double nu[3];
  if (L < 1e-12 * b.dx) {
    if (D == 2) return fallback;
    for (int d = 0; d < D; ++d) nu[d] = nbar[d];
  } else {
    double dot = 0.0;
    for (int d = 0; d < D; ++d) { t[d] /= L; dot += nbar[d] * t[d]; }
    double nl = 0.0;
    for (int d = 0; d < D; ++d) { nu[d] = nbar[d] - dot * t[d]; nl += nu[d] * nu[d]; }
    nl = sqrt(nl);
    if (nl < 1e-8) return fallback;
    for (int d = 0; d < D; ++d) nu[d] /= nl;
  }
  double dp = 0.0, dq = 0.0;
  for (int d = 0; d < D; ++d) { dp += (xp[d] - g1[d]) * nu[d]; dq += (xq[d] - g1[d]) * nu[d]; }
  if (fabs(dp) < 1e-10 * b.dx) return fallback;
  return dq / dp;
}

// Case 3 with boundary data: the weights of u_p and of the boundary values
// at the closest points x_G1 (of q) and x_G2 (of p) in the ghost value
// u_q = w_p u_p + w_1 u(x_G1) + w_2 u(x_G2), and the two points.  w_p is
// case3_weight's.  2D: the linear interpolant through p, x_G1, x_G2 (the
// paper's RBF with a linear tail, eqs. 2.5-2.6), so (w_p, w_1, w_2) are the
// barycentric coordinates of q; 3D (the plane reading): the boundary part
// 1 - w_p shared equally by the two points.  Degenerate configurations:
// one point, x_G1 (or x_q when rho has no gradient at q), with weight
// 1 - w_p (fallback != 0).
__device__ void case3_taps(const BoxDev& b, const double* __restrict__ rho, const int p[3], const int q[3],
                           double& wp, double& w1, double& w2, double g1[3], double g2[3], int& fallback) {
  const int D = b.dim;
  wp = case3_weight(b, rho, p, q);
  const double rp = rho[node_index(b, p[0], p[1], p[2])];
  const double rq = rho[node_index(b, q[0], q[1], q[2])];
  double gp[3], gq[3];
  central_grad(b, rho, p[0], p[1], p[2], gp);
  central_grad(b, rho, q[0], q[1], q[2], gq);
  double ggp = 0.0, ggq = 0.0;
  for (int d = 0; d < D; ++d) { ggp += gp[d] * gp[d]; ggq += gq[d] * gq[d]; }
  double xp[3] = {0.0, 0.0, 0.0}, xq[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < 3; ++d) { g1[d] = 0.0; g2[d] = 0.0; }
  for (int d = 0; d < D; ++d) {
    xp[d] = b.lo[d] + b.dx * p[d];
    xq[d] = b.lo[d] + b.dx * q[d];
  }
  const bool have_q = ggq >= 1e-300, have_p = ggp >= 1e-300;
  for (int d = 0; d < D; ++d) {
    g1[d] = have_q ? xq[d] - rq * gq[d] / ggq : xq[d];
    g2[d] = have_p ? xp[d] - rp * gp[d] / ggp : xp[d];
  }
  // the non-degenerate cases of case3_weight, re-derived for the flag
  fallback = 1;
  if (have_q && have_p) {
    const double np_ = sqrt(ggp), nq_ = sqrt(ggq);
    double ng[3] = {0.0, 0.0, 0.0}, nn = 0.0;
    for (int d = 0; d < D; ++d) { ng[d] = gq[d] / nq_ + gp[d] / np_; nn += ng[d] * ng[d]; }
    nn = sqrt(nn);
    if (nn >= 1e-12) {
      double nbar[3], t[3], L = 0.0;
      for (int d = 0; d < D; ++d) { nbar[d] = ng[d] / nn; t[d] = g2[d] - g1[d]; L += t[d] * t[d]; }
      L = sqrt(L);
      double nu[3];
      bool ok = true;
      if (L < 1e-12 * b.dx) {
        if (D == 2) ok = false;
        else for (int d = 0; d < D; ++d) nu[d] = nbar[d];
      } else {
        double dot = 0.0;
        for (int d = 0; d < D; ++d) { t[d] /= L; dot += nbar[d] * t[d]; }
        double nl = 0.0;
        for (int d = 0; d < D; ++d) { nu[d] = nbar[d] - dot * t[d]; nl += nu[d] * nu[d]; }
        nl = sqrt(nl);
        if (nl < 1e-8) ok = false;
        else for (int d = 0; d < D; ++d) nu[d] /= nl;
      }
      if (ok) {
        double dp = 0.0;
        for (int d = 0; d < D; ++d) dp += (xp[d] - g1[d]) * nu[d];
        if (fabs(dp) >= 1e-10 * b.dx) fallback = 0;
      }
    }
  }
  if (fallback) {
    w1 = 1.0 - wp;
    w2 = 0.0;
    return;
  }
  if (D == 3) {
    w1 = 0.5 * (1.0 - wp);
    w2 = 0.5 * (1.0 - wp);
    return;
  }
  // 2D barycentric: q - g1 - w_p (p - g1) = w_2 (g2 - g1)
  double num = 0.0, den = 0.0;
  for (int d = 0; d < 2; ++d) {
    const double e = g2[d] - g1[d];
    num += ((xq[d] - g1[d]) - wp * (xp[d] - g1[d])) * e;
    den += e * e;
  }
  w2 = num / den;
  w1 = 1.0 - wp - w2;
}

// Variable beta (one instance; grid = one block per box tile, inactive tiles
// return): for each computational point and face f = (d, -/+) in the order
// -x,+x,-y,+y,-z,+z with beta_f = beta at the face midpoint:
//   q computational: w_f = beta_f/h^2, diagonal -= beta_f/h^2 (eq. 2.4);
//   Case 2: diagonal -= beta_f/(h s), tap beta_f/(h s) at the crossing;
//   Case 3: diagonal -= beta_f (1 - w_p)/h^2, taps beta_f w_G/h^2 at x_G1, x_G2;
// ghost faces have w_f = 0 (the neighbour is not an unknown).
__global__ __launch_bounds__(256) void tile_var_kernel(const GeomInst* __restrict__ tab) {
  const GeomInst& I = tab[0];
  const BoxDev& b = I.b;
  const double* __restrict__ rho = I.rho;
  const uint8_t* __restrict__ mask = I.mask;
  const int t = (int)blockIdx.x;
  const int slot = I.tile_map[t];
  if (slot < 0) return;
  const int tcx = t % b.ntx, tcy = (t / b.ntx) % b.nty, tcz = t / (b.ntx * b.nty);
  const int l = threadIdx.x;
  const int lx = l % b.tx, ly = (l / b.tx) % b.ty, lz = l / (b.tx * b.ty);
  const int i = tcx * b.tx + lx, j = tcy * b.ty + ly, k = tcz * b.tz + lz;
  const size_t idx = (size_t)slot * TILE_PTS + l;
  const int D = b.dim;
  const double h2 = b.dx * b.dx;
  double wf[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double dg = 0.0;
  int nt = 0;
  bool comp = false;
  if (i < b.nx && j < b.ny && k < b.nz) {
    const size_t id = node_index(b, i, j, k);
    comp = mask[id] == 2;
    bool edge = i < 2 || i > b.nx - 3 || j < 2 || j > b.ny - 3;
    if (D == 3) edge = edge || k < 2 || k > b.nz - 3;
    if (comp && edge) comp = false;   // domain error (reported by classify_kernel)
  }
  if (comp) {
    const int p[3] = {i, j, k};
    for (int d = 0; d < D; ++d) {
      for (int s = -1; s <= 1; s += 2) {
        const int f = 2 * d + (s > 0 ? 1 : 0);
        int q[3] = {i, j, k};
        q[d] += s;
        const size_t qi = node_index(b, q[0], q[1], q[2]);
        const size_t lowi = s > 0 ? node_index(b, i, j, k) : qi;   // face midpoint = low node + h/2 e_d
        const double bf = I.beta_face[d][lowi];
        if (mask[qi] == 2) {
          wf[f] = bf / h2;
          dg -= bf / h2;
          continue;
        }
        int q2[3] = {q[0], q[1], q[2]};
        q2[d] += s;
        const double rq = rho[qi];
        const double rq2 = rho[node_index(b, q2[0], q2[1], q2[2])];
        const size_t tb = idx * TAPS_PER;
        if (!(rq2 < 0.0)) {
          const double theta = rq / (rq - rq2);
          const double dist = (1.0 + theta) * b.dx;
          const double cf = bf / (b.dx * dist);
          dg -= cf;
          I.tap_coef[tb + nt] = cf;
          for (int c = 0; c < 3; ++c) {
            double x = c < D ? b.lo[c] + b.dx * q[c] : 0.0;
            if (c == d) x += s * theta * b.dx;
            I.tap_pt[(tb + nt) * 3 + c] = x;
          }
          ++nt;
        } else {
          double wp, w1, w2, g1[3], g2[3];
          int fb;
          case3_taps(b, rho, p, q, wp, w1, w2, g1, g2, fb);
          dg -= bf * (1.0 - wp) / h2;
          I.tap_coef[tb + nt] = bf * w1 / h2;
          for (int c = 0; c < 3; ++c) I.tap_pt[(tb + nt) * 3 + c] = g1[c];
          ++nt;
          if (!fb) {
            I.tap_coef[tb + nt] = bf * w2 / h2;
            for (int c = 0; c < 3; ++c) I.tap_pt[(tb + nt) * 3 + c] = g2[c];
            ++nt;
          }
        }
      }
    }
  }
  for (int f = 0; f < 2 * D; ++f) I.vcoef[(size_t)f * I.ld + idx] = wf[f];
  I.vcoef[(size_t)(2 * D) * I.ld + idx] = comp ? dg : 0.0;
  I.tap_n[idx] = nt;
}

// Forcing vector in box layout: at computational points the sum of the
// point's taps coef * ub (in tap order), then plus src; 0 elsewhere.
__global__ void forcing_kernel(BoxDev b, const int* __restrict__ tile_map, const uint64_t* __restrict__ comp_bits,
                               const int* __restrict__ tap_n, const double* __restrict__ tap_coef,
                               const int* __restrict__ tap_off, const double* __restrict__ ub,
                               const double* __restrict__ src, double* __restrict__ out) {
  const size_t total = (size_t)b.nx * b.ny * b.nz;
  for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < total; id += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(id % b.nx);
    const int j = (int)((id / b.nx) % b.ny);
    const int k = (int)(id / ((size_t)b.nx * b.ny));
    const int slot = tile_map[tile_of(b, i, j, k)];
    double v = 0.0;
    if (slot >= 0) {
      const int l = (i % b.tx) + b.tx * ((j % b.ty) + b.ty * (k % b.tz));
      if (bit_of(comp_bits, slot, l)) {
        const size_t idx = (size_t)slot * TILE_PTS + l;
        double g = 0.0;
        const int n = tap_n[idx];
        for (int q = 0; q < n; ++q) g += tap_coef[idx * TAPS_PER + q] * ub[tap_off[idx] + q];
        v = src ? src[id] + g : g;
      }
    }
    out[id] = v;
  }
}

// Blocks loop over the instance's active tiles (slots, after the scan).
__device__ __forceinline__ void tile_coeff(const GeomInst& I, int slot);

__global__ __launch_bounds__(256) void tile_coeff_kernel(const GeomInst* __restrict__ tab,
                                                         const int* __restrict__ pre, int count) {
  const int inst = instance_of(pre, count, (int)blockIdx.x);
  const GeomInst& I = tab[inst];
  const int nblk = pre[inst + 1] - pre[inst];
  const int nact = I.counters[0];
  for (int slot = (int)blockIdx.x - pre[inst]; slot < nact; slot += nblk) tile_coeff(I, slot);
}

__device__ __forceinline__ void tile_coeff(const GeomInst& I, int slot) {
  const BoxDev& b = I.b;
  const double* __restrict__ rho = I.rho;
  const uint8_t* __restrict__ mask = I.mask;
  const int* __restrict__ tile_map = I.tile_map;
  uint64_t* __restrict__ comp_bits = I.comp_bits;
  uint64_t* __restrict__ irr_bits = I.irr_bits;
  double* __restrict__ cdiag = I.cdiag;
  int* __restrict__ nbr = I.nbr;
  int* __restrict__ counts = I.counters + 2;
  const int t = I.slot_tile[slot];
  const int tcx = t % b.ntx, tcy = (t / b.ntx) % b.nty, tcz = t / (b.ntx * b.nty);
  const int l = threadIdx.x;
  if (l < NBR_STRIDE) {
    // face-neighbour slots of the tile (-x,+x,-y,+y,-z,+z), -1 outside / inactive
    int s = -1;
    if (l < 2 * b.dim) {
      int cc[3] = {tcx, tcy, tcz};
      const int nn[3] = {b.ntx, b.nty, b.ntz};
      const int d = l >> 1;
      cc[d] += (l & 1) ? 1 : -1;
      if (cc[d] >= 0 && cc[d] < nn[d]) s = tile_map[((size_t)cc[2] * b.nty + cc[1]) * b.ntx + cc[0]];
    }
    nbr[(size_t)slot * NBR_STRIDE + l] = s;
  }
  const int lx = l % b.tx, ly = (l / b.tx) % b.ty, lz = l / (b.tx * b.ty);
  const int i = tcx * b.tx + lx, j = tcy * b.ty + ly, k = tcz * b.tz + lz;
  bool comp = false, irr = false;
  double c = 0.0;
  int n2 = 0, n3 = 0;
  if (i < b.nx && j < b.ny && k < b.nz) {
    const size_t id = node_index(b, i, j, k);
    comp = mask[id] == 2;
    bool edge = i < 2 || i > b.nx - 3 || j < 2 || j > b.ny - 3;
    if (b.dim == 3) edge = edge || k < 2 || k > b.nz - 3;
    if (comp && edge) {
      // domain error (reported by classify_kernel); keep every read in the box
      c = 2.0 * b.dim;
    } else if (comp) {
      const int p[3] = {i, j, k};
      for (int d = 0; d < b.dim; ++d) {
        for (int s = -1; s <= 1; s += 2) {
          int q[3] = {i, j, k};
          q[d] += s;
          const size_t qi = node_index(b, q[0], q[1], q[2]);
          if (mask[qi] == 2) {
            c += 1.0;
            continue;
          }
          irr = true;
          int q2[3] = {q[0], q[1], q[2]};
          q2[d] += s;
          const double rq = rho[qi];
          const double rq2 = rho[node_index(b, q2[0], q2[1], q2[2])];
          if (!(rq2 < 0.0)) {
            const double theta = rq / (rq - rq2);
            c += 1.0 / (1.0 + theta);
            ++n2;
          } else {
            c += 1.0 - case3_weight(b, rho, p, q);
            ++n3;
          }
        }
      }
    }
  }
  const uint64_t cb = __ballot(comp);
  const uint64_t ib = __ballot(irr);
  if ((l & 63) == 0) {
    comp_bits[(size_t)slot * 4 + (l >> 6)] = cb;
    irr_bits[(size_t)slot * 4 + (l >> 6)] = ib;
  }
  cdiag[(size_t)slot * TILE_PTS + l] = comp ? c : NOT_COMP;
  // Case 2 / Case 3 faces and computational points of the tile: one atomic
  // per counter and tile (a contended global atomic per thread serialises)
  __shared__ int red[3][4];
  int a = n2, b3 = n3;
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b3 += __shfl_xor(b3, o, 64);
  }
  if ((l & 63) == 0) {
    red[0][l >> 6] = a;
    red[1][l >> 6] = b3;
    red[2][l >> 6] = __popcll(cb);
  }
  __syncthreads();
  if (l < 3) {
    const int v = red[l][0] + red[l][1] + red[l][2] + red[l][3];
    if (v) atomicAdd(&counts[l], v);
  }
  __syncthreads();
}

// box -> tile layout (0 at non-computational points).  grid >= cap tiles.
__device__ __forceinline__ void gather_tile(const BoxDev& b, const double* __restrict__ box,
                                            const int* __restrict__ slot_tile,
                                            const uint64_t* __restrict__ comp_bits, int slot,
                                            double* __restrict__ vec) {
  const int t = slot_tile[slot];
  const int l = threadIdx.x;
  const int lx = l % b.tx, ly = (l / b.tx) % b.ty, lz = l / (b.tx * b.ty);
  const int i = (t % b.ntx) * b.tx + lx;
  const int j = ((t / b.ntx) % b.nty) * b.ty + ly;
  const int k = (t / (b.ntx * b.nty)) * b.tz + lz;
  double v = 0.0;
  if (bit_of(comp_bits, slot, l)) v = box[node_index(b, i, j, k)];
  vec[(size_t)slot * TILE_PTS + l] = v;
}

__device__ __forceinline__ void scatter_node(const BoxDev& b, const double* __restrict__ vec,
                                             const int* __restrict__ tile_map,
                                             const uint64_t* __restrict__ comp_bits, double* __restrict__ box,
                                             size_t id) {
  int i, j, k;
  node_coords(b, id, i, j, k);
  const int slot = tile_map[tile_of_node(b, i, j, k)];
  double v = 0.0;
  if (slot >= 0) {
    const int l = tile_local(b, i, j, k);
    if (bit_of(comp_bits, slot, l)) v = vec[(size_t)slot * TILE_PTS + l];
  }
  box[id] = v;
}

__global__ __launch_bounds__(256) void gather_kernel(BoxDev b, const double* __restrict__ box,
                                                     const int* __restrict__ slot_tile,
                                                     const uint64_t* __restrict__ comp_bits,
                                                     const int* __restrict__ n_active,
                                                     double* __restrict__ vec) {
  const int nact = *n_active;
  for (int slot = blockIdx.x; slot < nact; slot += gridDim.x) gather_tile(b, box, slot_tile, comp_bits, slot, vec);
}

// tile layout -> box: computational nodes get the vector, all others 0.
__global__ void scatter_kernel(BoxDev b, const double* __restrict__ vec, const int* __restrict__ tile_map,
                               const uint64_t* __restrict__ comp_bits, double* __restrict__ box) {
  const size_t total = (size_t)b.nx * b.ny * b.nz;
  for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < total;
       id += (size_t)gridDim.x * blockDim.x)
    scatter_node(b, vec, tile_map, comp_bits, box, id);
}

// tile layout -> box over the active tiles only: computational nodes get the
// vector, the tiles' other nodes 0; nodes outside the active tiles are not
// written.
__global__ __launch_bounds__(256) void scatter_tiles_kernel(BoxDev b, const double* __restrict__ vec,
                                                            const int* __restrict__ slot_tile,
                                                            const uint64_t* __restrict__ comp_bits,
                                                            const int* __restrict__ n_active,
                                                            double* __restrict__ box) {
  const int nact = *n_active;
  const int l = threadIdx.x;
  const int lx = l % b.tx, ly = (l / b.tx) % b.ty, lz = l / (b.tx * b.ty);
  for (int slot = blockIdx.x; slot < nact; slot += gridDim.x) {
    const int t = slot_tile[slot];
    const int i = (t % b.ntx) * b.tx + lx;
    const int j = ((t / b.ntx) % b.nty) * b.ty + ly;
    const int k = (t / (b.ntx * b.nty)) * b.tz + lz;
    if (i < b.nx && j < b.ny && k < b.nz)
      box[node_index(b, i, j, k)] = bit_of(comp_bits, slot, l) ? vec[(size_t)slot * TILE_PTS + l] : 0.0;
  }
}

// Batched transfers between the user box arrays boxes[i] and vector `vec`
// of each instance's workspace: gather with blocks looping over each
// instance's active tiles (prefix pre), scatter with 256 nodes per block
// (prefix pre).
__global__ __launch_bounds__(256) void gather_batch_kernel(const GeomInst* __restrict__ tab,
                                                           const int* __restrict__ pre, int count,
                                                           const double* const* __restrict__ boxes, int vec) {
  const int inst = instance_of(pre, count, (int)blockIdx.x);
  const GeomInst& I = tab[inst];
  const int nblk = pre[inst + 1] - pre[inst];
  for (int slot = (int)(blockIdx.x - pre[inst]); slot < I.counters[0]; slot += nblk)
    gather_tile(I.b, boxes[inst], I.slot_tile, I.comp_bits, slot, I.ws + (size_t)vec * I.ld);
}

__global__ __launch_bounds__(256) void scatter_batch_kernel(const GeomInst* __restrict__ tab,
                                                            const int* __restrict__ pre, int count,
                                                            double* const* __restrict__ boxes, int vec) {
  const int inst = instance_of(pre, count, (int)blockIdx.x);
  const GeomInst& I = tab[inst];
  const size_t id = (size_t)(blockIdx.x - pre[inst]) * 256 + threadIdx.x;
  if (id < I.nodes) scatter_node(I.b, I.ws + (size_t)vec * I.ld, I.tile_map, I.comp_bits, boxes[inst], id);
}

// Counters of every instance into one contiguous array (ncnt per instance).
__global__ void collect_counters_kernel(const GeomInst* __restrict__ tab, int count, int ncnt,
                                        int* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count * ncnt; e += gridDim.x * blockDim.x)
    out[e] = tab[e / ncnt].counters[e % ncnt];
}

// ------------------------------------------------------------ launchers

static int blocks_for(size_t n, int bs) {
  size_t g = (n + bs - 1) / bs;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t geom_batch_alloc(GeomBatch& gb, int count, int ncnt) {
  gb = GeomBatch{};
  gb.count = count;
  gb.ncnt = ncnt;
  hipError_t e;
  if ((e = hipHostMalloc(&gb.h_tab, sizeof(GeomInst) * count)) != hipSuccess) return e;
  if ((e = hipMalloc(&gb.d_tab, sizeof(GeomInst) * count)) != hipSuccess) return e;
  if ((e = hipHostMalloc(&gb.h_pre, sizeof(int) * GEOM_NPRE * (count + 1))) != hipSuccess) return e;
  if ((e = hipMalloc(&gb.d_pre, sizeof(int) * GEOM_NPRE * (count + 1))) != hipSuccess) return e;
  if ((e = hipHostMalloc(&gb.h_cnt, sizeof(int) * ncnt * count)) != hipSuccess) return e;
  if ((e = hipMalloc(&gb.d_cnt, sizeof(int) * ncnt * count)) != hipSuccess) return e;
  memset(gb.h_tab, 0, sizeof(GeomInst) * count);
  return hipSuccess;
}

void geom_batch_free(GeomBatch& gb) {
  if (gb.side) {
    (void)hipStreamSynchronize(gb.side);
    (void)hipStreamDestroy(gb.side);
  }
  if (gb.fork) (void)hipEventDestroy(gb.fork);
  if (gb.join) (void)hipEventDestroy(gb.join);
  if (gb.h_tab) (void)hipHostFree(gb.h_tab);
  if (gb.d_tab) (void)hipFree(gb.d_tab);
  if (gb.h_pre) (void)hipHostFree(gb.h_pre);
  if (gb.d_pre) (void)hipFree(gb.d_pre);
  if (gb.h_cnt) (void)hipHostFree(gb.h_cnt);
  if (gb.d_cnt) (void)hipFree(gb.d_cnt);
  gb = GeomBatch{};
}

// Block prefix sums of the table (sizes do not change after creation);
// synchronous upload.
hipError_t geom_batch_prefix(GeomBatch& gb) {
  const int n = gb.count;
  int* p = gb.h_pre;
  for (int q = 0; q < GEOM_NPRE; ++q) p[q * (n + 1)] = 0;
  for (int i = 0; i < n; ++i) {
    const GeomInst& I = gb.h_tab[i];
    for (int q = 0; q < GEOM_NPRE; ++q) p[q * (n + 1) + i + 1] = p[q * (n + 1) + i] + geom_blocks_per(q, I.nodes, I.ntiles);
  }
  for (int q = 0; q < GEOM_NPRE; ++q) gb.blocks[q] = p[q * (n + 1) + n];
  return hipMemcpy(gb.d_pre, gb.h_pre, sizeof(int) * GEOM_NPRE * (n + 1), hipMemcpyHostToDevice);
}

static const int* pre_of(const GeomBatch& gb, int q) { return gb.d_pre + q * (gb.count + 1); }

hipError_t geom_upload(GeomBatch& gb, hipStream_t s) {
  return hipMemcpyAsync(gb.d_tab, gb.h_tab, sizeof(GeomInst) * gb.count, hipMemcpyHostToDevice, s);
}

// Fewest tiles (summed over a table's instances) for which an eager build
// runs the distance chain beside the scan chain.
constexpr size_t GEOM_FORK_MIN_TILES = 16384;

hipError_t launch_geometry(GeomBatch& gb, const int* radii, hipStream_t s, bool device_sized) {
  const int n = gb.count;
  hipError_t e = hipSuccess;
  if (!device_sized && (e = geom_upload(gb, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(geom_zero_kernel, dim3(gb.blocks[GEOM_PRE_T256]), dim3(256), 0, s, gb.d_tab,
                     pre_of(gb, GEOM_PRE_T256), n);
  hipLaunchKernelGGL(classify_kernel, dim3(gb.blocks[GEOM_PRE_NODE]), dim3(256), 0, s, gb.d_tab,
                     pre_of(gb, GEOM_PRE_NODE), n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // The two chains that follow the classification touch disjoint data (the
  // scan and coefficients: tile map, slots, masks, diagonal weights,
  // counters 0 and 2-4; the distances and lists: their scratch, the lists,
  // the list counters).  Eager builds of large tables run the second on the
  // side stream, joined before the counters are collected (the fork and
  // join cost about 20 us, more than the overlap saves on small boxes);
  // device-sized builds (graph capture) keep one stream.
  size_t tiles = 0;
  for (int i = 0; i < n; ++i) tiles += (size_t)gb.h_tab[i].ntiles;
  hipStream_t s2 = s;
  if (!device_sized && tiles >= GEOM_FORK_MIN_TILES) {
    if (!gb.side) {
      if ((e = hipStreamCreateWithFlags(&gb.side, hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&gb.fork, hipEventDisableTiming)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&gb.join, hipEventDisableTiming)) != hipSuccess) return e;
    }
    if ((e = hipEventRecord(gb.fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(gb.side, gb.fork, 0)) != hipSuccess) return e;
    s2 = gb.side;
  }
  // tile radii of the distance passes: tiles k apart are >= (k-1) t + 1 nodes apart
  const int rmax = radii[0] > radii[1] ? radii[0] : radii[1];
  const BoxHost& b0 = gb.h_tab[0].b;
  const int dim = b0.dim;
  const int t[3] = {b0.tx, b0.ty, b0.tz};
  int r[3];
  for (int a = 0; a < 3; ++a) r[a] = (rmax - 1) / t[a] + 1;
  for (int axis = 0; axis < dim; ++axis)
    hipLaunchKernelGGL(band_dist_kernel, dim3(gb.blocks[GEOM_PRE_T256]), dim3(256), 0, s2, gb.d_tab,
                       pre_of(gb, GEOM_PRE_T256), n, axis, r[0], r[1], r[2], 1000);
  hipLaunchKernelGGL(band_lists_kernel, dim3(n), dim3(1024), 0, s2, gb.d_tab, dim - 1, radii[0], radii[1], radii[2],
                     radii[3], radii[4]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(n), dim3(1024), 0, s, gb.d_tab);
  hipLaunchKernelGGL(tile_coeff_kernel, dim3(gb.blocks[GEOM_PRE_TILE]), dim3(256), 0, s, gb.d_tab,
                     pre_of(gb, GEOM_PRE_TILE), n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (s2 != s) {
    if ((e = hipEventRecord(gb.join, s2)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, gb.join, 0)) != hipSuccess) return e;
  }
  if (device_sized) return hipSuccess;
  hipLaunchKernelGGL(collect_counters_kernel, dim3(blocks_for((size_t)n * gb.ncnt, 256)), dim3(256), 0, s,
                     gb.d_tab, n, gb.ncnt, gb.d_cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipMemcpyAsync(gb.h_cnt, gb.d_cnt, sizeof(int) * gb.ncnt * n, hipMemcpyDeviceToHost, s);
}

// m species (one instance): slots n .. m n - 1 repeat the n base slots (masks,
// diagonal weights, the tile of each slot; face-neighbour slots shifted into
// the same copy), counters[5] = m n and counters[6] = m N.
__global__ void replicate_species_kernel(const GeomInst* __restrict__ tab, int m) {
  const GeomInst& I = tab[0];
  const int n = I.counters[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    I.counters[5] = m * n;
    I.counters[6] = m * I.counters[4];
  }
  const long total = (long)(m - 1) * n * TILE_PTS;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int slot = n + (int)(e / TILE_PTS);
    const int l = (int)(e % TILE_PTS);
    const int base = slot % n, sp = slot / n;
    I.cdiag[(size_t)slot * TILE_PTS + l] = I.cdiag[(size_t)base * TILE_PTS + l];
    if (l < 4) {
      I.comp_bits[(size_t)slot * 4 + l] = I.comp_bits[(size_t)base * 4 + l];
      I.irr_bits[(size_t)slot * 4 + l] = I.irr_bits[(size_t)base * 4 + l];
    }
    if (l < NBR_STRIDE) {
      const int nb = I.nbr[(size_t)base * NBR_STRIDE + l];
      I.nbr[(size_t)slot * NBR_STRIDE + l] = nb >= 0 ? nb + sp * n : -1;
    }
    if (l == 0) I.slot_tile[slot] = I.slot_tile[base];
  }
}

hipError_t launch_replicate_species(GeomBatch& gb, int m, hipStream_t s) {
  hipLaunchKernelGGL(replicate_species_kernel, dim3(1024), dim3(256), 0, s, gb.d_tab, m);
  return hipGetLastError();
}

hipError_t launch_geometry_var(GeomBatch& gb, hipStream_t s) {
  hipLaunchKernelGGL(tile_var_kernel, dim3(gb.h_tab[0].ntiles), dim3(256), 0, s, gb.d_tab);
  return hipGetLastError();
}

hipError_t launch_forcing(const BoxHost& b, const int* tile_map, const uint64_t* comp_bits, const int* tap_n,
                          const double* tap_coef, const int* tap_off, const double* ub, const double* src,
                          double* out, hipStream_t s) {
  const size_t total = (size_t)b.nx * b.ny * b.nz;
  hipLaunchKernelGGL(forcing_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, b, tile_map, comp_bits, tap_n,
                     tap_coef, tap_off, ub, src, out);
  return hipGetLastError();
}

hipError_t launch_gather_batch(const GeomBatch& gb, const double* const* d_boxes, int vec, hipStream_t s) {
  hipLaunchKernelGGL(gather_batch_kernel, dim3(gb.blocks[GEOM_PRE_TILE]), dim3(256), 0, s, gb.d_tab,
                     pre_of(gb, GEOM_PRE_TILE), gb.count, d_boxes, vec);
  return hipGetLastError();
}

hipError_t launch_scatter_batch(const GeomBatch& gb, double* const* d_boxes, int vec, hipStream_t s) {
  hipLaunchKernelGGL(scatter_batch_kernel, dim3(gb.blocks[GEOM_PRE_NODE]), dim3(256), 0, s, gb.d_tab,
                     pre_of(gb, GEOM_PRE_NODE), gb.count, d_boxes, vec);
  return hipGetLastError();
}

hipError_t launch_gather(const BoxHost& b, const double* box, const int* slot_tile,
                         const uint64_t* comp_bits, const int* n_active, double* vec, int grid,
                         hipStream_t s) {
  hipLaunchKernelGGL(gather_kernel, dim3(grid), dim3(256), 0, s, b, box, slot_tile, comp_bits, n_active, vec);
  return hipGetLastError();
}

hipError_t launch_scatter_tiles(const BoxHost& b, const double* vec, const int* slot_tile,
                                const uint64_t* comp_bits, const int* n_active, double* box, int grid,
                                hipStream_t s) {
  hipLaunchKernelGGL(scatter_tiles_kernel, dim3(grid), dim3(256), 0, s, b, vec, slot_tile, comp_bits, n_active, box);
  return hipGetLastError();
}

hipError_t launch_scatter(const BoxHost& b, const double* vec, const int* tile_map,
                          const uint64_t* comp_bits, double* box, hipStream_t s) {
  const size_t n = (size_t)b.nx * b.ny * b.nz;
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, b, vec, tile_map, comp_bits,
                     box);
  return hipGetLastError();
}

}  // namespace etdfb
