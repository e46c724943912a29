// Device-side building blocks shared by the HIP kernels of libetdfb:
// the active-tile layout, the grid barrier of the persistent kernels and
// fixed-order (hence bitwise reproducible) reductions.
//
// Layout.  The box of n^d nodes is cut into tiles of 256 nodes
// (2D: 32 x 8, 3D: 16 x 4 x 4, x fastest inside a tile).  Only tiles that
// hold at least one computational point ("active" tiles) get storage; a
// vector is `slot * 256 + local` over the active slots, in lexicographic tile
// order.  Every vector is 0 at the non-computational nodes of active tiles,
// and nodes of inactive tiles read as 0, so the stencil never needs a mask for
// its neighbours.  Per active tile: a 256-bit mask of computational points, a
// 256-bit mask of "irregular" points (a neighbour face of Case 2 or 3) and,
// for irregular points only, the diagonal weight sum stored at slot*256+local.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "etdfb_internal.h"

namespace etdfb {

// Pointers typed in the global address space: device buffers accessed
// through them compile to global (not flat) loads and stores.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <class T>
using gptr = T*;   // host pass: address spaces play no role
#endif

template <class T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// Wave-uniform copies (lane 0's value) of a pointer and of a double: values
// the compiler cannot prove uniform (read from LDS, say) then live in scalar
// registers, and loads through the pointer take a scalar base address.
template <class T>
__device__ __forceinline__ gptr<T> uniform(gptr<T> p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (gptr<T>)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double uniform(double x) {
  const unsigned long long v = __double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Element i of an array through a 32-bit byte offset (a scalar base plus one
// offset register per lane).  Arrays addressed this way stay below 4 GiB.
template <class T>
__device__ __forceinline__ T at(gptr<const T> p, unsigned i) {
  return *(gptr<const T>)((gptr<const char>)p + i * (unsigned)sizeof(T));
}

template <class T>
__device__ __forceinline__ void put(gptr<T> p, unsigned i, T v) {
  *(gptr<T>)((gptr<char>)p + i * (unsigned)sizeof(T)) = v;
}

// Pointers typed in the LDS address space (ds_ instructions, not flat).
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using lptr = __attribute__((address_space(3))) T*;
#else
template <class T>
using lptr = T*;
#endif

template <class T>
__device__ __forceinline__ lptr<T> lds(T* p) {
  return (lptr<T>)p;
}

template <int DIM> struct TileShape;
template <> struct TileShape<2> { static constexpr int X = 32, Y = 8, Z = 1; };
template <> struct TileShape<3> { static constexpr int X = 16, Y = 4, Z = 4; };

__device__ __forceinline__ bool bit_of(const uint64_t* bits, int slot, int l) {
  return (bits[(size_t)slot * 4 + (l >> 6)] >> (l & 63)) & 1ull;
}

// Face-neighbour slot of a tile in direction dir (order -x,+x,-y,+y,-z,+z);
// -1 if outside the box or inactive.
template <int DIM>
__device__ __forceinline__ int face_neighbour_slot(const GeomDev& g, int slot, int dir) {
  int t = g.slot_tile[slot];
  int c[3] = {t % g.ntx, (t / g.ntx) % g.nty, t / (g.ntx * g.nty)};
  int n[3] = {g.ntx, g.nty, g.ntz};
  int d = dir >> 1;
  c[d] += (dir & 1) ? 1 : -1;
  if (c[d] < 0 || c[d] >= n[d]) return -1;
  return g.tile_map[((size_t)c[2] * g.nty + c[1]) * g.ntx + c[0]];
}

// Sum of the 2*DIM face-neighbour values of local point l of `slot`; val(i)
// gives the value at vector index i, nb[] the neighbour slots of the tile
// (NBR_STRIDE entries per slot).  Summation order -x,+x,-y,+y,-z,+z.
template <int DIM, class Val>
__device__ __forceinline__ double neighbour_sum(int slot, int l, gptr<const int> nb, Val&& val) {
  constexpr int X = TileShape<DIM>::X, Y = TileShape<DIM>::Y, Z = TileShape<DIM>::Z;
  const int lx = l % X, ly = (l / X) % Y, lz = l / (X * Y);
  const size_t base = (size_t)slot * TILE_PTS;
  double s = 0.0;
  if (lx > 0) s += val(base + l - 1);
  else if (nb[0] >= 0) s += val((size_t)nb[0] * TILE_PTS + l + (X - 1));
  if (lx < X - 1) s += val(base + l + 1);
  else if (nb[1] >= 0) s += val((size_t)nb[1] * TILE_PTS + l - (X - 1));
  if (ly > 0) s += val(base + l - X);
  else if (nb[2] >= 0) s += val((size_t)nb[2] * TILE_PTS + l + X * (Y - 1));
  if (ly < Y - 1) s += val(base + l + X);
  else if (nb[3] >= 0) s += val((size_t)nb[3] * TILE_PTS + l - X * (Y - 1));
  if (DIM == 3) {
    if (lz > 0) s += val(base + l - X * Y);
    else if (nb[4] >= 0) s += val((size_t)nb[4] * TILE_PTS + l + X * Y * (Z - 1));
    if (lz < Z - 1) s += val(base + l + X * Y);
    else if (nb[5] >= 0) s += val((size_t)nb[5] * TILE_PTS + l - X * Y * (Z - 1));
  }
  return s;
}

// (A v) at local point l of `slot` (0 at non-computational points):
// beta/h^2 * (sum of neighbours - c_p v_p), c_p = 2*DIM for regular points.
template <int DIM>
__device__ __forceinline__ double apply_A(const GeomDev& g, gptr<const double> v, int slot,
                                          int l, gptr<const int> nb, bool comp, bool irr) {
  if (!comp) return 0.0;
  const size_t i = (size_t)slot * TILE_PTS + l;
  const double vp = v[i];
  const double c = irr ? glb(g.cdiag)[i] : (double)(2 * DIM);
  return g.coef * (neighbour_sum<DIM>(slot, l, nb, [&](size_t j) { return v[j]; }) - c * vp);
}

// Bound on the polls of a grid synchronisation before it gives up (and
// raises the abort flag so that every block exits).
constexpr long SPIN_LIMIT = 1L << 24;

// ---------------------------------------------------------------- reductions

// Sum over a wavefront, fixed tree; the result is valid in lane 0.
__device__ __forceinline__ double wave_sum_lane0(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum of NR values over the NW = blockDim.x / 64 waves (fixed order);
// result in v[] for all threads.  `scratch` holds at least NW*NR doubles.
template <int NR>
__device__ __forceinline__ void block_sum(double (&v)[NR], double* scratch) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    double s = wave_sum_lane0(v[k]);
    if (lane == 0) scratch[w * NR + k] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    double t = scratch[k];
    for (int q = 1; q < nw; ++q) t += scratch[q * NR + k];
    v[k] = t;
  }
  __syncthreads();
}

}  // namespace etdfb
