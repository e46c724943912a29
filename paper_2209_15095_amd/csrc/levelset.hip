// Level-set sweeps that move the free boundary (Section 4.3 of the paper,
// Algorithm Steps 1-2).  Box layout, one thread per node, Jacobi updates
// (every node from the previous iterate, so the result does not depend on
// scheduling), nearest-node values beyond the box edge.
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

#include "levelset.h"

namespace etdfb {

namespace {

constexpr double WENO_EPS = 1e-6;

struct LB {
  int dim, nx, ny, nz;
  double h;
};

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

__device__ __forceinline__ void coords(const LB& b, size_t id, int& i, int& j, int& k) {
  i = (int)(id % b.nx);
  j = (int)((id / b.nx) % b.ny);
  k = (int)(id / ((size_t)b.nx * b.ny));
}

// value of a at (i,j,k) shifted by s along spatial axis d, clamped
__device__ __forceinline__ double at(const LB& b, const double* __restrict__ a, int i, int j, int k, int d,
                                     int s) {
  if (d == 0) i = clampi(i + s, b.nx);
  else if (d == 1) j = clampi(j + s, b.ny);
  else k = clampi(k + s, b.nz);
  return a[((size_t)k * b.ny + j) * b.nx + i];
}

__device__ __forceinline__ uint8_t atm(const LB& b, const uint8_t* __restrict__ a, int i, int j, int k, int d,
                                       int s) {
  if (d == 0) i = clampi(i + s, b.nx);
  else if (d == 1) j = clampi(j + s, b.ny);
  else k = clampi(k + s, b.nz);
  return a[((size_t)k * b.ny + j) * b.nx + i];
}

#define GRID_LOOP(b)                                                                  \
  const size_t total = (size_t)(b).nx * (b).ny * (b).nz;                             \
  for (size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x; id < total;        \
       id += (size_t)gridDim.x * blockDim.x)

__global__ void normals_kernel(LB b, const double* __restrict__ rho, double* __restrict__ nx,
                               double* __restrict__ ny, double* __restrict__ nz) {
  GRID_LOOP(b) {
    int i, j, k;
    coords(b, id, i, j, k);
    double g[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < b.dim; ++d) g[d] = (at(b, rho, i, j, k, d, 1) - at(b, rho, i, j, k, d, -1)) / (2.0 * b.h);
    double mag = 0.0;
    for (int d = 0; d < b.dim; ++d) mag += g[d] * g[d];
    mag = fmax(sqrt(mag), 1e-12);
    nx[id] = g[0] / mag;
    ny[id] = g[1] / mag;
    if (b.dim == 3) nz[id] = g[2] / mag;
  }
}

// bit 0: K0 (computational points of rho), also u0 = K0 ? u : 0
__global__ void known0_kernel(LB b, const double* __restrict__ rho, const double* __restrict__ u,
                              uint8_t* __restrict__ known, double* __restrict__ u0) {
  GRID_LOOP(b) {
    int i, j, k;
    coords(b, id, i, j, k);
    bool c = rho[id] < 0.0;
    if (c) {
      if (i == 0 || i == b.nx - 1 || j == 0 || j == b.ny - 1) c = false;
      if (b.dim == 3 && (k == 0 || k == b.nz - 1)) c = false;
    }
    if (c)
      for (int d = 0; d < b.dim && c; ++d)
        c = at(b, rho, i, j, k, d, -1) < 0.0 && at(b, rho, i, j, k, d, 1) < 0.0;
    known[id] = c ? 1 : 0;
    u0[id] = c ? u[id] : 0.0;
  }
}

// bit `dst` = bit `src` at the node and all 2d (clamped) neighbours
__global__ void known_next_kernel(LB b, uint8_t* __restrict__ known, int src, int dst) {
  GRID_LOOP(b) {
    int i, j, k;
    coords(b, id, i, j, k);
    bool c = (known[id] >> src) & 1;
    for (int d = 0; d < b.dim && c; ++d)
      c = ((atm(b, known, i, j, k, d, -1) >> src) & 1) && ((atm(b, known, i, j, k, d, 1) >> src) & 1);
    if (c) known[id] |= (uint8_t)(1u << dst);
  }
}

// dst = known(bit) ? n . central grad(src) : 0
__global__ void central_dir_kernel(LB b, const double* __restrict__ src, const double* __restrict__ nx,
                                   const double* __restrict__ ny, const double* __restrict__ nz,
                                   const uint8_t* __restrict__ known, int bit, double* __restrict__ dst) {
  GRID_LOOP(b) {
    int i, j, k;
    coords(b, id, i, j, k);
    double v = 0.0;
    if ((known[id] >> bit) & 1) {
      const double* n[3] = {nx, ny, nz};
      for (int d = 0; d < b.dim; ++d)
        v += n[d][id] * ((at(b, src, i, j, k, d, 1) - at(b, src, i, j, k, d, -1)) / (2.0 * b.h));
    }
    dst[id] = v;
  }
}

// one Jacobi sweep of v <- v - dtau (a.grad v - src) off the known set;
// a = sgn * n (sgn = 1, or sign(rho) when sgn_rho != nullptr)
__global__ void extend_kernel(LB b, const double* __restrict__ v, double* __restrict__ out,
                              const double* __restrict__ nx, const double* __restrict__ ny,
                              const double* __restrict__ nz, const double* __restrict__ src,
                              const uint8_t* __restrict__ known, int bit,
                              const double* __restrict__ sgn_rho) {
  GRID_LOOP(b) {
    int i, j, k;
    coords(b, id, i, j, k);
    const double vc = v[id];
    if ((known[id] >> bit) & 1) {
      out[id] = vc;
      continue;
    }
    double sg = 1.0;
    if (sgn_rho) {
      const double r = sgn_rho[id];
      sg = (r > 0.0) ? 1.0 : ((r < 0.0) ? -1.0 : 0.0);
    }
    const double* n[3] = {nx, ny, nz};
    double up = 0.0;
    for (int d = 0; d < b.dim; ++d) {
      const double a = sg * n[d][id];
      up += fmax(a, 0.0) * (vc - at(b, v, i, j, k, d, -1)) + fmin(a, 0.0) * (at(b, v, i, j, k, d, 1) - vc);
    }
    up = up / b.h;
    const double s = src ? src[id] : 0.0;
    out[id] = vc - (0.5 * b.h) * (up - s);
  }
}

// V = band ? mu |central grad u| : 0; band (|rho| < h) into bit 3; vmax reduction
__global__ void velocity_kernel(LB b, const double* __restrict__ u, const double* __restrict__ rho, double mu,
                                uint8_t* __restrict__ known, double* __restrict__ V) {
  GRID_LOOP(b) {
    int i, j, k;
    coords(b, id, i, j, k);
    const bool band = fabs(rho[id]) < b.h;
    double v = 0.0;
    if (band) {
      double s = 0.0;
      for (int d = 0; d < b.dim; ++d) {
        const double g = (at(b, u, i, j, k, d, 1) - at(b, u, i, j, k, d, -1)) / (2.0 * b.h);
        s += g * g;
      }
      v = mu * sqrt(s);
      known[id] |= 8;
    } else {
      known[id] &= (uint8_t)~8u;
    }
    V[id] = v;
  }
}

__global__ void max_kernel(LB b, const double* __restrict__ V, double* __restrict__ out) {
  __shared__ double sm[256];
  double m = 0.0;
  GRID_LOOP(b) { m = fmax(m, V[id]); }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // max of non-negative doubles: integer order equals value order
    atomicMax((unsigned long long*)out, (unsigned long long)__double_as_longlong(sm[0]));
  }
}

__global__ void zero_kernel(double* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0.0;
}

__device__ __forceinline__ double weno5(double v1, double v2, double v3, double v4, double v5) {
  const double p1 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0;
  const double p2 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0;
  const double p3 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0;
  const double t1 = v1 - 2.0 * v2 + v3, t1b = v1 - 4.0 * v2 + 3.0 * v3;
  const double t2 = v2 - 2.0 * v3 + v4, t2b = v2 - v4;
  const double t3 = v3 - 2.0 * v4 + v5, t3b = 3.0 * v3 - 4.0 * v4 + v5;
  const double s1 = 13.0 / 12.0 * (t1 * t1) + 0.25 * (t1b * t1b);
  const double s2 = 13.0 / 12.0 * (t2 * t2) + 0.25 * (t2b * t2b);
  const double s3 = 13.0 / 12.0 * (t3 * t3) + 0.25 * (t3b * t3b);
  const double e1 = s1 + WENO_EPS, e2 = s2 + WENO_EPS, e3 = s3 + WENO_EPS;
  const double a1 = 0.1 / (e1 * e1);
  const double a2 = 0.6 / (e2 * e2);
  const double a3 = 0.3 / (e3 * e3);
  return (a1 * p1 + a2 * p2 + a3 * p3) / (a1 + a2 + a3);
}

// Godunov |grad phi| for speed sign sg (+1 / -1 / 0), HJ-WENO5 derivatives
__device__ double godunov(const LB& b, const double* __restrict__ phi, int i, int j, int k, double sg) {
  double accp = 0.0, accn = 0.0;
  for (int d = 0; d < b.dim; ++d) {
    double f[7];
    for (int s = -3; s <= 3; ++s) f[s + 3] = at(b, phi, i, j, k, d, s);
    double dd[6];
    for (int q = 0; q < 6; ++q) dd[q] = (f[q + 1] - f[q]) / b.h;
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

// TVD-RK3 stage: out = c0 * base + c1 * (in - dt * L(in)), with
// L = V G(in) (advection, S == nullptr) or S (G_sign(S)(in) - 1) (reinit)
__global__ void rk_stage_kernel(LB b, const double* __restrict__ base, const double* __restrict__ in,
                                double* __restrict__ out, const double* __restrict__ V,
                                const double* __restrict__ S, double dt, double c0, double c1) {
  GRID_LOOP(b) {
    int i, j, k;
    coords(b, id, i, j, k);
    double L;
    if (S) {
      const double s = S[id];
      const double sg = (s > 0.0) ? 1.0 : ((s < 0.0) ? -1.0 : 0.0);
      L = s * (godunov(b, in, i, j, k, sg) - 1.0);
    } else {
      L = V[id] * godunov(b, in, i, j, k, 1.0);
    }
    const double stage = in[id] - dt * L;
    out[id] = (c0 == 0.0) ? stage : c0 * base[id] + c1 * stage;
  }
}

__global__ void sign_kernel(LB b, const double* __restrict__ rho, double* __restrict__ S) {
  GRID_LOOP(b) {
    const double r = rho[id];
    S[id] = r / sqrt(r * r + b.h * b.h);
  }
}

__global__ void copy_kernel(LB b, const double* __restrict__ src, double* __restrict__ dst) {
  GRID_LOOP(b) { dst[id] = src[id]; }
}

// u = comp(rho_new) ? u_ext : 0
__global__ void restrict_kernel(LB b, const double* __restrict__ rho, const double* __restrict__ uext,
                                double* __restrict__ u) {
  GRID_LOOP(b) {
    int i, j, k;
    coords(b, id, i, j, k);
    bool c = rho[id] < 0.0;
    if (c) {
      if (i == 0 || i == b.nx - 1 || j == 0 || j == b.ny - 1) c = false;
      if (b.dim == 3 && (k == 0 || k == b.nz - 1)) c = false;
    }
    if (c)
      for (int d = 0; d < b.dim && c; ++d)
        c = at(b, rho, i, j, k, d, -1) < 0.0 && at(b, rho, i, j, k, d, 1) < 0.0;
    u[id] = c ? uext[id] : 0.0;
  }
}

int grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

hipError_t levelset_alloc(LevelsetScratch& s, size_t nodes) {
  s.nodes = nodes;
  hipError_t e = hipMalloc(&s.buf, sizeof(double) * nodes * 12);
  if (e != hipSuccess) return e;
  e = hipMalloc(&s.known, nodes);
  if (e != hipSuccess) return e;
  e = hipMalloc(&s.vmax, sizeof(double));
  if (e != hipSuccess) return e;
  return hipHostMalloc(&s.h_vmax, sizeof(double));
}

void levelset_free(LevelsetScratch& s) {
  if (s.buf) (void)hipFree(s.buf);
  if (s.known) (void)hipFree(s.known);
  if (s.vmax) (void)hipFree(s.vmax);
  if (s.h_vmax) (void)hipHostFree(s.h_vmax);
  s = LevelsetScratch{};
}

// Box arrays of the level-set scratch.
struct LsBufs {
  double *nx, *ny, *nz, *u0, *un, *unn, *tmp, *V, *r1, *r2, *Sg, *r0;
  explicit LsBufs(const LevelsetScratch& s) {
    double* p[12];
    for (int i = 0; i < 12; ++i) p[i] = s.buf + (size_t)i * s.nodes;
    nx = p[0]; ny = p[1]; nz = p[2];
    u0 = p[3];   // u (extended)
    un = p[4]; unn = p[5]; tmp = p[6]; V = p[7];
    r1 = p[8]; r2 = p[9]; Sg = p[10]; r0 = p[11];
  }
};

#define L(kernel, ...)                                            \
  do {                                                            \
    hipLaunchKernelGGL(kernel, dim3(G), B, 0, st, __VA_ARGS__);   \
    hipError_t _e = hipGetLastError();                            \
    if (_e != hipSuccess) return _e;                              \
  } while (0)

// Steps 1 up to the maximum speed: normals, known sets, Aslam extrapolation,
// Stefan speed and its extension; max V is copied (asynchronously) to the
// pinned host word s.h_vmax.
hipError_t levelset_begin(const LevelsetArgs& a, LevelsetScratch& s, double* rho, double* u,
                          hipStream_t st) {
  LB b{a.box.dim, a.box.nx, a.box.ny, a.box.nz, a.box.dx};
  const LsBufs q(s);
  const int G = grid_for(s.nodes);
  const dim3 B(256);
  // normals and known sets of the current domain
  L(normals_kernel, b, rho, q.nx, q.ny, q.nz);
  L(known0_kernel, b, rho, u, s.known, q.u0);
  L(known_next_kernel, b, s.known, 0, 1);
  L(known_next_kernel, b, s.known, 1, 2);
  L(central_dir_kernel, b, q.u0, q.nx, q.ny, q.nz, s.known, 1, q.un);
  L(central_dir_kernel, b, q.un, q.nx, q.ny, q.nz, s.known, 2, q.unn);
  // Aslam: u_nn, u_n, u (ping-pong through tmp)
  auto extend = [&](double* v, const double* src, int bit, int iters) -> hipError_t {
    double* x = v;
    double* y = q.tmp;
    for (int it = 0; it < iters; ++it) {
      hipLaunchKernelGGL(extend_kernel, dim3(G), B, 0, st, b, x, y, q.nx, q.ny, q.nz, src, s.known, bit,
                         (const double*)nullptr);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      double* t = x; x = y; y = t;
    }
    if (x != v) {
      hipLaunchKernelGGL(copy_kernel, dim3(G), B, 0, st, b, x, v);
      return hipGetLastError();
    }
    return hipSuccess;
  };
  hipError_t e;
  if ((e = extend(q.unn, nullptr, 2, ASLAM_ITERS)) != hipSuccess) return e;
  if ((e = extend(q.un, q.unn, 1, ASLAM_ITERS)) != hipSuccess) return e;
  if ((e = extend(q.u0, q.un, 0, ASLAM_ITERS)) != hipSuccess) return e;
  // Stefan speed on the band, then constant extension along sign(rho) n
  L(velocity_kernel, b, q.u0, rho, a.mu, s.known, q.V);
  {
    double* x = q.V;
    double* y = q.tmp;
    for (int it = 0; it < VEL_ITERS; ++it) {
      L(extend_kernel, b, x, y, q.nx, q.ny, q.nz, (const double*)nullptr, s.known, 3, (const double*)rho);
      double* t = x; x = y; y = t;
    }
    if (x != q.V) L(copy_kernel, b, x, q.V);
  }
  // number of advection substeps from max V (one readback)
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, st, s.vmax);
  L(max_kernel, b, q.V, s.vmax);
  if ((e = hipMemcpyAsync(s.h_vmax, s.vmax, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  return hipSuccess;
}

// The rest of the step (the caller has synchronised the stream, so s.h_vmax
// holds max V): advection substeps, reinitialisation, restriction of u.
hipError_t levelset_end(const LevelsetArgs& a, LevelsetScratch& s, double* rho, double* u,
                        hipStream_t st) {
  LB b{a.box.dim, a.box.nx, a.box.ny, a.box.nz, a.box.dx};
  const LsBufs q(s);
  const int G = grid_for(s.nodes);
  const dim3 B(256);
  const double vmax = *s.h_vmax;
  int nsub = (int)ceil(vmax * a.dt / (0.5 * b.h));
  if (nsub < 1) nsub = 1;
  const double ds = a.dt / nsub;
  // TVD-RK3 advection; rho (user array) is the running state
  for (int it = 0; it < nsub; ++it) {
    L(copy_kernel, b, rho, q.r0);
    L(rk_stage_kernel, b, q.r0, q.r0, q.r1, q.V, (const double*)nullptr, ds, 0.0, 1.0);
    L(rk_stage_kernel, b, q.r0, q.r1, q.r2, q.V, (const double*)nullptr, ds, 0.75, 0.25);
    L(rk_stage_kernel, b, q.r0, q.r2, rho, q.V, (const double*)nullptr, ds, 1.0 / 3.0, 2.0 / 3.0);
  }
  if (a.reinit) {
    L(sign_kernel, b, rho, q.Sg);
    const double dtau = 0.5 * b.h;
    for (int it = 0; it < REINIT_ITERS; ++it) {
      L(copy_kernel, b, rho, q.r0);
      L(rk_stage_kernel, b, q.r0, q.r0, q.r1, (const double*)nullptr, q.Sg, dtau, 0.0, 1.0);
      L(rk_stage_kernel, b, q.r0, q.r1, q.r2, (const double*)nullptr, q.Sg, dtau, 0.75, 0.25);
      L(rk_stage_kernel, b, q.r0, q.r2, rho, (const double*)nullptr, q.Sg, dtau, 1.0 / 3.0, 2.0 / 3.0);
    }
  }
  L(restrict_kernel, b, rho, q.u0, u);
  return hipSuccess;
}
#undef L

hipError_t levelset_run(const LevelsetArgs& a, LevelsetScratch& s, double* rho, double* u,
                        hipStream_t st) {
  hipError_t e = levelset_begin(a, s, rho, u, st);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  return levelset_end(a, s, rho, u, st);
}

}  // namespace etdfb
