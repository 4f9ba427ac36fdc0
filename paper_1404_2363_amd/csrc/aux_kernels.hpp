// Initialisation, readout and FP64 reduction kernels (all lattices).
#pragma once

#include <hip/hip_fp16.h>

#include "common.hpp"
#include "d2q9.hpp"
#include "d3q15.hpp"

namespace lbm {

constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;

// Per-node FP64 velocity for initialisation and readout.
template <typename R>
LBM_FORCEINLINE void velocity_at(const RunArgs& a, int dim, int64_t x, int64_t y, int64_t z, double* u) {
  const int64_t N = a.nx * a.ny * a.nz;
  const int64_t node = (z * a.ny + y) * a.nx + x;
  for (int c = 0; c < dim; ++c) {
    if (a.u_kind == U_CONST) {
      u[c] = a.u_const[c];
    } else if (a.u_kind == U_SEPARABLE) {
      const R* t = (const R*)a.u_tab + c * (1 + a.nx + a.ny + a.nz);
      u[c] = (double)(((t[0] * t[1 + x]) * t[1 + a.nx + y]) * t[1 + a.nx + a.ny + z]);
    } else {
      u[c] = (double)(R)(*a.u_slot)[c * N + node];  // rounded as the step rounds it
    }
  }
}

// Populations of the equilibrium of phi0 (the state at t = 0).
template <typename R>
__global__ __launch_bounds__(256) void k_init_d2q9(const RunArgs a, const double* __restrict__ phi0) {
  const int64_t N = a.nx * a.ny;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  const int64_t x = node % a.nx, y = node / a.nx;
  double u[3];
  velocity_at<R>(a, 2, x, y, 0, u);
  double f[9];
  equilibrium_d2q9(f, phi0[node], u[0], u[1], a.phi_ref, a.model);
  R* dst = (R*)a.dst;
  for (int i = 0; i < 9; ++i) dst[i * a.plane + node] = (R)f[i];
}

template <typename R>
__global__ __launch_bounds__(256) void k_init_d3q15(const RunArgs a, const double* __restrict__ phi0) {
  const int64_t N = a.nx * a.ny * a.nz;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  const int64_t x = node % a.nx, y = (node / a.nx) % a.ny, z = node / (a.nx * a.ny);
  double u[3];
  velocity_at<R>(a, 3, x, y, z, u);
  double f[15];
  equilibrium_d3q15(f, phi0[node], u[0], u[1], u[2], a.phi_ref);
  R* dst = (R*)a.dst;
  for (int i = 0; i < 15; ++i) dst[i * a.plane + node] = (R)f[i];
}

// A stored population value in FP64 (16-bit storage carries a scale).
template <typename S>
LBM_FORCEINLINE double ld_pop(const void* p, int64_t i, double inv) {
  if constexpr (sizeof(S) == 2) return (double)__half2float(((const __half*)p)[i]) * inv;
  else return (double)((const S*)p)[i];
}

// phi of one node and the number of non-finite stored values there.  Split
// storage keeps phi itself; otherwise phi = sum_i f_i (+ phi_ref).
template <typename S>
LBM_FORCEINLINE double node_phi(const RunArgs& a, int Q, int64_t node, int& nonfinite) {
  if (a.src_phi) {
    const double phi = (double)((const float*)a.src_phi)[node];
    nonfinite += !isfinite(phi);
    for (int i = 0; i < Q; ++i) nonfinite += !isfinite(ld_pop<S>(a.src, i * a.plane + node, 1.0));
    return phi;
  }
  double s = 0.0;
  for (int i = 0; i < Q; ++i) {
    const double v = ld_pop<S>(a.src, i * a.plane + node, a.fp16_inv_scale);
    nonfinite += !isfinite(v);
    s += v;
  }
  return s + a.phi_ref;
}

// Quadrature weight of a node in domain sums: nodes on an on-node plate
// (the first and last node of a NODE_MIRROR axis) stand for half a cell, so
// the weighted sum of phi is the quantity the plate rule conserves.
LBM_FORCEINLINE double plate_weight(const RunArgs& a, int64_t node) {
  double w = 1.0;
  if (a.bc[0] == LBM_CDE_NODE_MIRROR) {
    const int64_t x = node % a.nx;
    if (x == 0 || x == a.nx - 1) w *= 0.5;
  }
  if (a.bc[1] == LBM_CDE_NODE_MIRROR) {
    const int64_t y = (node / a.nx) % a.ny;
    if (y == 0 || y == a.ny - 1) w *= 0.5;
  }
  return w;
}

// phi = sum_i f_i (+ phi_ref for shifted storage), FP64.
template <typename S>
__global__ __launch_bounds__(256) void k_moments(const RunArgs a, int Q, double* __restrict__ phi) {
  const int64_t N = a.nx * a.ny * a.nz;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  int bad = 0;
  phi[node] = node_phi<S>(a, Q, node, bad);
}

// Deterministic two-pass FP64 reduction.  Pass 1: each of RED_BLOCKS blocks
// walks a fixed grid-stride set of nodes and tree-reduces 4 sums in LDS.
// Pass 2: one block adds the partials in a fixed tree.
template <typename S>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_partial(const RunArgs a, int Q, int kind, double x_ref,
                                                               double* __restrict__ partial) {
  __shared__ double sh[4][RED_THREADS];
  const int64_t N = a.nx * a.ny * a.nz;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, bad = 0.0;
  const double nxd = (double)a.nx;
  for (int64_t node = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; node < N;
       node += (int64_t)gridDim.x * RED_THREADS) {
    int nonfinite = 0;
    const double phi = node_phi<S>(a, Q, node, nonfinite) * plate_weight(a, node);
    bad += (double)nonfinite;
    if (kind == LBM_CDE_RED_XMOMENTS) {
      double d = (double)(node % a.nx) - x_ref;
      d -= nxd * floor(d / nxd + 0.5);
      s0 += phi;
      s1 += d * phi;
      s2 += d * d * phi;
    } else {
      s0 += phi;
    }
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  sh[2][threadIdx.x] = s2;
  sh[3][threadIdx.x] = bad;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce_final(const double* __restrict__ partial, int nblocks,
                                                             double* __restrict__ out) {
  __shared__ double sh[4][RED_THREADS];
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) s += partial[b * 4 + k];
    sh[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x][0];
}

// Step count of run `a` at global step t (a run stops at its budget).
LBM_FORCEINLINE int64_t run_steps(const RunArgs& a, int64_t t) {
  return (a.max_steps >= 0 && t > a.max_steps) ? a.max_steps : t;
}

// Batched x-moments, pass 1: block (b, r) reduces part of run r (S0, S1, S2
// about x_ref(t_r) = xref0 + xref_drift t_r of that run) into partial[r][b].
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_batch_xmom_partial(const RunArgs* __restrict__ runs, int Q,
                                                                   const int64_t* __restrict__ clock,
                                                                   double* __restrict__ partial) {
  __shared__ double sh[3][RED_THREADS];
  const RunArgs& a = runs[blockIdx.y];
  const int64_t tr = run_steps(a, clock[0]);
  const R* src = (const R*)((tr & 1) ? a.dst : a.src);
  const double nxd = (double)a.nx;
  double x_ref = a.xref0 + a.xref_drift * (double)tr;
  x_ref -= nxd * floor(x_ref / nxd);
  const int64_t N = a.nx * a.ny * a.nz;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t node = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; node < N;
       node += (int64_t)gridDim.x * RED_THREADS) {
    double phi = 0.0;
    for (int i = 0; i < Q; ++i) phi += (double)src[i * a.plane + node];
    phi = (phi + a.phi_ref) * plate_weight(a, node);
    double d = (double)(node % a.nx) - x_ref;
    d -= nxd * floor(d / nxd + 0.5);
    s0 += phi;
    s1 += d * phi;
    s2 += d * d * phi;
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  sh[2][threadIdx.x] = s2;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) partial[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

// Pass 2: block r adds the nb partials of run r into hist[row][r][0..2],
// row = clock[1].
__global__ __launch_bounds__(RED_THREADS) void k_batch_xmom_final(const double* __restrict__ partial, int nb,
                                                                 int nruns, const int64_t* __restrict__ clock,
                                                                 double* __restrict__ hist) {
  __shared__ double sh[3][RED_THREADS];
  const int r = blockIdx.x;
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += RED_THREADS) s += partial[((int64_t)r * nb + b) * 3 + k];
    sh[k][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) hist[(clock[1] * nruns + r) * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

// Advance the device step clock (clock[0]: steps, clock[1]: history rows).
// Batch clock: [0] steps, [1] history rows, [2] population buffer of the
// next launch.  which = 0: one step (flips the buffer); 1: one history row;
// 2: a launch of n steps (flips the buffer).
__global__ void k_tick(int64_t* __restrict__ clock, int which, int n) {
  if (threadIdx.x != 0) return;
  if (which == 1) {
    clock[1] += 1;
  } else {
    clock[0] += which == 0 ? 1 : n;
    clock[2] ^= 1;
  }
}

// Point a velocity slot at a field (a kernel, so that it is ordered on the
// stream and may be captured).
__global__ void k_store_ptr(const double** slot, const double* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *slot = p;
}

// Flag nodes of a velocity field [dim][N] with |u| >= c_s.
__global__ __launch_bounds__(256) void k_check_speed(const double* __restrict__ u, int dim, int64_t N,
                                                     unsigned* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double u2 = 0.0;
  for (int c = 0; c < dim; ++c) u2 += u[c * N + i] * u[c * N + i];
  if (!(u2 < 1.0 / 3.0)) *flag = 1u;
}

// Copy of a device FP64 array into storage precision R.
template <typename R>
__global__ __launch_bounds__(256) void k_convert(const double* __restrict__ in, R* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (R)in[i];
}

// Per-node relaxation parameters of a D field (2D): A = (D/kappa + I/2)^-1 and
// the heat-flux rates by rule.  Counts nodes whose D is not SPD.
template <typename R>
__global__ __launch_bounds__(256) void k_node_params_2d(const double* __restrict__ Dfield, int64_t N, double kappa,
                                                        int rule, double h4, double h6, R* __restrict__ par,
                                                        unsigned long long* __restrict__ nonspd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double dxx = Dfield[i], dyy = Dfield[N + i], dxy = Dfield[2 * N + i];
  if (!(dxx > 0.0) || !(dxx * dyy - dxy * dxy > 0.0)) atomicAdd(nonspd, 1ull);
  // B = D/kappa + I/2, A = B^-1
  const double bxx = dxx / kappa + 0.5, byy = dyy / kappa + 0.5, bxy = dxy / kappa;
  const double det = bxx * byy - bxy * bxy;
  const double axx = byy / det, ayy = bxx / det, axy = -bxy / det;
  double s4 = h4, s6 = h6;
  if (rule == LBM_CDE_HEAT_LAMBDA_MIN) {
    const double m = 0.5 * (axx + ayy), d = 0.5 * (axx - ayy);
    s4 = s6 = m - sqrt(d * d + axy * axy);
  } else if (rule == LBM_CDE_HEAT_PAPER) {
    s4 = axx;
    s6 = ayy;
  }
  par[i] = (R)axx;
  par[N + i] = (R)axy;
  par[2 * N + i] = (R)ayy;
  par[3 * N + i] = (R)s4;
  par[4 * N + i] = (R)s6;
}

}  // namespace lbm
