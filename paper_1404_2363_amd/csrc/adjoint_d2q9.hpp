// Discrete adjoint of the D2Q9 pull step, for gradients with respect to D.
//
// Forward step t (pull form): g_t = Pi p_t (gather, with the wall rules) and
// p_{t+1} = C g_t, with the per-node collision C = I - M^-1 S (M - E 1^T),
// E = m_eq(phi = 1, u) = (1, -2, 2, ux, -ux, uy, -uy, 0, 0) (Eq. 37), S the
// modified relaxation matrix (Eq. 31).  For a loss L of the phi snapshots,
// lambda_t = dL/dp_t obeys lambda_t = Pi^T C^T lambda_{t+1} + dL/dp_t|direct,
// and dL/dD = sum_t lambda_{t+1}^T (dC/dD) g_t.
//
// With mu_t = C^T lambda_{t+1}, one reverse kernel (step t) computes at node y
//   lambda = (Pi^T mu_{t+1})(y) + dL/dphi_{t+1}(y)    (every population of y)
//   w = M^-T lambda = diag(1/norm^2) M lambda
//   grad_c(y) += (1/kappa) (A w')^T E_c (A v)          (w' = (w3, w5))
//   z = S^T w,  mu_t(y) = lambda - M^T z + 1 (E^T z)
// where v = (n3 + s4 n4 / 2, n5 + s6 n6 / 2) from the non-equilibrium moments
// n of the forward g_t(y), and E_c the symmetric unit tensor of component c
// (xx, yy, xy).  This uses dC g = -M^-1 dS n, dS depending on A only through
// the flux block (heat-flux rates s4, s6 held fixed), and dA = -A (dD/kappa) A.
// Pi^T gathers each population from its push destination: the neighbour
// y + e_j, or across a wall the population that the wall rule sends there.
//
// mu_t does not depend on the forward state (the step is linear); the forward
// state enters only through v.  The recomputation of a checkpoint segment
// therefore keeps v_t (two values per node and step) instead of the states:
// the reverse step reads 8 (FP32) bytes per node from the forward pass
// rather than gathering nine populations.
#pragma once

#include "common.hpp"
#include "d2q9.hpp"

namespace lbm {

// Index that the transposed streaming reads for population (EX, EY) at node
// (x, y): the destination of that population in a push step.
template <int EX, int EY>
LBM_FORCEINLINE int64_t push_index_d2q9(const RunArgs& a, int64_t x, int64_t y) {
  int64_t dx = x + EX, dy = y + EY;
  bool cx = false, cy = false;
  if (EX != 0) {
    const bool out = dx < 0 || dx >= a.nx;
    if (a.bc[0] == LBM_CDE_PERIODIC) dx = dx < 0 ? dx + a.nx : (dx >= a.nx ? dx - a.nx : dx);
    else cx = out;
  }
  if (EY != 0) {
    const bool out = dy < 0 || dy >= a.ny;
    if (a.bc[1] == LBM_CDE_PERIODIC) dy = dy < 0 ? dy + a.ny : (dy >= a.ny ? dy - a.ny : dy);
    else cy = out;
  }
  const bool bounce = (cx && a.bc[0] == LBM_CDE_BOUNCE_BACK) || (cy && a.bc[1] == LBM_CDE_BOUNCE_BACK);
  int vx = EX, vy = EY;
  if (bounce) {
    vx = -EX;
    vy = -EY;
    dx = x;
    dy = y;
  } else {
    if (cx) { vx = -EX; dx = x; }
    if (cy) { vy = -EY; dy = y; }
  }
  return (int64_t)pop_of_d2q9(vx, vy) * a.plane + dy * a.nx + dx;
}

// Forward pull gather of population (EX, EY) from the state, with walls.
template <typename R, bool WALLS, int EX, int EY>
LBM_FORCEINLINE R gather_fwd(const RunArgs& a, const R* src, int64_t x, int64_t y) {
  if constexpr (WALLS) return src[pull_index_d2q9<EX, EY>(a, x, y)];
  const int64_t sx = EX == 1 ? wrap_m(x, a.nx) : EX == -1 ? wrap_p(x, a.nx) : x;
  const int64_t sy = EY == 1 ? wrap_m(y, a.ny) : EY == -1 ? wrap_p(y, a.ny) : y;
  return src[(int64_t)pop_of_d2q9(EX, EY) * a.plane + sy * a.nx + sx];
}

template <typename R, bool WALLS, int EX, int EY>
LBM_FORCEINLINE R gather_adj(const RunArgs& a, const R* mu, int64_t x, int64_t y) {
  if constexpr (WALLS) return mu[push_index_d2q9<EX, EY>(a, x, y)];
  const int64_t dx = EX == 1 ? wrap_p(x, a.nx) : EX == -1 ? wrap_m(x, a.nx) : x;
  const int64_t dy = EY == 1 ? wrap_p(y, a.ny) : EY == -1 ? wrap_m(y, a.ny) : y;
  return mu[(int64_t)pop_of_d2q9(EX, EY) * a.plane + dy * a.nx + dx];
}

// v = (n3 + s4 n4 / 2, n5 + s6 n6 / 2) of the pre-collision populations f of
// a node (n = M f - m_eq, Eq. 11 and 37; phi_ref = 0 unless shifted storage).
template <typename R>
LBM_FORCEINLINE void adjoint_v(const R (&f)[9], R ux, R uy, R phi_ref, const Rel2<R>& r, R& vx, R& vy) {
  const R phi = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8] + phi_ref;
  const R dx13 = f[1] - f[3], dx58 = f[5] - f[6] - f[7] + f[8];
  const R dy24 = f[2] - f[4], dy56 = f[5] + f[6] - f[7] - f[8];
  const R n3 = dx13 + dx58 - phi * ux, n4 = dx58 - (R)2 * dx13 + phi * ux;
  const R n5 = dy24 + dy56 - phi * uy, n6 = dy56 - (R)2 * dy24 + phi * uy;
  vx = n3 + (R)0.5 * r.s4 * n4;
  vy = n5 + (R)0.5 * r.s6 * n6;
}

// The reverse step at one node: from the gathered adjoint populations l
// (lambda_{t+1} at the node, injection included), the forward step's v, the
// velocity and the relaxation rates, the outgoing mu_t (m) and the gradient
// contributions g_c (xx, yy, xy; before the 1/kappa factor).
template <typename R>
LBM_FORCEINLINE void adjoint_node(const R (&l)[9], R vx, R vy, R ux, R uy, const Rel2<R>& r, R (&m)[9], R (&gc)[3]) {
  // w = M^-T lambda (moments of lambda over the squared row norms)
  const R sa = l[1] + l[2] + l[3] + l[4], sd = l[5] + l[6] + l[7] + l[8];
  const R w1 = ((R)2 * sd - sa - (R)4 * l[0]) * (R)(1.0 / 36.0);
  const R w2 = ((R)4 * l[0] - (R)2 * sa + sd) * (R)(1.0 / 36.0);
  const R lx13 = l[1] - l[3], lx58 = l[5] - l[6] - l[7] + l[8];
  const R ly24 = l[2] - l[4], ly56 = l[5] + l[6] - l[7] - l[8];
  const R w3 = (lx13 + lx58) * (R)(1.0 / 6.0), w4 = (lx58 - (R)2 * lx13) * (R)(1.0 / 12.0);
  const R w5 = (ly24 + ly56) * (R)(1.0 / 6.0), w6 = (ly56 - (R)2 * ly24) * (R)(1.0 / 12.0);
  const R w7 = (l[1] - l[2] + l[3] - l[4]) * (R)0.25, w8 = (l[5] - l[6] + l[7] - l[8]) * (R)0.25;

  // gradient with respect to the D components (xx, yy, xy) of this node
  const R awx = r.axx * w3 + r.axy * w5, awy = r.axy * w3 + r.ayy * w5;
  const R avx = r.axx * vx + r.axy * vy, avy = r.axy * vx + r.ayy * vy;
  gc[0] = awx * avx;
  gc[1] = awy * avy;
  gc[2] = awx * avy + awy * avx;

  // z = S^T w (Eq. 31 transposed)
  const R z1 = r.s1 * w1, z2 = r.s2 * w2;
  const R z3 = r.axx * w3 + r.axy * w5, z5 = r.axy * w3 + r.ayy * w5;
  const R z4 = r.s4 * w4 + r.c34 * w3 + r.c54 * w5;
  const R z6 = r.s6 * w6 + r.c36 * w3 + r.c56 * w5;
  const R z7 = r.s7 * w7, z8 = r.s8 * w8;
  const R ez = (R)2 * (z2 - z1) + ux * (z3 - z4) + uy * (z5 - z6);   // E^T z
  // mu = lambda - M^T z + E^T z (every population)
  const R ax = -z1 - (R)2 * z2, dg = (R)2 * z1 + z2;
  const R q3 = z3 - (R)2 * z4, q5 = z5 - (R)2 * z6, p3 = z3 + z4, p5 = z5 + z6;
  m[0] = l[0] - (R)4 * (z2 - z1) + ez;
  m[1] = l[1] - (ax + q3 + z7) + ez;
  m[2] = l[2] - (ax + q5 - z7) + ez;
  m[3] = l[3] - (ax - q3 + z7) + ez;
  m[4] = l[4] - (ax - q5 - z7) + ez;
  m[5] = l[5] - (dg + p3 + p5 + z8) + ez;
  m[6] = l[6] - (dg - p3 + p5 - z8) + ez;
  m[7] = l[7] - (dg - p3 - p5 + z8) + ez;
  m[8] = l[8] - (dg + p3 - p5 - z8) + ez;
}

// One forward step of the segment recomputation (256-wide row tiles): the
// pull step of k_step_d2q9 from a.src to a.dst (when STORE; the same
// arithmetic, so the states are bitwise those of the run), plus v of every
// node into vout[2][N].
template <typename R, bool WALLS, bool STORE>
__global__ __launch_bounds__(256) void k_step_v_d2q9(const RunArgs a, R* __restrict__ vout, const FastDiv ntx) {
  const int64_t N = a.nx * a.ny;
  const uint32_t yq = fdiv(blockIdx.x, ntx);
  const int64_t x = (int64_t)(blockIdx.x - yq * ntx.d) * 256 + threadIdx.x, y = yq;
  if (x >= a.nx) return;
  const int64_t node = y * a.nx + x;
  const R* src = (const R*)a.src;
  R f[9];
  f[0] = src[node];
  f[1] = gather_fwd<R, WALLS, 1, 0>(a, src, x, y);
  f[2] = gather_fwd<R, WALLS, 0, 1>(a, src, x, y);
  f[3] = gather_fwd<R, WALLS, -1, 0>(a, src, x, y);
  f[4] = gather_fwd<R, WALLS, 0, -1>(a, src, x, y);
  f[5] = gather_fwd<R, WALLS, 1, 1>(a, src, x, y);
  f[6] = gather_fwd<R, WALLS, -1, 1>(a, src, x, y);
  f[7] = gather_fwd<R, WALLS, -1, -1>(a, src, x, y);
  f[8] = gather_fwd<R, WALLS, 1, -1>(a, src, x, y);
  R ux, uy;
  velocity2<R>(a, x, y, ux, uy);
  const R phi_ref = (R)a.phi_ref;
  const Rel2<R> r = a.node_par ? node_rel2<R>(a, node) : const_rel2<R>(a);
  R vx, vy;
  adjoint_v<R>(f, ux, uy, phi_ref, r, vx, vy);
  store_pop<R, true>(vout + node, vx);
  store_pop<R, true>(vout + N + node, vy);
  if constexpr (STORE) {
    collide_d2q9<R>(f, ux, uy, phi_ref, r);
    R* dst = (R*)a.dst;
#pragma unroll
    for (int i = 0; i < 9; ++i) store_pop<R, true>(dst + i * a.plane + node, f[i]);
  }
}

// How a reverse step stores its gradient contribution g_c (c = xx, yy, xy)
// of a node.  FP64 storage always accumulates in the FP64 output; FP32
// storage accumulates the FP32 contributions of a checkpoint segment in an
// FP32 partial and adds it to the FP64 output once, in the segment's last
// reverse step:
//   GRAD_F64       grad += g / kappa                     (read-modify-write, FP64)
//   GRAD_F32_SET   part  = g                             (write, FP32)
//   GRAD_F32_ADD   part += g                             (read-modify-write, FP32)
//   GRAD_F32_FOLD  grad += ((double)part + g) / kappa     (FP32 read, FP64 read-modify-write)
enum GradMode : int32_t { GRAD_F64 = 0, GRAD_F32_SET = 1, GRAD_F32_ADD = 2, GRAD_F32_FOLD = 3 };

// One reverse step over every node: vin = v_t of the forward step t ([2][N],
// from k_step_v_d2q9), mu_in = mu_{t+1}, inj = dL/dphi_{t+1} (read when INJ),
// mu_out = mu_t, grad (FP64, [3][N]) and part (FP32, [3][N]) per GMODE; NT:
// streaming stores.  One block per blockDim.x-wide row tile.  The loads of a
// thread (adjoint populations, v, injection, gradient accumulators) are
// issued together, without branches between them, before its first store.
// Without walls every address is a 32-bit byte offset from a
// kernel-argument base (the host checks that every offset fits).
template <typename R, bool WALLS, int GMODE, bool INJ, bool NT>
__global__ __launch_bounds__(512) void k_adjoint_d2q9(const RunArgs a, const R* __restrict__ vin,
                                                      const R* __restrict__ mu_in, const double* __restrict__ inj,
                                                      R* __restrict__ mu_out, double* __restrict__ grad,
                                                      float* __restrict__ part, double inv_kappa, const FastDiv ntx) {
  const int64_t N = a.nx * a.ny;
  const uint32_t bx = blockDim.x;
  const uint32_t yq = fdiv(blockIdx.x, ntx);
  const int64_t x = (int64_t)(blockIdx.x - yq * ntx.d) * bx + threadIdx.x, y = yq;
  if (x >= a.nx) return;
  const int64_t node = y * a.nx + x;

  R l[9];  // adjoint populations lambda_{t+1}(y)
  R vx, vy;  // v of the forward step at y
  double injv = 0.0;
  double g64[3] = {0.0, 0.0, 0.0};
  float g32[3] = {0.0f, 0.0f, 0.0f};
  uint32_t o_node = 0, pb = 0;  // byte offsets (no walls)
  if constexpr (WALLS) {
    l[0] = mu_in[node];
    l[1] = gather_adj<R, WALLS, 1, 0>(a, mu_in, x, y);
    l[2] = gather_adj<R, WALLS, 0, 1>(a, mu_in, x, y);
    l[3] = gather_adj<R, WALLS, -1, 0>(a, mu_in, x, y);
    l[4] = gather_adj<R, WALLS, 0, -1>(a, mu_in, x, y);
    l[5] = gather_adj<R, WALLS, 1, 1>(a, mu_in, x, y);
    l[6] = gather_adj<R, WALLS, -1, 1>(a, mu_in, x, y);
    l[7] = gather_adj<R, WALLS, -1, -1>(a, mu_in, x, y);
    l[8] = gather_adj<R, WALLS, 1, -1>(a, mu_in, x, y);
    vx = vin[node];
    vy = vin[N + node];
    if constexpr (INJ) injv = inj[node];
    if constexpr (GMODE == GRAD_F64 || GMODE == GRAD_F32_FOLD)
#pragma unroll
      for (int c = 0; c < 3; ++c) g64[c] = grad[c * N + node];
    if constexpr (GMODE == GRAD_F32_ADD || GMODE == GRAD_F32_FOLD)
#pragma unroll
      for (int c = 0; c < 3; ++c) g32[c] = part[c * N + node];
  } else {
    constexpr uint32_t E = sizeof(R);
    const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny, xu = (uint32_t)x, yu = (uint32_t)y;
    const uint32_t xm = xu == 0 ? nx - 1u : xu - 1u, xp = xu + 1u == nx ? 0u : xu + 1u;
    const uint32_t r0 = yu * nx, rm = (yu == 0 ? ny - 1u : yu - 1u) * nx, rp = (yu + 1u == ny ? 0u : yu + 1u) * nx;
    pb = (uint32_t)a.plane * E;
    o_node = (r0 + xu) * E;
    const char* mb = (const char*)mu_in;
    auto ld = [](const char* b, uint32_t o) { return *(const R*)(b + o); };
    // lambda: population (ex, ey) from its push destination (x + ex, y + ey)
    l[0] = ld(mb, o_node);
    l[1] = ld(mb, pb + (r0 + xp) * E);
    l[2] = ld(mb, 2u * pb + (rp + xu) * E);
    l[3] = ld(mb, 3u * pb + (r0 + xm) * E);
    l[4] = ld(mb, 4u * pb + (rm + xu) * E);
    l[5] = ld(mb, 5u * pb + (rp + xp) * E);
    l[6] = ld(mb, 6u * pb + (rp + xm) * E);
    l[7] = ld(mb, 7u * pb + (rm + xm) * E);
    l[8] = ld(mb, 8u * pb + (rm + xp) * E);
    vx = ld((const char*)vin, o_node);
    vy = ld((const char*)vin, (uint32_t)N * E + o_node);
    const uint32_t o8 = (r0 + xu) * 8u, o4 = (r0 + xu) * 4u, n8 = (uint32_t)N * 8u, n4 = (uint32_t)N * 4u;
    if constexpr (INJ) injv = *(const double*)((const char*)inj + o8);
    if constexpr (GMODE == GRAD_F64 || GMODE == GRAD_F32_FOLD)
#pragma unroll
      for (int c = 0; c < 3; ++c) g64[c] = *(const double*)((const char*)grad + c * n8 + o8);
    if constexpr (GMODE == GRAD_F32_ADD || GMODE == GRAD_F32_FOLD)
#pragma unroll
      for (int c = 0; c < 3; ++c) g32[c] = *(const float*)((const char*)part + c * n4 + o4);
  }
  R ux, uy;
  velocity2<R>(a, x, y, ux, uy);
  const Rel2<R> r = a.node_par ? node_rel2<R>(a, node) : const_rel2<R>(a);

  if constexpr (INJ) {
    const R g = (R)injv;
#pragma unroll
    for (int i = 0; i < 9; ++i) l[i] += g;
  }
  R m[9], gc[3];
  adjoint_node<R>(l, vx, vy, ux, uy, r, m, gc);
  double gout[3];
  float pout[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (GMODE == GRAD_F64) gout[c] = g64[c] + inv_kappa * (double)gc[c];
    else if constexpr (GMODE == GRAD_F32_FOLD) gout[c] = g64[c] + inv_kappa * ((double)g32[c] + (double)gc[c]);
    else pout[c] = g32[c] + (float)gc[c];
  }
  if constexpr (WALLS) {
#pragma unroll
    for (int i = 0; i < 9; ++i) store_pop<R, NT>(mu_out + i * a.plane + node, m[i]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (GMODE == GRAD_F64 || GMODE == GRAD_F32_FOLD) store_pop<double, NT>(grad + c * N + node, gout[c]);
      else store_pop<float, NT>(part + c * N + node, pout[c]);
    }
  } else {
    char* ob = (char*)mu_out;
#pragma unroll
    for (int i = 0; i < 9; ++i) store_pop<R, NT>((R*)(ob + (uint32_t)i * pb + o_node), m[i]);
    const uint32_t o8 = o_node / (uint32_t)sizeof(R) * 8u, o4 = o_node / (uint32_t)sizeof(R) * 4u;
    const uint32_t n8 = (uint32_t)N * 8u, n4 = (uint32_t)N * 4u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (GMODE == GRAD_F64 || GMODE == GRAD_F32_FOLD)
        store_pop<double, NT>((double*)((char*)grad + c * n8 + o8), gout[c]);
      else
        store_pop<float, NT>((float*)((char*)part + c * n4 + o4), pout[c]);
    }
  }
}

// dL/dphi0 from lambda_0 = Pi^T mu_0 + dL/dphi_0: the initial state is
// f_eq(phi0, u), linear in phi0 with coefficients f_eq(1, u).
template <typename R, bool WALLS>
__global__ __launch_bounds__(256) void k_adjoint_phi0_d2q9(const RunArgs a, const R* __restrict__ mu0,
                                                           const double* __restrict__ inj0,
                                                           double* __restrict__ dphi0) {
  const int64_t N = a.nx * a.ny;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  const int64_t x = node % a.nx, y = node / a.nx;
  double l[9];
  l[0] = (double)mu0[node];
  l[1] = (double)gather_adj<R, WALLS, 1, 0>(a, mu0, x, y);
  l[2] = (double)gather_adj<R, WALLS, 0, 1>(a, mu0, x, y);
  l[3] = (double)gather_adj<R, WALLS, -1, 0>(a, mu0, x, y);
  l[4] = (double)gather_adj<R, WALLS, 0, -1>(a, mu0, x, y);
  l[5] = (double)gather_adj<R, WALLS, 1, 1>(a, mu0, x, y);
  l[6] = (double)gather_adj<R, WALLS, -1, 1>(a, mu0, x, y);
  l[7] = (double)gather_adj<R, WALLS, -1, -1>(a, mu0, x, y);
  l[8] = (double)gather_adj<R, WALLS, 1, -1>(a, mu0, x, y);
  R ux, uy;
  velocity2<R>(a, x, y, ux, uy);
  double w[9];
  equilibrium_d2q9(w, 1.0, (double)ux, (double)uy, 0.0);
  double s = 0.0;
  for (int i = 0; i < 9; ++i) s += l[i] * w[i];
  if (inj0) s += 1.0 * inj0[node];  // sum_i f_eq_i(1, u) = 1
  dphi0[node] = s;
}

}  // namespace lbm
