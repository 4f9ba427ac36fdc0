// D2Q9 modified-MRT collide-and-stream for gfx950.
//
// Velocities (Eq. 2): 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
//                     5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).
// Moments (Eq. 12): m0 = rho, m1 = e, m2 = eps, m3 = j_x, m4 = q_x, m5 = j_y,
// m6 = q_y, m7 = p_xx, m8 = p_xy.  The rows of M are orthogonal with squared
// norms (9, 36, 36, 6, 12, 6, 12, 4, 4), so M^-1 = M^T diag(1/norm^2) and the
// back-transform is the same integer add/sub tree as the forward one.
//
// Per node the step is linear in f: with n = m - m_eq (Eq. 37:
// m_eq = phi (1, -2, 2, ux, -ux, uy, -uy, 0, 0)), the modified S of Eq. (31)
// gives the increments
//   d_k = s_k n_k                                    (k = 1, 2, 4, 6, 7, 8)
//   d_3 = s_xx n3 + (s_xx/2 - 1) s4 n4 + s_xy n5 + (s_xy/2) s6 n6
//   d_5 = s_yx n3 + (s_yx/2) s4 n4 + s_yy n5 + (s_yy/2 - 1) s6 n6
// (d_0 = 0 because m0 = m0_eq), and f' = f - M^-1 d.
//
// Shifted storage keeps g = f - w phi_ref with w = f_eq(1, 0) = (5/9, 1/18 x 8).
// Because M w = (1, -2, 2, 0, ...) equals m_eq(1, 0), the background cancels in
// n except in the velocity moments: n1 = m1(g) + 2 phi_g, n2 = m2(g) - 2 phi_g,
// n3 = m3(g) - phi ux, ... with phi = phi_g + phi_ref; and g' = g - M^-1 d.
// Streaming and every wall rule map populations to populations of equal
// weight, so the uniform shift is preserved.
//
// The unmodified models MRT-B1/B2/B3 (Sec. 3) use the same kernel: S of
// Eq. (24) has no coupling of j to q (the c coefficients vanish), and the
// equilibria of Eq. (38)/(39) add 3 phi u^2 to n1 and n2 and phi (ux^2 - uy^2),
// phi ux uy to m7_eq, m8_eq.  For MRT-B1, m2_eq(phi, 0) = phi, and the shift
// uses its own w = (4/9, 1/9 x 4, 1/36 x 4) so that n2 = m2(g) - phi_g again.
#pragma once

#include "common.hpp"

namespace lbm {

template <typename R>
LBM_HD Rel2<R> make_rel2_vals(R axx, R axy, R ayy, R s4, R s6, double s1, double s2, double s7, double s8,
                              int model) {
  Rel2<R> r;
  r.s1 = (R)s1;
  r.s2 = (R)s2;
  r.s7 = (R)s7;
  r.s8 = (R)s8;
  r.s4 = s4;
  r.s6 = s6;
  r.axx = axx;
  r.axy = axy;
  r.ayy = ayy;
  const bool modified = model == LBM_CDE_MRT_A;
  r.c34 = modified ? (axx * (R)0.5 - (R)1) * s4 : (R)0;
  r.c36 = modified ? (axy * (R)0.5) * s6 : (R)0;
  r.c54 = modified ? (axy * (R)0.5) * s4 : (R)0;
  r.c56 = modified ? (ayy * (R)0.5 - (R)1) * s6 : (R)0;
  r.nl = (model == LBM_CDE_MRT_B1 || model == LBM_CDE_MRT_B2) ? (R)1 : (R)0;
  r.c2 = model == LBM_CDE_MRT_B1 ? (R)1 : (R)2;
  r.lin = model == LBM_CDE_MRT_A || model == LBM_CDE_MRT_B3;
  const R i36 = (R)(1.0 / 36.0), i12 = (R)(1.0 / 12.0), i6 = (R)(1.0 / 6.0), i4 = (R)0.25;
  r.k1 = r.s1 * i36;
  r.k2 = r.s2 * i36;
  r.k4 = r.s4 * i12;
  r.k6 = r.s6 * i12;
  r.k7 = r.s7 * i4;
  r.k8 = r.s8 * i4;
  r.g33 = r.axx * i6;
  r.g34 = r.c34 * i6;
  r.g35 = r.axy * i6;
  r.g36 = r.c36 * i6;
  r.g53 = r.axy * i6;
  r.g54 = r.c54 * i6;
  r.g55 = r.ayy * i6;
  r.g56 = r.c56 * i6;
  return r;
}

template <typename R>
LBM_FORCEINLINE Rel2<R> make_rel2(R axx, R axy, R ayy, R s4, R s6, const RunArgs& a) {
  return make_rel2_vals<R>(axx, axy, ayy, s4, s6, a.s[1], a.s[2], a.s[7], a.s[8], a.model);
}

// The coefficients of a run's constant rates (host: filling RunArgs::relf
// and reld; device: runs described by a compact batch record).
template <typename R>
LBM_HD Rel2<R> rel2_of_rates(const RunArgs& a) {
  return make_rel2_vals<R>((R)a.A[0][0], (R)a.A[0][1], (R)a.A[1][1], (R)a.heat[0], (R)a.heat[1], a.s[1], a.s[2],
                           a.s[7], a.s[8], a.model);
}

// The coefficients of the run's constant rates, as the host rounded them.
template <typename R>
LBM_FORCEINLINE Rel2<R> const_rel2(const RunArgs& a) {
  if constexpr (sizeof(R) == sizeof(float)) return a.relf;
  else return a.reld;
}

// Per-node relaxation parameters (D field): axx, axy, ayy, s4, s6 planes; the
// last two are not read when the heat-flux rates are the same at every node.
template <typename R>
LBM_FORCEINLINE Rel2<R> node_rel2(const RunArgs& a, int64_t node) {
  const R* p = (const R*)a.node_par;
  const int64_t N = a.nx * a.ny;
  if (a.node_heat_const) return make_rel2<R>(p[node], p[N + node], p[2 * N + node], (R)a.heat[0], (R)a.heat[1], a);
  return make_rel2<R>(p[node], p[N + node], p[2 * N + node], p[3 * N + node], p[4 * N + node], a);
}

// The collision of one node, in place.  phi_ref = 0 for unshifted storage.
// LIN = 1: the equilibrium is linear (r.lin: MRT-A, MRT-B3), LIN = 0: any
// model through the general formulas, LIN = -1: chosen by r.lin at run time.
// For a linear equilibrium both forms give the same increments; the linear
// one skips the u^2 terms, whose coefficients are zero there.
template <typename R, int LIN = -1>
LBM_FORCEINLINE void collide_d2q9(R (&f)[9], R ux, R uy, R phi_ref, const Rel2<R>& r) {
  if constexpr (LIN < 0) {
    if (r.lin) collide_d2q9<R, 1>(f, ux, uy, phi_ref, r);
    else collide_d2q9<R, 0>(f, ux, uy, phi_ref, r);
    return;
  } else {
    const R sa = f[1] + f[2] + f[3] + f[4];
    const R sd = f[5] + f[6] + f[7] + f[8];
    const R phig = f[0] + sa + sd;
    const R phi = phig + phi_ref;
    // moments of the stored populations
    const R m1 = (R)2 * sd - sa - (R)4 * f[0];
    const R m2 = (R)4 * f[0] - (R)2 * sa + sd;
    const R dx13 = f[1] - f[3];
    const R dx58 = f[5] - f[6] - f[7] + f[8];  // diagonal x-flux
    const R dy24 = f[2] - f[4];
    const R dy56 = f[5] + f[6] - f[7] - f[8];  // diagonal y-flux
    const R m3 = dx13 + dx58;
    const R m4 = dx58 - (R)2 * dx13;
    const R m5 = dy24 + dy56;
    const R m6 = dy56 - (R)2 * dy24;
    const R m7 = f[1] - f[2] + f[3] - f[4];
    const R m8 = f[5] - f[6] + f[7] - f[8];
    // non-equilibrium parts (the u^2 terms only for the MRT-B1/B2 equilibria)
    const R jx = phi * ux, jy = phi * uy;
    R n1, n2, n7, n8;
    if constexpr (LIN == 1) {
      n1 = m1 + (R)2 * phig;
      n2 = m2 - (R)2 * phig;
      n7 = m7;
      n8 = m8;
    } else {
      const R q = r.nl * phi;
      const R u2 = ux * ux + uy * uy;
      n1 = m1 + (R)2 * phig - (R)3 * q * u2;
      n2 = m2 - r.c2 * phig + (R)3 * q * u2;
      n7 = m7 - q * (ux * ux - uy * uy);
      n8 = m8 - q * ux * uy;
    }
    const R n3 = m3 - jx;
    const R n4 = m4 + jx;
    const R n5 = m5 - jy;
    const R n6 = m6 + jy;
    // relaxation increments S n, divided by the squared row norms
    const R a1 = r.k1 * n1;
    const R a2 = r.k2 * n2;
    const R a3 = r.g33 * n3 + r.g34 * n4 + r.g35 * n5 + r.g36 * n6;
    const R a4 = r.k4 * n4;
    const R a5 = r.g53 * n3 + r.g54 * n4 + r.g55 * n5 + r.g56 * n6;
    const R a6 = r.k6 * n6;
    const R a7 = r.k7 * n7;
    const R a8 = r.k8 * n8;
    // f' = f - M^T a
    const R ax = -a1 - (R)2 * a2;          // common to the axis populations
    const R dg = (R)2 * a1 + a2;           // common to the diagonals
    const R q3 = a3 - (R)2 * a4, q5 = a5 - (R)2 * a6;
    const R p3 = a3 + a4, p5 = a5 + a6;
    f[0] -= (R)4 * (a2 - a1);
    f[1] -= ax + q3 + a7;
    f[2] -= ax + q5 - a7;
    f[3] -= ax - q3 + a7;
    f[4] -= ax - q5 - a7;
    f[5] -= dg + p3 + p5 + a8;
    f[6] -= dg - p3 + p5 - a8;
    f[7] -= dg - p3 - p5 + a8;
    f[8] -= dg + p3 - p5 - a8;
  }
}

// f_eq(phi, u) of the model, in double: m_eq is Eq. (37) for MRT-A and
// MRT-B3, Eq. (38) for MRT-B1 and Eq. (39) for MRT-B2.
LBM_FORCEINLINE void feq_model_d2q9(double (&f)[9], double phi, double ux, double uy, int model) {
  const bool nl = model == LBM_CDE_MRT_B1 || model == LBM_CDE_MRT_B2;
  const double u2 = ux * ux + uy * uy;
  const double e1 = nl ? phi * (-2.0 + 3.0 * u2) : -2.0 * phi;
  const double e2 = (model == LBM_CDE_MRT_B1 ? phi : 2.0 * phi) - (nl ? 3.0 * phi * u2 : 0.0);
  const double e7 = nl ? phi * (ux * ux - uy * uy) : 0.0;
  const double e8 = nl ? phi * ux * uy : 0.0;
  // M^-1 m_eq = M^T diag(1/norm^2) m_eq
  const double a0 = phi / 9.0, a1 = e1 / 36.0, a2 = e2 / 36.0;
  const double a3 = phi * ux / 6.0, a4 = -phi * ux / 12.0;
  const double a5 = phi * uy / 6.0, a6 = -phi * uy / 12.0;
  const double a7 = e7 / 4.0, a8 = e8 / 4.0;
  const double ax = a0 - a1 - 2.0 * a2, dg = a0 + 2.0 * a1 + a2;
  const double q3 = a3 - 2.0 * a4, q5 = a5 - 2.0 * a6, p3 = a3 + a4, p5 = a5 + a6;
  f[0] = a0 - 4.0 * a1 + 4.0 * a2;
  f[1] = ax + q3 + a7;
  f[2] = ax + q5 - a7;
  f[3] = ax - q3 + a7;
  f[4] = ax - q5 - a7;
  f[5] = dg + p3 + p5 + a8;
  f[6] = dg - p3 + p5 - a8;
  f[7] = dg - p3 - p5 + a8;
  f[8] = dg + p3 - p5 - a8;
}

// Stored initial populations f_eq(phi, u) - w phi_ref with w = f_eq(1, 0) of
// the model (5/9, 1/18 x 8 for MRT-A/B2/B3; 4/9, 1/9 x 4, 1/36 x 4 for B1).
LBM_FORCEINLINE void equilibrium_d2q9(double (&f)[9], double phi, double ux, double uy, double phi_ref,
                                      int model = LBM_CDE_MRT_A) {
  double w[9];
  feq_model_d2q9(f, phi, ux, uy, model);
  feq_model_d2q9(w, 1.0, 0.0, 0.0, model);
  for (int i = 0; i < 9; ++i) f[i] -= w[i] * phi_ref;
}

// Velocity at node (x, y).
template <typename R>
LBM_FORCEINLINE void velocity2(const RunArgs& a, int64_t x, int64_t y, R& ux, R& uy) {
  if (a.u_kind == U_CONST) {
    ux = (R)a.u_const[0];
    uy = (R)a.u_const[1];
  } else if (a.u_kind == U_SEPARABLE) {
    const R* t = (const R*)a.u_tab;
    const int64_t stride = 1 + a.nx + a.ny + a.nz;
    const R* t1 = t + stride;
    ux = ((t[0] * t[1 + x]) * t[1 + a.nx + y]) * t[1 + a.nx + a.ny];
    uy = ((t1[0] * t1[1 + x]) * t1[1 + a.nx + y]) * t1[1 + a.nx + a.ny];
  } else {
    const double* u = *a.u_slot;
    const int64_t N = a.nx * a.ny;
    const double vx = u[y * a.nx + x], vy = u[N + y * a.nx + x];
    check_speed(a, vx * vx + vy * vy);
    ux = (R)vx;
    uy = (R)vy;
  }
}

// Population index of velocity (vx, vy).
LBM_FORCEINLINE int pop_of_d2q9(int vx, int vy) {
  // rows vx = -1, 0, 1; columns vy = -1, 0, 1
  const int t = (vx + 1) * 3 + (vy + 1);
  // (-1,-1)=7 (-1,0)=3 (-1,1)=6 (0,-1)=4 (0,0)=0 (0,1)=2 (1,-1)=8 (1,0)=1 (1,1)=5
  return (int)((0x518204637ull >> (4 * t)) & 0xF);
}

// Index (population plane * plane + node) that the pull of population (EX, EY)
// reads at node (x, y), honouring each axis' boundary kind.  Periodic axes
// wrap; if the source lies beyond a wall, bounce-back takes the opposite
// population of the same node, the halfway mirror takes the population with
// the normal component reversed from the neighbour along the wall, and the
// on-node mirror (Sec. 3.2: f2 = f4, f5 = f8, f6 = f7 at a bottom wall node)
// takes that reversed population as it arrives at the wall node, i.e. from
// the node's inner neighbour.
template <int EX, int EY>
LBM_FORCEINLINE int64_t pull_index_d2q9(const RunArgs& a, int64_t x, int64_t y) {
  int64_t sx = x - EX, sy = y - EY;
  bool cx = false, cy = false;
  if (EX != 0) {
    const bool out = sx < 0 || sx >= a.nx;
    if (a.bc[0] == LBM_CDE_PERIODIC) sx = sx < 0 ? sx + a.nx : (sx >= a.nx ? sx - a.nx : sx);
    else cx = out;
  }
  if (EY != 0) {
    const bool out = sy < 0 || sy >= a.ny;
    if (a.bc[1] == LBM_CDE_PERIODIC) sy = sy < 0 ? sy + a.ny : (sy >= a.ny ? sy - a.ny : sy);
    else cy = out;
  }
  const bool bounce = (cx && a.bc[0] == LBM_CDE_BOUNCE_BACK) || (cy && a.bc[1] == LBM_CDE_BOUNCE_BACK);
  int vx = EX, vy = EY;
  if (bounce) {
    vx = -EX;
    vy = -EY;
    sx = x;
    sy = y;
  } else {
    // mirror: at a halfway wall the source is the node itself, at an on-node
    // wall (the wall passes through the first node) the node's inner neighbour
    if (cx) { vx = -EX; sx = a.bc[0] == LBM_CDE_NODE_MIRROR ? x + EX : x; }
    if (cy) { vy = -EY; sy = a.bc[1] == LBM_CDE_NODE_MIRROR ? y + EY : y; }
  }
  return (int64_t)pop_of_d2q9(vx, vy) * a.plane + sy * a.nx + sx;
}

// One pull step over a tile of BX x (BY*NY) nodes.  Thread (tx, ty) owns
// column x and rows ty, ty + BY, ... of the tile.  All loads of a thread are
// issued before its collisions.
template <typename R, int BX, int BY, int NY, bool WALLS, bool NT>
LBM_FORCEINLINE void tile_d2q9(const RunArgs& a, int64_t tile_x, int64_t tile_y) {
  const int64_t x = tile_x * BX + threadIdx.x;
  if (x >= a.nx) return;
  const R* __restrict__ src = (const R*)a.src;
  R* __restrict__ dst = (R*)a.dst;
  const int64_t P = a.plane;
  const int64_t y0 = tile_y * (BY * NY) + threadIdx.y;

  R f[NY][9];
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    const int64_t y = y0 + (int64_t)k * BY;
    if (y >= a.ny) continue;
    if constexpr (!WALLS) {
      const int64_t xm = wrap_m(x, a.nx), xp = wrap_p(x, a.nx);
      const int64_t r0 = y * a.nx, rm = wrap_m(y, a.ny) * a.nx, rp = wrap_p(y, a.ny) * a.nx;
      f[k][0] = src[r0 + x];
      f[k][1] = src[1 * P + r0 + xm];
      f[k][2] = src[2 * P + rm + x];
      f[k][3] = src[3 * P + r0 + xp];
      f[k][4] = src[4 * P + rp + x];
      f[k][5] = src[5 * P + rm + xm];
      f[k][6] = src[6 * P + rm + xp];
      f[k][7] = src[7 * P + rp + xp];
      f[k][8] = src[8 * P + rp + xm];
    } else {
      f[k][0] = src[y * a.nx + x];
      f[k][1] = src[pull_index_d2q9<1, 0>(a, x, y)];
      f[k][2] = src[pull_index_d2q9<0, 1>(a, x, y)];
      f[k][3] = src[pull_index_d2q9<-1, 0>(a, x, y)];
      f[k][4] = src[pull_index_d2q9<0, -1>(a, x, y)];
      f[k][5] = src[pull_index_d2q9<1, 1>(a, x, y)];
      f[k][6] = src[pull_index_d2q9<-1, 1>(a, x, y)];
      f[k][7] = src[pull_index_d2q9<-1, -1>(a, x, y)];
      f[k][8] = src[pull_index_d2q9<1, -1>(a, x, y)];
    }
  }
  const R phi_ref = (R)a.phi_ref;
  const Rel2<R> rc = const_rel2<R>(a);
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    const int64_t y = y0 + (int64_t)k * BY;
    if (y >= a.ny) continue;
    const int64_t node = y * a.nx + x;
    R ux, uy;
    velocity2<R>(a, x, y, ux, uy);
    if (a.node_par) collide_d2q9<R>(f[k], ux, uy, phi_ref, node_rel2<R>(a, node));
    else collide_d2q9<R>(f[k], ux, uy, phi_ref, rc);
#pragma unroll
    for (int i = 0; i < 9; ++i) store_pop<R, NT>(dst + i * P + node, f[k][i]);
  }
}

// One step of one run: one block per tile, in the chosen block order.
template <typename R, int BX, int BY, int NY, bool WALLS, bool NT>
__global__ __launch_bounds__(BX * BY) void k_step_d2q9(const RunArgs a) {
  const uint32_t b = tile_of_block32(blockIdx.x, gridDim.x, a.tiles_x, a.xcd_remap);
  const uint32_t ty = fdiv(b, a.tiles_x);
  tile_d2q9<R, BX, BY, NY, WALLS, NT>(a, b - ty * a.tiles_x.d, ty);
}

// Where population (EX, EY) of row y comes from when x is periodic: the
// stored population, the source row and the x shift, the same for every node
// of the row (the wall rule of pull_index_d2q9 restricted to y walls).
template <int EX, int EY>
LBM_FORCEINLINE void row_source_d2q9(const RunArgs& a, int32_t y, int32_t ny, int& pop, int32_t& sy, int& dx) {
  pop = pop_of_d2q9(EX, EY);
  dx = -EX;
  sy = y - EY;
  if (EY != 0 && (sy < 0 || sy >= ny)) {
    if (a.bc[1] == LBM_CDE_PERIODIC) {
      sy = sy < 0 ? sy + ny : sy - ny;
    } else if (a.bc[1] == LBM_CDE_BOUNCE_BACK) {
      pop = pop_of_d2q9(-EX, -EY);
      sy = y;
      dx = 0;
    } else {
      pop = pop_of_d2q9(EX, -EY);
      sy = a.bc[1] == LBM_CDE_NODE_MIRROR ? y + EY : y;
    }
  }
}

// One row tile of a run with periodic x and constant D, addressed with 32-bit
// byte offsets from uniform bases: the same loads, velocities and collision
// as tile_d2q9 with walls (bitwise the same result), with the wall rule
// evaluated once per row.
template <typename R, int BX, bool NT>
LBM_FORCEINLINE void tile_rows_d2q9(const RunArgs& a, int64_t tile_x, int64_t tile_y) {
  const uint32_t nx = (uint32_t)a.nx;
  const int32_t ny = (int32_t)a.ny;
  const uint32_t x = (uint32_t)tile_x * BX + threadIdx.x;
  if (x >= nx) return;
  const int32_t y = (int32_t)tile_y;
  const uint32_t xm = x == 0 ? nx - 1u : x - 1u, xp = x + 1u == nx ? 0u : x + 1u;
  const char* __restrict__ src = (const char*)a.src;
  char* __restrict__ dst = (char*)a.dst;
  const uint32_t pb = (uint32_t)a.plane * (uint32_t)sizeof(R);
  R f[9];
#define LBM_ROW_PULL(I, EX, EY)                                                                 \
  {                                                                                           \
    int pop, dx;                                                                              \
    int32_t sy;                                                                               \
    row_source_d2q9<EX, EY>(a, y, ny, pop, sy, dx);                                           \
    const uint32_t sx = dx < 0 ? xm : (dx > 0 ? xp : x);                                      \
    f[I] = *(const R*)(src + (uint32_t)pop * pb + ((uint32_t)sy * nx + sx) * (uint32_t)sizeof(R)); \
  }
  LBM_ROW_PULL(0, 0, 0)
  LBM_ROW_PULL(1, 1, 0)
  LBM_ROW_PULL(2, 0, 1)
  LBM_ROW_PULL(3, -1, 0)
  LBM_ROW_PULL(4, 0, -1)
  LBM_ROW_PULL(5, 1, 1)
  LBM_ROW_PULL(6, -1, 1)
  LBM_ROW_PULL(7, -1, -1)
  LBM_ROW_PULL(8, 1, -1)
#undef LBM_ROW_PULL
  R ux, uy;
  if (a.u_kind == U_CONST) {
    ux = (R)a.u_const[0];
    uy = (R)a.u_const[1];
  } else if (a.u_kind == U_SEPARABLE) {
    const char* t = (const char*)a.u_tab;
    const uint32_t stride = (1u + nx + (uint32_t)ny + (uint32_t)a.nz) * (uint32_t)sizeof(R);
    const uint32_t ox = (1u + x) * (uint32_t)sizeof(R), oy = (1u + nx + (uint32_t)y) * (uint32_t)sizeof(R);
    const uint32_t oz = (1u + nx + (uint32_t)ny) * (uint32_t)sizeof(R);
    ux = ((*(const R*)t * *(const R*)(t + ox)) * *(const R*)(t + oy)) * *(const R*)(t + oz);
    uy = ((*(const R*)(t + stride) * *(const R*)(t + stride + ox)) * *(const R*)(t + stride + oy)) *
         *(const R*)(t + stride + oz);
  } else {
    const char* u = (const char*)*a.u_slot;
    const uint32_t o = ((uint32_t)y * nx + x) * 8u;
    const double vx = *(const double*)(u + o), vy = *(const double*)(u + nx * (uint32_t)ny * 8u + o);
    check_speed(a, vx * vx + vy * vy);
    ux = (R)vx;
    uy = (R)vy;
  }
  collide_d2q9<R>(f, ux, uy, (R)a.phi_ref, const_rel2<R>(a));
  const uint32_t nb = ((uint32_t)y * nx + x) * (uint32_t)sizeof(R);
#pragma unroll
  for (int i = 0; i < 9; ++i) store_pop<R, NT>((R*)(dst + i * pb + nb), f[i]);
}

// One step of every active run of a batch, in one persistent launch: the
// grid walks a flat list of BX-wide row tiles spanning all runs.  The
// global step t is read from device memory (so a captured graph stays valid)
// and fixes the buffer parity.  The tile list holds the runs in order[] of
// decreasing step budget (unlimited first), so the runs still active at t
// (budget max_steps > t) own a prefix of it: blocks past that prefix exit at
// once instead of searching and skipping the tiles of finished runs.
template <typename R, int BX, bool NT>
__global__ __launch_bounds__(BX) void k_batch_d2q9(const RunArgs* __restrict__ runs,
                                                   const int64_t* __restrict__ tile_start,
                                                   const int32_t* __restrict__ order, int nruns,
                                                   const int64_t* __restrict__ clock) {
  const int64_t t_global = clock[0];
  // number of active runs: the first position in order[] whose run is done
  int na;
  {
    int lo = 0, hi = nruns;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      const int64_t ms = runs[order[mid]].max_steps;
      if (ms >= 0 && t_global >= ms) hi = mid;
      else lo = mid + 1;
    }
    na = lo;
  }
  const int64_t total = tile_start[na];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = na - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (tile_start[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const RunArgs& ar = runs[order[lo]];
    RunArgs a = ar;
    if (t_global & 1) {
      a.src = ar.dst;
      a.dst = const_cast<void*>(ar.src);
    }
    const int64_t local = t - tile_start[lo];
    const int64_t ntx = (a.nx + BX - 1) / BX;
    if (a.rows32) tile_rows_d2q9<R, BX, NT>(a, local % ntx, local / ntx);
    else tile_d2q9<R, BX, 1, 1, true, NT>(a, local % ntx, local / ntx);
  }
}

// ---- lean batched step ------------------------------------------------------
//
// A batch whose runs all take the row-tile path (x periodic, constant D,
// 32-bit offsets) is stepped from a compact per-run record in device memory
// instead of the full RunArgs: the tile's run is found by a binary search of
// 32-bit tile starts, the row by one multiplication with the run's
// reciprocal tile count, and every access is a global-address-space base
// plus a 32-bit byte offset.  The collision is the same function with the
// same operands, so the state is bitwise that of the other step kernels.

struct BatchRun {
  const char* pop[2];            // population buffers of parity 0 and 1
  const char* u_tab;             // SEPARABLE: tables (type R)
  const double* const* u_slot;   // FIELD: slot of the current FP64 field
  unsigned* u_flag;              // FIELD: set where |u| >= c_s
  uint32_t nx, ny, pb, ntx;      // grid, bytes per population plane, row tiles per row
  uint32_t tile0;                // first tile of the run in the flat list
  int32_t bc_y, u_kind, model;
  int64_t max_steps;             // < 0: unlimited
  double inv_ntx;                // 1 / ntx
  double u_const[2], phi_ref;
  double s1, s2, s7, s8, axx, axy, ayy, s4, s6;
};

// Where population (EX, EY) of row y comes from (row_source_d2q9 on the
// compact record).
template <int EX, int EY>
LBM_FORCEINLINE void row_source_b(int32_t bc_y, int32_t y, int32_t ny, int& pop, int32_t& sy, int& dx) {
  pop = pop_of_d2q9(EX, EY);
  dx = -EX;
  sy = y - EY;
  if (EY != 0 && (sy < 0 || sy >= ny)) {
    if (bc_y == LBM_CDE_PERIODIC) {
      sy = sy < 0 ? sy + ny : sy - ny;
    } else if (bc_y == LBM_CDE_BOUNCE_BACK) {
      pop = pop_of_d2q9(-EX, -EY);
      sy = y;
      dx = 0;
    } else {
      pop = pop_of_d2q9(EX, -EY);
      sy = bc_y == LBM_CDE_NODE_MIRROR ? y + EY : y;
    }
  }
}

template <typename R, int BX, bool NT>
__global__ __launch_bounds__(BX) void k_batch_rows_d2q9(const BatchRun* __restrict__ runs,
                                                        const uint32_t* __restrict__ tile_start, int nruns,
                                                        const int64_t* __restrict__ clock) {
  const int64_t t_global = clock[0];
  // active runs: a prefix of the list (runs are stored by decreasing budget)
  int na;
  {
    int lo = 0, hi = nruns;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      const int64_t ms = runs[mid].max_steps;
      if (ms >= 0 && t_global >= ms) hi = mid;
      else lo = mid + 1;
    }
    na = lo;
  }
  const uint32_t total = tile_start[na];
  const int par = (int)(t_global & 1);
  for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = na - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (tile_start[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const BatchRun& br = runs[lo];
    const uint32_t local = t - br.tile0;
    const uint32_t row = (uint32_t)(((double)local + 0.5) * br.inv_ntx);
    const uint32_t tx = local - row * br.ntx;
    const uint32_t nx = br.nx;
    const int32_t ny = (int32_t)br.ny;
    const uint32_t x = tx * BX + threadIdx.x;
    if (x >= nx) continue;
    const int32_t y = (int32_t)row;
    const uint32_t xm = x == 0 ? nx - 1u : x - 1u, xp = x + 1u == nx ? 0u : x + 1u;
    const char* src = br.pop[par];
    char* dst = (char*)br.pop[par ^ 1];
    const uint32_t pb = br.pb;
    R f[9];
#define LBM_BATCH_PULL(I, EX, EY)                                                                      \
  {                                                                                                  \
    int pop, dx;                                                                                     \
    int32_t sy;                                                                                      \
    row_source_b<EX, EY>(br.bc_y, y, ny, pop, sy, dx);                                               \
    const uint32_t sx = dx < 0 ? xm : (dx > 0 ? xp : x);                                             \
    f[I] = gld<R>(src, (uint32_t)pop * pb + ((uint32_t)sy * nx + sx) * (uint32_t)sizeof(R));         \
  }
    LBM_BATCH_PULL(0, 0, 0)
    LBM_BATCH_PULL(1, 1, 0)
    LBM_BATCH_PULL(2, 0, 1)
    LBM_BATCH_PULL(3, -1, 0)
    LBM_BATCH_PULL(4, 0, -1)
    LBM_BATCH_PULL(5, 1, 1)
    LBM_BATCH_PULL(6, -1, 1)
    LBM_BATCH_PULL(7, -1, -1)
    LBM_BATCH_PULL(8, 1, -1)
#undef LBM_BATCH_PULL
    R ux, uy;
    if (br.u_kind == U_CONST) {
      ux = (R)br.u_const[0];
      uy = (R)br.u_const[1];
    } else if (br.u_kind == U_SEPARABLE) {
      const char* tb = br.u_tab;
      const uint32_t stride = (1u + nx + (uint32_t)ny + 1u) * (uint32_t)sizeof(R);
      const uint32_t ox = (1u + x) * (uint32_t)sizeof(R), oy = (1u + nx + (uint32_t)y) * (uint32_t)sizeof(R);
      const uint32_t oz = (1u + nx + (uint32_t)ny) * (uint32_t)sizeof(R);
      ux = ((gld<R>(tb, 0) * gld<R>(tb, ox)) * gld<R>(tb, oy)) * gld<R>(tb, oz);
      uy = ((gld<R>(tb, stride) * gld<R>(tb, stride + ox)) * gld<R>(tb, stride + oy)) * gld<R>(tb, stride + oz);
    } else {
      const char* u = (const char*)*br.u_slot;
      const uint32_t o = ((uint32_t)y * nx + x) * 8u;
      const double vx = gld<double>(u, o), vy = gld<double>(u, nx * (uint32_t)ny * 8u + o);
      if (vx * vx + vy * vy >= 1.0 / 3.0) *br.u_flag = 1u;
      ux = (R)vx;
      uy = (R)vy;
    }
    const Rel2<R> rc = make_rel2_vals<R>((R)br.axx, (R)br.axy, (R)br.ayy, (R)br.s4, (R)br.s6, br.s1, br.s2, br.s7,
                                         br.s8, br.model);
    collide_d2q9<R>(f, ux, uy, (R)br.phi_ref, rc);
    const uint32_t nb = ((uint32_t)y * nx + x) * (uint32_t)sizeof(R);
#pragma unroll
    for (int i = 0; i < 9; ++i) gst<R, NT>(dst, (uint32_t)i * pb + nb, f[i]);
  }
}

}  // namespace lbm
