// D3Q15 modified-MRT collide-and-stream for gfx950 (the paper's Appendix A).
//
// Velocities (Eq. A.1, in the column order of M in Eq. A.2):
//   0:(0,0,0) 1:(1,0,0) 2:(-1,0,0) 3:(0,1,0) 4:(0,-1,0) 5:(0,0,1) 6:(0,0,-1)
//   7:(1,1,1) 8:(-1,1,1) 9:(1,-1,1) 10:(-1,-1,1) 11:(1,1,-1) 12:(-1,1,-1)
//   13:(1,-1,-1) 14:(-1,-1,-1).
// Rows of M: rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, p_ww, p_xy,
// p_yz, p_xz, m_xyz; squared norms (15, 18, 360, 10, 40, 10, 40, 10, 40, 12,
// 4, 8, 8, 8, 8), so M^-1 = M^T diag(1/norm^2).
//
// Equilibrium (Eq. A.3-A.4) with alpha1 = -6/5, alpha2 = 192 (the values that
// give the prefactor 1/3 in Eq. A.6 and the rest weights 8/15, 1/30):
//   m_eq = phi (1, -1, 8, ux, -ux, uy, -uy, uz, -uz, 0, 0, 0, 0, 0, 0).
// Modified S (Eq. A.5): with v_a = n_{j_a} + s_{q_a} n_{q_a} / 2 the flux rows
// give d_{j_a} = (A v)_a - s_{q_a} n_{q_a}; every other row is diagonal.
// Shifted storage subtracts w phi_ref, w = (8/15, 1/30 x 14); M w = (1, -1, 8, 0...)
// so only the velocity moments see phi_ref (as in 2D).
#pragma once

#include "common.hpp"

namespace lbm {

template <typename R>
struct Rel3 {
  R s1, s2, s4, s6, s8, s9, s10, s11, s12, s13, s14;
  R axx, axy, axz, ayy, ayz, azz;
};

template <typename R>
LBM_FORCEINLINE Rel3<R> const_rel3(const RunArgs& a) {
  Rel3<R> r;
  r.s1 = (R)a.s[1];
  r.s2 = (R)a.s[2];
  r.s9 = (R)a.s[9];
  r.s10 = (R)a.s[10];
  r.s11 = (R)a.s[11];
  r.s12 = (R)a.s[12];
  r.s13 = (R)a.s[13];
  r.s14 = (R)a.s[14];
  r.s4 = (R)a.heat[0];
  r.s6 = (R)a.heat[1];
  r.s8 = (R)a.heat[2];
  r.axx = (R)a.A[0][0];
  r.axy = (R)a.A[0][1];
  r.axz = (R)a.A[0][2];
  r.ayy = (R)a.A[1][1];
  r.ayz = (R)a.A[1][2];
  r.azz = (R)a.A[2][2];
  return r;
}

template <typename R>
LBM_FORCEINLINE void collide_d3q15(R (&f)[15], R ux, R uy, R uz, R phi_ref, const Rel3<R>& r) {
  const R sax = f[1] + f[2] + f[3] + f[4] + f[5] + f[6];
  const R sdg = f[7] + f[8] + f[9] + f[10] + f[11] + f[12] + f[13] + f[14];
  const R phig = f[0] + sax + sdg;
  const R phi = phig + phi_ref;
  const R m1 = sdg - sax - (R)2 * f[0];
  const R m2 = (R)16 * f[0] - (R)4 * sax + sdg;
  const R xa = f[1] - f[2], ya = f[3] - f[4], za = f[5] - f[6];
  // diagonal sums by sign pattern
  const R p78 = f[7] + f[8], m78 = f[7] - f[8];
  const R p910 = f[9] + f[10], m910 = f[9] - f[10];
  const R p1112 = f[11] + f[12], m1112 = f[11] - f[12];
  const R p1314 = f[13] + f[14], m1314 = f[13] - f[14];
  const R xd = m78 + m910 + m1112 + m1314;
  const R yd = p78 - p910 + p1112 - p1314;
  const R zd = p78 + p910 - p1112 - p1314;
  const R m9 = (R)2 * (f[1] + f[2]) - (f[3] + f[4]) - (f[5] + f[6]);
  const R m10 = (f[3] + f[4]) - (f[5] + f[6]);
  const R m11 = m78 - m910 + m1112 - m1314;   // e_x e_y
  const R m12 = p78 - p910 - p1112 + p1314;   // e_y e_z
  const R m13 = m78 + m910 - m1112 - m1314;   // e_x e_z
  const R m14 = m78 - m910 - m1112 + m1314;   // e_x e_y e_z
  // non-equilibrium parts
  const R jx = phi * ux, jy = phi * uy, jz = phi * uz;
  const R n1 = m1 + phig;
  const R n2 = m2 - (R)8 * phig;
  const R n3 = xa + xd - jx, n4 = xd - (R)4 * xa + jx;
  const R n5 = ya + yd - jy, n6 = yd - (R)4 * ya + jy;
  const R n7 = za + zd - jz, n8 = zd - (R)4 * za + jz;
  // heat-flux increments and the coupled flux increments (Eq. A.5)
  const R d4 = r.s4 * n4, d6 = r.s6 * n6, d8 = r.s8 * n8;
  const R vx = n3 + (R)0.5 * d4, vy = n5 + (R)0.5 * d6, vz = n7 + (R)0.5 * d8;
  const R d3 = r.axx * vx + r.axy * vy + r.axz * vz - d4;
  const R d5 = r.axy * vx + r.ayy * vy + r.ayz * vz - d6;
  const R d7 = r.axz * vx + r.ayz * vy + r.azz * vz - d8;
  // increments divided by the squared row norms
  const R a1 = r.s1 * n1 * (R)(1.0 / 18.0);
  const R a2 = r.s2 * n2 * (R)(1.0 / 360.0);
  const R a3 = d3 * (R)0.1, a4 = d4 * (R)0.025;
  const R a5 = d5 * (R)0.1, a6 = d6 * (R)0.025;
  const R a7 = d7 * (R)0.1, a8 = d8 * (R)0.025;
  const R a9 = r.s9 * m9 * (R)(1.0 / 12.0);
  const R a10 = r.s10 * m10 * (R)0.25;
  const R a11 = r.s11 * m11 * (R)0.125;
  const R a12 = r.s12 * m12 * (R)0.125;
  const R a13 = r.s13 * m13 * (R)0.125;
  const R a14 = r.s14 * m14 * (R)0.125;
  // f' = f - M^T a
  const R bax = -a1 - (R)4 * a2;
  const R bdg = a1 + a2;
  const R Xa = a3 - (R)4 * a4, Ya = a5 - (R)4 * a6, Za = a7 - (R)4 * a8;
  const R X = a3 + a4, Y = a5 + a6, Z = a7 + a8;
  f[0] -= (R)16 * a2 - (R)2 * a1;
  f[1] -= bax + Xa + (R)2 * a9;
  f[2] -= bax - Xa + (R)2 * a9;
  f[3] -= bax + Ya - a9 + a10;
  f[4] -= bax - Ya - a9 + a10;
  f[5] -= bax + Za - a9 - a10;
  f[6] -= bax - Za - a9 - a10;
  const R pXY = X + Y, mXY = X - Y;
  const R q1 = a11 + a14, q2 = a11 - a14;    // x y and x y z terms
  const R q3 = a12 + a13, q4 = a12 - a13;    // y z and x z terms
  f[7] -= bdg + pXY + Z + q1 + q3;
  f[8] -= bdg - mXY + Z - q1 + q4;
  f[9] -= bdg + mXY + Z - q1 - q4;
  f[10] -= bdg - pXY + Z + q1 - q3;
  f[11] -= bdg + pXY - Z + q2 - q3;
  f[12] -= bdg - mXY - Z - q2 - q4;
  f[13] -= bdg + mXY - Z - q2 + q4;
  f[14] -= bdg - pXY - Z + q2 + q3;
}

// f_eq(phi, u) - w phi_ref, in double (initialisation).
LBM_FORCEINLINE void equilibrium_d3q15(double (&f)[15], double phi, double ux, double uy, double uz,
                                       double phi_ref) {
  // M^-1 m_eq: axis f = phi (1/30 + e.u/5), diagonal f = phi (1/30 + 3 e.u/40), rest 8 phi/15
  const double a0 = phi / 15.0, a1 = -phi / 18.0, a2 = 8.0 * phi / 360.0;
  const double a3 = phi * ux / 10.0, a4 = -phi * ux / 40.0;
  const double a5 = phi * uy / 10.0, a6 = -phi * uy / 40.0;
  const double a7 = phi * uz / 10.0, a8 = -phi * uz / 40.0;
  const double bax = a0 - a1 - 4.0 * a2, bdg = a0 + a1 + a2;
  const double Xa = a3 - 4.0 * a4, Ya = a5 - 4.0 * a6, Za = a7 - 4.0 * a8;
  const double X = a3 + a4, Y = a5 + a6, Z = a7 + a8;
  const double w0 = 8.0 / 15.0, w = 1.0 / 30.0;
  f[0] = a0 - 2.0 * a1 + 16.0 * a2 - phi_ref * w0;
  f[1] = bax + Xa - phi_ref * w;
  f[2] = bax - Xa - phi_ref * w;
  f[3] = bax + Ya - phi_ref * w;
  f[4] = bax - Ya - phi_ref * w;
  f[5] = bax + Za - phi_ref * w;
  f[6] = bax - Za - phi_ref * w;
  f[7] = bdg + X + Y + Z - phi_ref * w;
  f[8] = bdg - X + Y + Z - phi_ref * w;
  f[9] = bdg + X - Y + Z - phi_ref * w;
  f[10] = bdg - X - Y + Z - phi_ref * w;
  f[11] = bdg + X + Y - Z - phi_ref * w;
  f[12] = bdg - X + Y - Z - phi_ref * w;
  f[13] = bdg + X - Y - Z - phi_ref * w;
  f[14] = bdg - X - Y - Z - phi_ref * w;
}

template <typename R>
LBM_FORCEINLINE void velocity3(const RunArgs& a, int64_t x, int64_t y, int64_t z, R& ux, R& uy, R& uz) {
  if (a.u_kind == U_CONST) {
    ux = (R)a.u_const[0];
    uy = (R)a.u_const[1];
    uz = (R)a.u_const[2];
  } else if (a.u_kind == U_SEPARABLE) {
    const int64_t stride = 1 + a.nx + a.ny + a.nz;
    const R* t = (const R*)a.u_tab;
    R u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R* tc = t + c * stride;
      u[c] = ((tc[0] * tc[1 + x]) * tc[1 + a.nx + y]) * tc[1 + a.nx + a.ny + z];
    }
    ux = u[0];
    uy = u[1];
    uz = u[2];
  } else {
    const double* u = *a.u_slot;
    const int64_t N = a.nx * a.ny * a.nz;
    const int64_t node = (z * a.ny + y) * a.nx + x;
    const double vx = u[node], vy = u[N + node], vz = u[2 * N + node];
    check_speed(a, vx * vx + vy * vy + vz * vz);
    ux = (R)vx;
    uy = (R)vy;
    uz = (R)vz;
  }
}

// Population index of velocity (vx, vy, vz) in the D3Q15 order.
LBM_FORCEINLINE int pop_of_d3q15(int vx, int vy, int vz) {
  const int n = (vx != 0) + (vy != 0) + (vz != 0);
  if (n == 0) return 0;
  if (n == 1) return vx ? (vx > 0 ? 1 : 2) : vy ? (vy > 0 ? 3 : 4) : (vz > 0 ? 5 : 6);
  // diagonals: 7 + (vx < 0) + 2 (vy < 0) + 4 (vz < 0)
  return 7 + (vx < 0) + 2 * (vy < 0) + 4 * (vz < 0);
}

// Pull source of population (EX, EY, EZ) at node (x, y, z) with the
// boundary rules of each axis (see the D2Q9 version).
template <int EX, int EY, int EZ>
LBM_FORCEINLINE int64_t pull_index_d3q15(const RunArgs& a, int64_t x, int64_t y, int64_t z) {
  int64_t s[3] = {x - EX, y - EY, z - EZ};
  const int64_t c0[3] = {x, y, z};
  const int64_t n[3] = {a.nx, a.ny, a.nz};
  const int e[3] = {EX, EY, EZ};
  bool cross[3] = {false, false, false};
  bool bounce = false;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (e[ax] == 0) continue;
    const bool out = s[ax] < 0 || s[ax] >= n[ax];
    if (a.bc[ax] == LBM_CDE_PERIODIC) s[ax] = s[ax] < 0 ? s[ax] + n[ax] : (s[ax] >= n[ax] ? s[ax] - n[ax] : s[ax]);
    else {
      cross[ax] = out;
      bounce |= out && a.bc[ax] == LBM_CDE_BOUNCE_BACK;
    }
  }
  int v[3] = {EX, EY, EZ};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (bounce) {
      v[ax] = -e[ax];
      s[ax] = c0[ax];
    } else if (cross[ax]) {
      v[ax] = -e[ax];
      s[ax] = c0[ax];
    }
  }
  return (int64_t)pop_of_d3q15(v[0], v[1], v[2]) * a.plane + (s[2] * a.ny + s[1]) * a.nx + s[0];
}

// One pull step: block BX x BY threads over (x, y) of one z-plane; each
// thread owns NY rows (y, y + BY, ...).  Loads precede collisions.
template <typename R, int BX, int BY, int NY, bool WALLS, bool NT>
__global__ __launch_bounds__(BX * BY) void k_step_d3q15(const RunArgs a) {
  const uint32_t b = tile_of_block32(blockIdx.x, gridDim.x, a.tiles_x, a.xcd_remap);
  const uint32_t rest = fdiv(b, a.tiles_x), zq = fdiv(rest, a.tiles_y);
  const int64_t tile_x = b - rest * a.tiles_x.d;
  const int64_t tile_y = rest - zq * a.tiles_y.d, z = zq;
  const int64_t x = tile_x * BX + threadIdx.x;
  if (x >= a.nx || z >= a.nz) return;
  const R* __restrict__ src = (const R*)a.src;
  R* __restrict__ dst = (R*)a.dst;
  const int64_t P = a.plane;
  const int64_t y0 = tile_y * (BY * NY) + threadIdx.y;
  const int64_t sxy = a.nx * a.ny;

  R f[NY][15];
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    const int64_t y = y0 + (int64_t)k * BY;
    if (y >= a.ny) continue;
    if constexpr (!WALLS) {
      const int64_t xm = wrap_m(x, a.nx), xp = wrap_p(x, a.nx);
      const int64_t ym = wrap_m(y, a.ny), yp = wrap_p(y, a.ny);
      const int64_t zm = wrap_m(z, a.nz), zp = wrap_p(z, a.nz);
      const int64_t r00 = z * sxy + y * a.nx;             // (y, z)
      const int64_t rm0 = z * sxy + ym * a.nx, rp0 = z * sxy + yp * a.nx;
      const int64_t r0m = zm * sxy + y * a.nx, r0p = zp * sxy + y * a.nx;
      const int64_t rmm = zm * sxy + ym * a.nx, rpm = zm * sxy + yp * a.nx;
      const int64_t rmp = zp * sxy + ym * a.nx, rpp = zp * sxy + yp * a.nx;
      f[k][0] = src[r00 + x];
      f[k][1] = src[1 * P + r00 + xm];    // (1,0,0)   from x-1
      f[k][2] = src[2 * P + r00 + xp];    // (-1,0,0)  from x+1
      f[k][3] = src[3 * P + rm0 + x];     // (0,1,0)   from y-1
      f[k][4] = src[4 * P + rp0 + x];     // (0,-1,0)  from y+1
      f[k][5] = src[5 * P + r0m + x];     // (0,0,1)   from z-1
      f[k][6] = src[6 * P + r0p + x];     // (0,0,-1)  from z+1
      f[k][7] = src[7 * P + rmm + xm];    // (1,1,1)
      f[k][8] = src[8 * P + rmm + xp];    // (-1,1,1)
      f[k][9] = src[9 * P + rpm + xm];    // (1,-1,1)
      f[k][10] = src[10 * P + rpm + xp];  // (-1,-1,1)
      f[k][11] = src[11 * P + rmp + xm];  // (1,1,-1)
      f[k][12] = src[12 * P + rmp + xp];  // (-1,1,-1)
      f[k][13] = src[13 * P + rpp + xm];  // (1,-1,-1)
      f[k][14] = src[14 * P + rpp + xp];  // (-1,-1,-1)
    } else {
      f[k][0] = src[(z * a.ny + y) * a.nx + x];
      f[k][1] = src[pull_index_d3q15<1, 0, 0>(a, x, y, z)];
      f[k][2] = src[pull_index_d3q15<-1, 0, 0>(a, x, y, z)];
      f[k][3] = src[pull_index_d3q15<0, 1, 0>(a, x, y, z)];
      f[k][4] = src[pull_index_d3q15<0, -1, 0>(a, x, y, z)];
      f[k][5] = src[pull_index_d3q15<0, 0, 1>(a, x, y, z)];
      f[k][6] = src[pull_index_d3q15<0, 0, -1>(a, x, y, z)];
      f[k][7] = src[pull_index_d3q15<1, 1, 1>(a, x, y, z)];
      f[k][8] = src[pull_index_d3q15<-1, 1, 1>(a, x, y, z)];
      f[k][9] = src[pull_index_d3q15<1, -1, 1>(a, x, y, z)];
      f[k][10] = src[pull_index_d3q15<-1, -1, 1>(a, x, y, z)];
      f[k][11] = src[pull_index_d3q15<1, 1, -1>(a, x, y, z)];
      f[k][12] = src[pull_index_d3q15<-1, 1, -1>(a, x, y, z)];
      f[k][13] = src[pull_index_d3q15<1, -1, -1>(a, x, y, z)];
      f[k][14] = src[pull_index_d3q15<-1, -1, -1>(a, x, y, z)];
    }
  }
  const R phi_ref = (R)a.phi_ref;
  const Rel3<R> rc = const_rel3<R>(a);
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    const int64_t y = y0 + (int64_t)k * BY;
    if (y >= a.ny) continue;
    const int64_t node = (z * a.ny + y) * a.nx + x;
    R ux, uy, uz;
    velocity3<R>(a, x, y, z, ux, uy, uz);
    collide_d3q15<R>(f[k], ux, uy, uz, phi_ref, rc);
#pragma unroll
    for (int i = 0; i < 15; ++i) store_pop<R, NT>(dst + i * P + node, f[k][i]);
  }
}

}  // namespace lbm
