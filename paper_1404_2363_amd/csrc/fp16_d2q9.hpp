// D2Q9 steps with 16-bit population storage (arithmetic in FP32).
//
// Split storage (the accurate form): per node phi (float) and the
// non-equilibrium part of the post-collision populations,
// h_i = half(2^k (p_i - f_eq_i(phi, u))).  The pull step rebuilds each
// incoming population at its source node s as f_eq_j(phi(s), u(s)) + 2^-k h_j(s)
// (j = i, or the population the wall rule takes), collides in FP32 and keeps
// the new non-equilibrium part, computed in moment space as M^-1 (n - S n);
// 4 + 18 bytes are read and written per node.  phi, phi ux
// and phi uy of a tile and its one-node halo are staged through LDS, so each
// phi is fetched from memory about (BY + 2) / BY times instead of nine and u
// is evaluated once per node of the halo tile instead of at nine sources.
//
// Literal storage: g_i = f_i - w_i phi_ref (as FP32 shifted storage) kept as
// half(2^k g_i).
//
// MRT-A equilibrium in velocity space (Eq. 17 with alpha1 = -8, alpha2 = 8):
//   f_eq_0 = 5 phi / 9, axis f_eq_i = phi (1/18 + e_i.u / 3),
//   diagonal f_eq_i = phi (1/18 + e_i.u / 12).
#pragma once

#include <hip/hip_fp16.h>

#include "common.hpp"
#include "d2q9.hpp"

namespace lbm {

constexpr float kHalfMax = 65504.0f;

// The non-equilibrium part of the post-collision populations times the
// storage scale, h = scale (f' - f_eq(phi, u)), of one node of an MRT-A run
// with unshifted populations f, and phi = sum f.  Since f_eq = M^-1 m_eq
// (m_eq of Eq. 37), h = scale M^-1 (I - S) n with n = M f - m_eq, and
// M^-1 = M^T diag(1/|M_k|^2).  g holds the rows of (I - S) (Eq. 31) already
// multiplied by scale/|M_k|^2 and rounded once on the host: (1 - s1) k36,
// (1 - s2) k36, (1 - s4) k12, (1 - s6) k12, (1 - s7) k4, (1 - s8) k4, then
// row 3 and row 5 of (I - S) over n3..n6 times k6 (kN = scale / N).
LBM_FORCEINLINE void collide_neq_d2q9(const float (&f)[9], float ux, float uy, const float (&g)[14], float (&h)[9],
                                      float& phi) {
  const float sa = f[1] + f[2] + f[3] + f[4];
  const float sd = f[5] + f[6] + f[7] + f[8];
  phi = f[0] + sa + sd;
  const float m1 = 2.0f * sd - sa - 4.0f * f[0];
  const float m2 = 4.0f * f[0] - 2.0f * sa + sd;
  const float dx13 = f[1] - f[3];
  const float dx58 = f[5] - f[6] - f[7] + f[8];
  const float dy24 = f[2] - f[4];
  const float dy56 = f[5] + f[6] - f[7] - f[8];
  const float m3 = dx13 + dx58;
  const float m4 = dx58 - 2.0f * dx13;
  const float m5 = dy24 + dy56;
  const float m6 = dy56 - 2.0f * dy24;
  const float m7 = f[1] - f[2] + f[3] - f[4];
  const float m8 = f[5] - f[6] + f[7] - f[8];
  const float jx = phi * ux, jy = phi * uy;
  const float n1 = m1 + 2.0f * phi, n2 = m2 - 2.0f * phi;
  const float n3 = m3 - jx, n4 = m4 + jx, n5 = m5 - jy, n6 = m6 + jy;
  const float b1 = g[0] * n1, b2 = g[1] * n2, b4 = g[2] * n4, b6 = g[3] * n6;
  const float b7 = g[4] * m7, b8 = g[5] * m8;
  const float b3 = __builtin_fmaf(g[9], n6, __builtin_fmaf(g[8], n5, __builtin_fmaf(g[7], n4, g[6] * n3)));
  const float b5 = __builtin_fmaf(g[13], n6, __builtin_fmaf(g[12], n5, __builtin_fmaf(g[11], n4, g[10] * n3)));
  const float ax = -b1 - 2.0f * b2;
  const float dg = 2.0f * b1 + b2;
  const float q3 = b3 - 2.0f * b4, q5 = b5 - 2.0f * b6;
  const float p3 = b3 + b4, p5 = b5 + b6;
  h[0] = 4.0f * (b2 - b1);
  h[1] = ax + q3 + b7;
  h[2] = ax + q5 - b7;
  h[3] = ax - q3 + b7;
  h[4] = ax - q5 - b7;
  h[5] = dg + p3 + p5 + b8;
  h[6] = dg - p3 + p5 - b8;
  h[7] = dg - p3 - p5 + b8;
  h[8] = dg + p3 - p5 - b8;
}


LBM_FORCEINLINE float feq_d2q9(int i, float phi, float ux, float uy) {
  if (i == 0) return phi * (5.0f / 9.0f);
  const int ex = (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0;
  const int ey = (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0;
  const float eu = (float)ex * ux + (float)ey * uy;
  return i <= 4 ? phi * (1.0f / 18.0f + eu * (1.0f / 3.0f)) : phi * (1.0f / 18.0f + eu * (1.0f / 12.0f));
}

// FP32 rest weights of the split rebuild, 1/18 and 5/9 to 6e-8 and chosen so
// that kW0 + 8 kW1 == 1 exactly: the stored part h sums to zero over a node,
// so the rebuilt populations carry exactly phi times the sum of these
// weights, and weights rounded independently (5/9 and 1/18 each to nearest)
// would add 3e-8 phi per node and step.
constexpr float kW1 = 0x1.c71c7p-5f;  // 0.05555555224...
constexpr float kW0 = 0x1.1c71c8p-1f;  // 0.55555558204... = 1 - 8 kW1
static_assert(kW0 + 8.0f * kW1 == 1.0f, "split rest weights must sum to one");

// f_eq of a moving population from phi and e.(phi u) at its node, in one
// fixed rounding order (both split kernels use it, so their results are
// bitwise equal): c = 1/3 on the axes, 1/12 on the diagonals.  The two
// populations of a node with opposite velocities carry e.(phi u) of opposite
// sign; both come from t = w phi + c |e.(phi u)|, one as t and the other as
// 2 w phi - t (exact), so every such pair sums to exactly 2 w phi.  Rounding
// w phi + c e.(phi u) and w phi - c e.(phi u) separately is biased where one
// of them crosses a power of two (the rounding grid changes there, and both
// terms scale with phi): the total then drifted by about +3e-10 per step.
// p = w phi = phi * kW1.
LBM_FORCEINLINE float feq_moving_w(float p, float ej, float c) {
  const float t = __builtin_fmaf(fabsf(ej), c, p);
  return ej >= 0.0f ? t : __builtin_fmaf(2.0f, p, -t);
}
LBM_FORCEINLINE float feq_moving(float ph, float ej, float c) { return feq_moving_w(ph * kW1, ej, c); }

// e.(phi u) with e = (ex, ey), ex, ey in {-1, 0, 1}: exact for one nonzero
// component (no addition of a zero product), one rounding for two.
LBM_FORCEINLINE float e_dot_j(int ex, int ey, float jx, float jy) {
  if (ex == 0) return (float)ey * jy;
  if (ey == 0) return (float)ex * jx;
  return __builtin_fmaf((float)ey, jy, (float)ex * jx);
}

// Scale, round and saturate to half; flags an out-of-range value.
LBM_FORCEINLINE __half to_half(float v, float scale, bool& over) {
  float s = v * scale;
  if (!(fabsf(s) <= kHalfMax)) {
    over = true;
    s = s != s ? 0.0f : (s > 0.0f ? kHalfMax : -kHalfMax);
  }
  return __float2half_rn(s);
}

// Already scaled value to half: clamped to the half range (finite values
// saturate); the largest magnitude seen is kept for the overflow flag.
LBM_FORCEINLINE __half to_half_clamped(float s, float& mx) {
  mx = fmaxf(mx, fabsf(s));
  return __float2half_rn(__builtin_amdgcn_fmed3f(s, -kHalfMax, kHalfMax));
}

LBM_FORCEINLINE int64_t wrap_any(int64_t i, int64_t n) {
  const int64_t r = i % n;
  return r < 0 ? r + n : r;
}

// Source of population (EX, EY) at (x, y): population index, node, and the
// offset (dx, dy) of the source node from (x, y) (for the LDS phi tile).
template <int EX, int EY>
LBM_FORCEINLINE void pull_source_d2q9(const RunArgs& a, int64_t x, int64_t y, int& pop, int64_t& sx, int64_t& sy,
                                      int& dx, int& dy) {
  sx = x - EX;
  sy = y - EY;
  dx = -EX;
  dy = -EY;
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
    dx = dy = 0;
  } else {
    if (cx) { vx = -EX; sx = x; dx = 0; }
    if (cy) { vy = -EY; sy = y; dy = 0; }
  }
  pop = pop_of_d2q9(vx, vy);
}

// Halo coordinate: periodic axes wrap (one conditional step when the axis is
// longer than the tile, a modulo otherwise), other axes clamp (the value of
// a node beyond a wall is never used).
LBM_FORCEINLINE int64_t halo_coord(int64_t g, int64_t n, bool periodic, bool long_axis) {
  if (!periodic) return g < 0 ? 0 : (g >= n ? n - 1 : g);
  if (long_axis) return g < 0 ? g + n : (g >= n ? g - n : g);
  return wrap_any(g, n);
}

template <int BX, int BY, bool WALLS>
__global__ __launch_bounds__(BX * BY) void k_step_d2q9_split(const RunArgs a, unsigned* __restrict__ overflow) {
  // phi, phi ux, phi uy of the tile and its one-node halo
  __shared__ float sphi[BY + 2][BX + 2], sjx[BY + 2][BX + 2], sjy[BY + 2][BX + 2];
  const uint32_t b = tile_of_block32(blockIdx.x, gridDim.x, a.tiles_x, a.xcd_remap);
  const uint32_t tyi = fdiv(b, a.tiles_x);
  const int64_t tx0 = (int64_t)(b - tyi * a.tiles_x.d) * BX, ty0 = (int64_t)tyi * BY;
  const float* __restrict__ phis = (const float*)a.src_phi;
  const int tid = threadIdx.y * BX + threadIdx.x;
  const bool px = a.bc[0] == LBM_CDE_PERIODIC, py = a.bc[1] == LBM_CDE_PERIODIC;
  const bool lx_long = a.nx > BX, ly_long = a.ny > BY;
  for (int k = tid; k < (BX + 2) * (BY + 2); k += BX * BY) {
    const int lx = k % (BX + 2), ly = k / (BX + 2);
    const int64_t gx = halo_coord(tx0 + lx - 1, a.nx, px, lx_long);
    const int64_t gy = halo_coord(ty0 + ly - 1, a.ny, py, ly_long);
    const float ph = phis[gy * a.nx + gx];
    float ux, uy;
    velocity2<float>(a, gx, gy, ux, uy);
    sphi[ly][lx] = ph;
    sjx[ly][lx] = ph * ux;
    sjy[ly][lx] = ph * uy;
  }
  __syncthreads();
  const int64_t x = tx0 + threadIdx.x, y = ty0 + threadIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  const __half* __restrict__ src = (const __half*)a.src;
  const float inv = a.split_inv;
  float f[9];
  // f_i = f_eq_j(phi(s), u(s)) + h_j(s) / scale with f_eq_j = w phi + c e_j.(phi u)
#define LBM_SPLIT_PULL(I, EX, EY)                                                        \
  {                                                                                      \
    int pop, dx, dy;                                                                     \
    int64_t sx, sy;                                                                      \
    if constexpr (WALLS) {                                                               \
      pull_source_d2q9<EX, EY>(a, x, y, pop, sx, sy, dx, dy);                            \
    } else {                                                                             \
      pop = I;                                                                           \
      dx = -(EX);                                                                        \
      dy = -(EY);                                                                        \
      sx = (EX) == 1 ? wrap_m(x, a.nx) : (EX) == -1 ? wrap_p(x, a.nx) : x;               \
      sy = (EY) == 1 ? wrap_m(y, a.ny) : (EY) == -1 ? wrap_p(y, a.ny) : y;               \
    }                                                                                    \
    const int ly = threadIdx.y + 1 + dy, lx = threadIdx.x + 1 + dx;                      \
    const float ph = sphi[ly][lx], jx = sjx[ly][lx], jy = sjy[ly][lx];                   \
    float feq;                                                                           \
    if (pop == 0) feq = ph * kW0;                                                        \
    else {                                                                               \
      const int ex = (pop == 1 || pop == 5 || pop == 8) ? 1 : (pop == 3 || pop == 6 || pop == 7) ? -1 : 0; \
      const int ey = (pop == 2 || pop == 5 || pop == 6) ? 1 : (pop == 4 || pop == 7 || pop == 8) ? -1 : 0; \
      const float ej = e_dot_j(ex, ey, jx, jy);                                          \
      feq = feq_moving(ph, ej, pop <= 4 ? (1.0f / 3.0f) : (1.0f / 12.0f));               \
    }                                                                                    \
    f[I] = __builtin_fmaf(__half2float(src[(int64_t)pop * a.plane + sy * a.nx + sx]), inv, feq); \
  }
  LBM_SPLIT_PULL(0, 0, 0)
  LBM_SPLIT_PULL(1, 1, 0)
  LBM_SPLIT_PULL(2, 0, 1)
  LBM_SPLIT_PULL(3, -1, 0)
  LBM_SPLIT_PULL(4, 0, -1)
  LBM_SPLIT_PULL(5, 1, 1)
  LBM_SPLIT_PULL(6, -1, 1)
  LBM_SPLIT_PULL(7, -1, -1)
  LBM_SPLIT_PULL(8, 1, -1)
#undef LBM_SPLIT_PULL
  float ux, uy;
  velocity2<float>(a, x, y, ux, uy);
  float h[9], phi;
  collide_neq_d2q9(f, ux, uy, a.split_g, h, phi);
  const int64_t node = y * a.nx + x;
  ((float*)a.dst_phi)[node] = phi;
  __half* __restrict__ dst = (__half*)a.dst;
  float mx = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) dst[i * a.plane + node] = to_half_clamped(h[i], mx);
  if (!(mx <= kHalfMax)) overflow[0] = 1u;
}

// x mod n for x in [0, 3n) (one or two conditional subtractions).
LBM_FORCEINLINE uint32_t mod3n(uint32_t x, uint32_t n) {
  x = x >= n ? x - n : x;
  return x >= n ? x - n : x;
}

// Split storage on a fully periodic grid with nx >= BX, ny >= BY and every
// byte offset below 4 GiB (phi plane and the nine half planes): every access is a
// uniform base plus a 32-bit byte offset, the tile's halo indices need at
// most two conditional subtractions, every load is issued before the one
// barrier, and the stored part comes straight out of the moment-space
// collision, already scaled.  A separable u is multiplied in the same order
// as velocity2, so both kernels give bitwise the same state.  NT: streaming
// stores.  UK: the velocity, 0 constant, 1 separable, 2 separable with unit
// z factors (exactly 1, so the last product of velocity2's order is skipped).
template <int BX, int BY, bool NT, int UK>
__global__ __launch_bounds__(BX * BY) void k_step_d2q9_split_p(const RunArgs a, unsigned* __restrict__ overflow) {
  constexpr int NT_ = BX * BY, RN = 2 * (BX + 2) + 2 * BY;  // ring (halo) entries of the tile
  constexpr int NR = (RN + NT_ - 1) / NT_;                      // ring entries per thread
  // w phi, phi ux, phi uy of the tile and its halo
  __shared__ float swp[BY + 2][BX + 2], sjx[BY + 2][BX + 2], sjy[BY + 2][BX + 2];
  const uint32_t nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
  const uint32_t b = tile_of_block32(blockIdx.x, gridDim.x, a.tiles_x, a.xcd_remap);
  const uint32_t tyi = fdiv(b, a.tiles_x);
  const uint32_t tx0 = (b - tyi * a.tiles_x.d) * BX, ty0 = tyi * BY;
  const char* __restrict__ phis = (const char*)a.src_phi;
  const int tid = threadIdx.y * BX + threadIdx.x;
  constexpr bool sep = UK != 0;
  const char* __restrict__ tb = (const char*)a.u_tab;
  const uint32_t tstride = (1u + nx + ny + 1u) * 4u;  // bytes per velocity component table
  const float ax0 = sep ? *(const float*)tb : 0.0f, ay0 = sep ? *(const float*)(tb + tstride) : 0.0f;
  const float zx = UK == 1 ? *(const float*)(tb + (1u + nx + ny) * 4u) : 1.0f;
  const float zy = UK == 1 ? *(const float*)(tb + tstride + (1u + nx + ny) * 4u) : 1.0f;
  const float cux = (float)a.u_const[0], cuy = (float)a.u_const[1];
  // velocity2's product order; a unit z factor is exact and skipped
  auto su = [&](float a0, float xv, float yv, float z) { return UK == 1 ? ((a0 * xv) * yv) * z : (a0 * xv) * yv; };
  // Loads in the order their results are needed, all issued before the first
  // wait: this thread's node (phi, velocity factors), one ring entry of the
  // tile's halo, then the nine stored halves (waited for after the barrier).
  // A thread past the grid edge stages the node its tile position wraps to
  // (a neighbour may pull from it) and reads, and discards, valid halves.
  const uint32_t xr = tx0 + threadIdx.x, yr = ty0 + threadIdx.y;
  const bool active = xr < nx && yr < ny;
  const uint32_t x = xr < nx ? xr : xr - nx, y = yr < ny ? yr : yr - ny;
  const float ph_own = *(const float*)(phis + (y * nx + x) * 4u);
  float ox = 0.0f, oy = 0.0f, px = 0.0f, py = 0.0f;
  if constexpr (sep) {
    ox = *(const float*)(tb + (1u + x) * 4u);
    oy = *(const float*)(tb + (1u + nx + y) * 4u);
    px = *(const float*)(tb + tstride + (1u + x) * 4u);
    py = *(const float*)(tb + tstride + (1u + nx + y) * 4u);
  }
  float hphi[NR], hx[NR], hy[NR], vx[NR], vy[NR];
  int hl[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    // the ring is not a multiple of the block: waves past its end skip the
    // staging (uniformly, so the remaining loads keep their order)
    if (tid + j * NT_ >= RN) continue;
    const int r = tid + j * NT_;
    int lx, ly;
    if (r < BX + 2) {
      lx = r;
      ly = 0;
    } else if (r < 2 * (BX + 2)) {
      lx = r - (BX + 2);
      ly = BY + 1;
    } else if (r < 2 * (BX + 2) + BY) {
      lx = 0;
      ly = 1 + r - 2 * (BX + 2);
    } else {
      lx = BX + 1;
      ly = 1 + r - 2 * (BX + 2) - BY;
    }
    hl[j] = ly * (BX + 2) + lx;
    const uint32_t gx = mod3n(tx0 + (uint32_t)lx + nx - 1u, nx), gy = mod3n(ty0 + (uint32_t)ly + ny - 1u, ny);
    hphi[j] = *(const float*)(phis + (gy * nx + gx) * 4u);
    hx[j] = hy[j] = vx[j] = vy[j] = 0.0f;
    if constexpr (sep) {
      hx[j] = *(const float*)(tb + (1u + gx) * 4u);
      vx[j] = *(const float*)(tb + (1u + nx + gy) * 4u);
      hy[j] = *(const float*)(tb + tstride + (1u + gx) * 4u);
      vy[j] = *(const float*)(tb + tstride + (1u + nx + gy) * 4u);
    }
  }
  const uint32_t xm = x == 0 ? nx - 1u : x - 1u, xp = x + 1u == nx ? 0u : x + 1u;
  const uint32_t rm = (y == 0 ? ny - 1u : y - 1u) * nx, r0 = y * nx, rp = (y + 1u == ny ? 0u : y + 1u) * nx;
  const char* __restrict__ src = (const char*)a.src;
  const uint32_t pb = (uint32_t)a.plane * 2u;  // bytes per plane
  const uint32_t off[9] = {r0 + x, r0 + xm, rm + x, r0 + xp, rp + x, rm + xm, rm + xp, rp + xp, rp + xm};
  __half raw[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) raw[i] = *(const __half*)(src + i * pb + off[i] * 2u);
  // w phi, phi ux, phi uy of the tile; u in velocity2's product order
  const float ux = sep ? su(ax0, ox, oy, zx) : cux;
  const float uy = sep ? su(ay0, px, py, zy) : cuy;
  swp[threadIdx.y + 1][threadIdx.x + 1] = ph_own * kW1;
  sjx[threadIdx.y + 1][threadIdx.x + 1] = ph_own * ux;
  sjy[threadIdx.y + 1][threadIdx.x + 1] = ph_own * uy;
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (tid + j * NT_ < RN) {
      const float hux = sep ? su(ax0, hx[j], vx[j], zx) : cux;
      const float huy = sep ? su(ay0, hy[j], vy[j], zy) : cuy;
      (&swp[0][0])[hl[j]] = hphi[j] * kW1;
      (&sjx[0][0])[hl[j]] = hphi[j] * hux;
      (&sjy[0][0])[hl[j]] = hphi[j] * huy;
    }
  }
  __syncthreads();
  if (!active) return;
  const float inv = a.split_inv;
  const int lx = threadIdx.x + 1, ly = threadIdx.y + 1;
  float f[9];
#define LBM_SPLIT_P(I, EX, EY)                                                                       \
  {                                                                                                \
    const int sx = lx - (EX), sy = ly - (EY);                                                      \
    float feq;                                                                                     \
    if ((I) == 0) feq = ph_own * kW0;                                                              \
    else                                                                                           \
      feq = feq_moving_w(swp[sy][sx], e_dot_j((EX), (EY), (EX) != 0 ? sjx[sy][sx] : 0.0f,           \
                                              (EY) != 0 ? sjy[sy][sx] : 0.0f),                     \
                         ((EX) == 0 || (EY) == 0) ? (1.0f / 3.0f) : (1.0f / 12.0f));               \
    f[I] = __builtin_fmaf(__half2float(raw[I]), inv, feq);                                         \
  }
  LBM_SPLIT_P(0, 0, 0)
  LBM_SPLIT_P(1, 1, 0)
  LBM_SPLIT_P(2, 0, 1)
  LBM_SPLIT_P(3, -1, 0)
  LBM_SPLIT_P(4, 0, -1)
  LBM_SPLIT_P(5, 1, 1)
  LBM_SPLIT_P(6, -1, 1)
  LBM_SPLIT_P(7, -1, -1)
  LBM_SPLIT_P(8, 1, -1)
#undef LBM_SPLIT_P
  float h[9], phi;
  collide_neq_d2q9(f, ux, uy, a.split_g, h, phi);
  uint32_t nb = (r0 + x) * 2u;  // byte offset of the node in a half plane
  // keep nb an opaque 32-bit value so that every store below takes the
  // uniform-base + 32-bit-offset form instead of a 64-bit address per store
  asm volatile("" : "+v"(nb));
  store_pop<float, NT>((float*)((char*)a.dst_phi + nb * 2u), phi);
  float mx = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const unsigned short v = __half_as_ushort(to_half_clamped(h[i], mx));
    // a uniform plane base from the arguments plus the node's 32-bit offset
    unsigned short* p = (unsigned short*)((char*)a.split_dst[i] + nb);
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
  }
  if (!(mx <= kHalfMax)) overflow[0] = 1u;
}

// Literal half storage of the shifted populations, same step as FP32.
template <int BX, bool WALLS>
__global__ __launch_bounds__(BX) void k_step_d2q9_half(const RunArgs a, unsigned* __restrict__ overflow) {
  const uint32_t b = tile_of_block32(blockIdx.x, gridDim.x, a.tiles_x, a.xcd_remap);
  const uint32_t yq = fdiv(b, a.tiles_x);
  const int64_t x = (int64_t)(b - yq * a.tiles_x.d) * BX + threadIdx.x, y = yq;
  if (x >= a.nx) return;
  const __half* __restrict__ src = (const __half*)a.src;
  const float inv = (float)a.fp16_inv_scale;
  float f[9];
#define LBM_HALF_PULL(I, EX, EY)                                                                       \
  {                                                                                                    \
    int64_t idx;                                                                                       \
    if constexpr (WALLS) {                                                                             \
      idx = pull_index_d2q9<EX, EY>(a, x, y);                                                          \
    } else {                                                                                           \
      const int64_t sx = (EX) == 1 ? wrap_m(x, a.nx) : (EX) == -1 ? wrap_p(x, a.nx) : x;              \
      const int64_t sy = (EY) == 1 ? wrap_m(y, a.ny) : (EY) == -1 ? wrap_p(y, a.ny) : y;              \
      idx = (int64_t)(I) * a.plane + sy * a.nx + sx;                                                   \
    }                                                                                                  \
    f[I] = __half2float(src[idx]) * inv;                                                               \
  }
  LBM_HALF_PULL(0, 0, 0)
  LBM_HALF_PULL(1, 1, 0)
  LBM_HALF_PULL(2, 0, 1)
  LBM_HALF_PULL(3, -1, 0)
  LBM_HALF_PULL(4, 0, -1)
  LBM_HALF_PULL(5, 1, 1)
  LBM_HALF_PULL(6, -1, 1)
  LBM_HALF_PULL(7, -1, -1)
  LBM_HALF_PULL(8, 1, -1)
#undef LBM_HALF_PULL
  float ux, uy;
  velocity2<float>(a, x, y, ux, uy);
  collide_d2q9<float>(f, ux, uy, (float)a.phi_ref, const_rel2<float>(a));
  const int64_t node = y * a.nx + x;
  __half* __restrict__ dst = (__half*)a.dst;
  const float scale = (float)a.fp16_scale;
  bool over = false;
#pragma unroll
  for (int i = 0; i < 9; ++i) dst[i * a.plane + node] = to_half(f[i], scale, over);
  if (over) overflow[0] = 1u;
}

// Largest magnitude, per block, of what 16-bit storage will hold for this
// run: the non-equilibrium part after the first step (split form), or the
// shifted equilibrium populations (literal form).  Block maxima go to
// partial[blockIdx.x]; a second pass takes the maximum of those.
__global__ __launch_bounds__(256) void k_fp16_probe(const RunArgs a, const double* __restrict__ phi0, int split,
                                                    float* __restrict__ partial) {
  __shared__ float sh[256];
  const int64_t N = a.nx * a.ny;
  float m = 0.0f;
  for (int64_t node = (int64_t)blockIdx.x * 256 + threadIdx.x; node < N; node += (int64_t)gridDim.x * 256) {
    const int64_t x = node % a.nx, y = node / a.nx;
    if (split) {
      // first step from the equilibrium state: f_i = f_eq(phi0(s), u(s)) at the pull sources
      float f[9];
      const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
      const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
      for (int i = 0; i < 9; ++i) {
        int64_t sx = x - ex[i], sy = y - ey[i];
        int pop = i;
        const bool ox = sx < 0 || sx >= a.nx, oy = sy < 0 || sy >= a.ny;
        if (a.bc[0] == LBM_CDE_PERIODIC) sx = wrap_any(sx, a.nx);
        if (a.bc[1] == LBM_CDE_PERIODIC) sy = wrap_any(sy, a.ny);
        const bool cx = ox && a.bc[0] != LBM_CDE_PERIODIC, cy = oy && a.bc[1] != LBM_CDE_PERIODIC;
        int vx = ex[i], vy = ey[i];
        if ((cx && a.bc[0] == LBM_CDE_BOUNCE_BACK) || (cy && a.bc[1] == LBM_CDE_BOUNCE_BACK)) {
          vx = -vx;
          vy = -vy;
          sx = x;
          sy = y;
        } else {
          if (cx) { vx = -vx; sx = x; }
          if (cy) { vy = -vy; sy = y; }
        }
        pop = pop_of_d2q9(vx, vy);
        float ux, uy;
        velocity2<float>(a, sx, sy, ux, uy);
        f[i] = feq_d2q9(pop, (float)phi0[sy * a.nx + sx], ux, uy);
      }
      float ux, uy;
      velocity2<float>(a, x, y, ux, uy);
      const float phi = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
      collide_d2q9<float>(f, ux, uy, 0.0f, const_rel2<float>(a));
      for (int i = 0; i < 9; ++i) m = fmaxf(m, fabsf(f[i] - feq_d2q9(i, phi, ux, uy)));
    } else {
      double u[3];
      float ux, uy;
      velocity2<float>(a, x, y, ux, uy);
      u[0] = ux;
      u[1] = uy;
      double f[9];
      equilibrium_d2q9(f, phi0[node], u[0], u[1], a.phi_ref);
      for (int i = 0; i < 9; ++i) m = fmaxf(m, fabsf((float)f[i]));
    }
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_max_final(const float* __restrict__ partial, int n, float* __restrict__ out) {
  __shared__ float sh[256];
  float m = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) m = fmaxf(m, partial[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Initial split or literal 16-bit state from phi0 (the equilibrium).
__global__ __launch_bounds__(256) void k_init_d2q9_fp16(const RunArgs a, const double* __restrict__ phi0, int split,
                                                        unsigned* __restrict__ overflow) {
  const int64_t N = a.nx * a.ny;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  __half* dst = (__half*)a.dst;
  bool over = false;
  if (split) {
    ((float*)a.dst_phi)[node] = (float)phi0[node];
    for (int i = 0; i < 9; ++i) dst[i * a.plane + node] = __float2half_rn(0.0f);
  } else {
    const int64_t x = node % a.nx, y = node / a.nx;
    float ux, uy;
    velocity2<float>(a, x, y, ux, uy);
    double f[9];
    equilibrium_d2q9(f, phi0[node], (double)ux, (double)uy, a.phi_ref);
    for (int i = 0; i < 9; ++i) dst[i * a.plane + node] = to_half((float)f[i], (float)a.fp16_scale, over);
  }
  if (over) overflow[0] = 1u;
}

}  // namespace lbm
