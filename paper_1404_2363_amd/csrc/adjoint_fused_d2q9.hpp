// Several adjoint steps per launch for D2Q9 runs periodic on both axes: the
// checkpoint segment's forward recomputation and its reverse sweep through
// LDS, as the multi-step forward kernel does (fused_d2q9.hpp).
//
// The reverse step at a node gathers mu_{t+1} from the push destinations
// y + e_i, so it too depends only on nodes within one node: a block owns a
// tile, the first of its T reverse steps gathers mu from memory over the tile
// widened by T - 1 nodes, the next ones from LDS over rings shrinking by one
// node per step, and the last stores mu_t of the tile itself.  Each node's
// step is adjoint_node with v of that step read from the segment's scratch,
// so mu is bitwise that of one-step launches.  The gradient contributions of
// the tile's own nodes (each computed once per step by the block that owns
// it) accumulate in LDS in the one-step sequence's order and precision: FP32
// runs add them to the segment's FP32 partial and, when the launch ends with
// the segment's first step, fold partial and last contribution into the FP64
// gradient; FP64 runs add them to the FP64 gradient.  The segment's last step
// (first reverse step), which takes the injected dL/dphi, stays a one-step
// launch.
#pragma once

#include <type_traits>

#include "adjoint_d2q9.hpp"
#include "fused_d2q9.hpp"

namespace lbm {

// Forward recomputation: T steps of the run from a.src, v of every step into
// vout (step s of the launch at vout + s * vstep bytes, planes [2][nx ny]),
// the end state into a.dst when store_end.
template <typename R, int BX, int BY, int NY, int T, int UK, bool NP>
__global__ __launch_bounds__(BX * BY) void k_fused_v_d2q9(const RunArgs a, char* vout, int64_t vstep, int store_end) {
  // XCD-contiguous block order: neighbouring tiles, which share halo rows,
  // run on one XCD and its L2
  const uint32_t b = tile_of_block32(blockIdx.x, gridDim.x, a.tiles_x, 1);
  const uint32_t ntx = ((uint32_t)a.nx + BX - 1) / BX, tyi = b / ntx;
  fused_tile<R, BX, BY, NY, T, UK, false, true, NP>(a, b - tyi * ntx, tyi, vout, vstep, store_end != 0);
}

// Reverse steps k_hi, k_hi - 1, ..., k_hi - T + 1 of a segment: mu_in =
// mu_{k_hi + 1}, v of step k_hi - s at v_hi - s * vstep bytes, mu_out =
// mu_{k_hi - T + 1}; grad (FP64 [3][N]) and part (FP32 [3][N]) as described
// above (fold: the launch ends with the segment's first step, FP32 only).
template <typename R, int BX, int BY, int NY, int T, bool NP>
__global__ __launch_bounds__(BX * BY) void k_fused_adj_d2q9(const RunArgs a, const char* __restrict__ v_hi,
                                                           int64_t vstep, const R* __restrict__ mu_in,
                                                           R* __restrict__ mu_out, double* __restrict__ grad,
                                                           float* __restrict__ part, double inv_kappa, int fold) {
  constexpr bool F64 = sizeof(R) == 8;
  using Acc = typename std::conditional<F64, double, float>::type;
  constexpr int NTH = BX * BY, TX = BX, TY = BY * NY, RG = T - 1;
  constexpr int W0 = TX + 2 * RG, H0 = TY + 2 * RG, C0 = W0 * H0, NI = TX * TY;
  constexpr int K0 = (C0 + NTH - 1) / NTH;
  __shared__ R lds[9 * C0];
  __shared__ Acc acc[3 * NI];

  const int tid = threadIdx.y * BX + threadIdx.x;
  const int32_t nx = (int32_t)a.nx, ny = (int32_t)a.ny;
  // XCD-contiguous block order, as the forward recomputation
  const uint32_t b = tile_of_block32(blockIdx.x, gridDim.x, a.tiles_x, 1);
  const uint32_t ntx = ((uint32_t)nx + BX - 1) / BX, tyi = b / ntx, txi = b - tyi * ntx;
  const int32_t x0 = (int32_t)txi * TX - RG, y0 = (int32_t)tyi * TY - RG;
  const uint32_t N = (uint32_t)nx * (uint32_t)ny;
  const size_t pb = (size_t)a.plane * sizeof(R);
  constexpr uint32_t E = sizeof(R);
  const Rel2<R> rc = const_rel2<R>(a);

  // the running sums of the tile's own nodes
  for (int j = tid; j < NI; j += NTH) {
    const int ly = j / TX, lx = j - ly * TX;
    const int32_t x = x0 + RG + lx, y = y0 + RG + ly;
    if (x >= nx || y >= ny) continue;
    const uint32_t n = __umul24((uint32_t)y, (uint32_t)nx) + x;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c * NI + j] = F64 ? (Acc)grad[c * N + n] : (Acc)part[c * N + n];
  }

  auto own = [&](int lx, int ly) {
    return lx >= RG && lx < RG + TX && ly >= RG && ly < RG + TY && x0 + lx < nx && y0 + ly < ny;
  };
  // reverse step s of the launch at grid node (x, y), local (lx, ly)
  auto step = [&](R(&l)[9], int32_t x, int32_t y, int s, R(&m)[9], R(&gc)[3]) {
    const char* vb = v_hi - s * vstep;
    const uint32_t o = (__umul24((uint32_t)y, (uint32_t)nx) + x) * E;
    const R vx = gld<R>(vb, o), vy = gld<R>(vb + (size_t)N * E, o);
    R ux, uy;
    velocity2<R>(a, x, y, ux, uy);
    if constexpr (NP) adjoint_node<R>(l, vx, vy, ux, uy, node_rel2<R>(a, (int64_t)y * nx + x), m, gc);
    else adjoint_node<R>(l, vx, vy, ux, uy, rc, m, gc);
  };
  auto add = [&](int lx, int ly, const R(&gc)[3]) {
    const int ii = (ly - RG) * TX + (lx - RG);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if constexpr (F64) acc[c * NI + ii] = acc[c * NI + ii] + inv_kappa * (double)gc[c];
      else acc[c * NI + ii] = acc[c * NI + ii] + (float)gc[c];
    }
  };
  // gather of local node (lx, ly) from LDS: population i from (lx + ex, ly + ey)
  auto gather = [&](R(&l)[9], int lx, int ly) {
#pragma unroll
    for (int i = 0; i < 9; ++i) l[i] = lds[i * C0 + (ly + kEy9[i]) * W0 + (lx + kEx9[i])];
  };
  __syncthreads();

  // step 0 of the launch: mu from memory over the widened tile
  {
    const char* mb = (const char*)mu_in;
    const uint32_t rlast = (uint32_t)(ny - 1) * (uint32_t)nx;  // offset of the last row
    R f[K0][9];
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      const int j = tid + k * NTH;
      if (K0 * NTH > C0 && j >= C0) continue;
      const int ly = j / W0, lx = j - ly * W0;
      const int32_t x = wrap_once(x0 + lx, nx), y = wrap_once(y0 + ly, ny);
      const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x + 1 == nx ? 0 : x + 1;
      const uint32_t r0 = __umul24((uint32_t)y, (uint32_t)nx), rm = y == 0 ? rlast : r0 - nx,
                     rp = y + 1 == ny ? 0u : r0 + nx;
      // population (ex, ey) from its push destination (x + ex, y + ey)
      f[k][0] = gld<R>(mb, (r0 + x) * E);
      f[k][1] = gld<R>(mb + 1 * pb, (r0 + xp) * E);
      f[k][2] = gld<R>(mb + 2 * pb, (rp + x) * E);
      f[k][3] = gld<R>(mb + 3 * pb, (r0 + xm) * E);
      f[k][4] = gld<R>(mb + 4 * pb, (rm + x) * E);
      f[k][5] = gld<R>(mb + 5 * pb, (rp + xp) * E);
      f[k][6] = gld<R>(mb + 6 * pb, (rp + xm) * E);
      f[k][7] = gld<R>(mb + 7 * pb, (rm + xm) * E);
      f[k][8] = gld<R>(mb + 8 * pb, (rm + xp) * E);
    }
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      const int j = tid + k * NTH;
      if (K0 * NTH > C0 && j >= C0) continue;
      const int ly = j / W0, lx = j - ly * W0;
      R m[9], gc[3];
      step(f[k], wrap_once(x0 + lx, nx), wrap_once(y0 + ly, ny), 0, m, gc);
      if (own(lx, ly)) add(lx, ly, gc);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[i * C0 + j] = m[i];
    }
  }
  __syncthreads();

  // steps 1 .. T-2: in place in LDS over the ring of width T - 1 - s
#pragma unroll
  for (int s = 1; s < T - 1; ++s) {
    const int r = T - 1 - s, W = TX + 2 * r, H = TY + 2 * r, C = W * H, off = RG - r;
    R f[K0][9];
    int at[K0];
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      const int j = tid + k * NTH;
      at[k] = -1;
      if (j >= C) continue;
      const int ly = j / W + off, lx = j % W + off;
      at[k] = ly * W0 + lx;
      gather(f[k], lx, ly);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      if (at[k] < 0) continue;
      const int ly = at[k] / W0, lx = at[k] - ly * W0;
      R m[9], gc[3];
      step(f[k], wrap_once(x0 + lx, nx), wrap_once(y0 + ly, ny), s, m, gc);
      if (own(lx, ly)) add(lx, ly, gc);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[i * C0 + at[k]] = m[i];
    }
    __syncthreads();
  }

  // step T-1: mu and the gradient of the tile's own nodes to memory
  char* ob = (char*)mu_out;
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    const int lx = threadIdx.x + RG, ly = threadIdx.y + k * BY + RG;
    const int32_t x = x0 + lx, y = y0 + ly;
    if (x >= nx || y >= ny) continue;
    R l[9], m[9], gc[3];
    gather(l, lx, ly);
    step(l, x, y, T - 1, m, gc);
    const uint32_t n = __umul24((uint32_t)y, (uint32_t)nx) + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) gst<R, true>(ob + i * pb, n * E, m[i]);
    const int ii = (ly - RG) * TX + (lx - RG);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const Acc s = acc[c * NI + ii];
      if constexpr (F64) {
        store_pop<double, true>(grad + c * N + n, s + inv_kappa * (double)gc[c]);
      } else if (fold) {
        store_pop<double, true>(grad + c * N + n, grad[c * N + n] + inv_kappa * ((double)s + (double)gc[c]));
      } else {
        store_pop<float, true>(part + c * N + n, s + (float)gc[c]);
      }
    }
  }
}

}  // namespace lbm
