// Several D2Q9 steps per launch for runs periodic on both axes (temporal
// blocking through LDS).
//
// A population moves at most one node per step (Eq. 5), so the state of an
// output tile T steps later depends only on the stored state within T nodes
// of it.  A block owns a tile of TX x TY output nodes and:
//   step 1      pulls the stored state from HBM for the tile widened by T-1
//               nodes on every side, collides, and keeps the result in LDS;
//   steps 2..T-1 pull from LDS and update it in place over a ring that
//               shrinks by one node per step (all reads, barrier, writes,
//               barrier);
//   step T      pulls from LDS for the tile itself and stores to HBM.
// Every node's step uses the same pull, velocity, relaxation and collision
// arithmetic as the one-step kernel (tile_d2q9 without walls), so T steps of
// this kernel equal T one-step launches bitwise.  It is built for the
// equilibria linear in phi and phi u (MRT-A, Eq. 37, and MRT-B3), whose
// collision has no u^2 terms.  HBM sees one read and one
// write of the state per T steps (72 B per node for FP32, 144 B for FP64)
// instead of per step; the price is the recomputed rings (the widened tiles'
// extra collisions) and LDS traffic.  x is periodic: halo nodes take periodic
// images, which needs nx >= TX + 2(T-1) (one wrap per coordinate).  y is
// periodic the same way (ny >= TY + 2(T-1)) or, with WY, bounded by walls:
// rows beyond a wall are not computed, and a population whose source lies
// beyond it takes the wall rule's source (the node itself or its neighbour
// along or inside the wall, all within one node: row_source_d2q9), from LDS
// in steps 2..T as from memory in step 1.
//
// UK selects the velocity: 0 constant, 1 separable (a product of per-axis
// factors: the block stages the widened tile's column and row factors in LDS
// once and multiplies them in the one-step kernel's order), 2 a per-node
// field (read from memory at every step).  Byte offsets within a population
// plane are 32-bit (nodes * sizeof(R) < 2^32), node coordinates below 2^24
// (row offsets are 24-bit products).
#pragma once

#include "adjoint_d2q9.hpp"
#include "d2q9.hpp"

namespace lbm {

// Velocity components of population i (Eq. 2), in the order of d2q9.hpp.
__device__ constexpr int kEx9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEy9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// v mod n for v in [-n, 2n): of v, v + n and v - n the one in [0, n) is the
// smallest as an unsigned number (the others are n or more, or negative).
LBM_FORCEINLINE int32_t wrap_once(int32_t v, int32_t n) {
  return (int32_t)min(min((uint32_t)v, (uint32_t)(v + n)), (uint32_t)(v - n));
}

// Source of population I (velocity (EX, EY)) at row y: (population, row,
// x shift) under the run's y boundary (walls), as in the one-step kernel.
template <int I>
LBM_FORCEINLINE void wall_source(const RunArgs& a, int32_t y, int32_t ny, int& pop, int32_t& sy, int& dx) {
  constexpr int EX = I == 1 || I == 5 || I == 8 ? 1 : (I == 3 || I == 6 || I == 7 ? -1 : 0);
  constexpr int EY = I == 2 || I == 5 || I == 6 ? 1 : (I == 4 || I == 7 || I == 8 ? -1 : 0);
  row_source_d2q9<EX, EY>(a, y, ny, pop, sy, dx);
}

// T steps of output tile (txi, tyi) of the run described by a; block (BX,
// BY) threads, tile BX x (BY * NY).  With VOUT (the adjoint's forward
// recomputation) every step also stores v = (n3 + s4 n4 / 2, n5 + s6 n6 / 2)
// of the tile's own nodes (adjoint_v; two planes of nx ny values at
// vout + s * vstep bytes for the launch's step s), and the final state goes to
// memory only with store_end.
template <typename R, int BX, int BY, int NY, int T, int UK, bool WY, bool VOUT = false, bool NP = false>
LBM_FORCEINLINE void fused_tile(const RunArgs& a, uint32_t txi, uint32_t tyi, char* vout = nullptr,
                                int64_t vstep = 0, bool store_end = true) {
  static_assert(T >= 2, "one step per launch is k_step_d2q9");
  constexpr int NTH = BX * BY, TX = BX, TY = BY * NY, RG = T - 1;
  constexpr int W0 = TX + 2 * RG, H0 = TY + 2 * RG, C0 = W0 * H0;
  constexpr int K0 = (C0 + NTH - 1) / NTH;
  static_assert(W0 <= NTH && H0 <= NTH, "one thread per staged column and row");
  __shared__ R lds[9 * C0];
  __shared__ R ucol[UK == 1 ? 2 * W0 : 1], urow[UK == 1 ? 2 * H0 : 1];

  const int tid = threadIdx.y * BX + threadIdx.x;
  // the launch's block is BX x BY: the slots below that every thread fills
  // then need no guard, and a slot's collision waits only for its own loads
  // (a guarded slot before it would make the wait cover every load issued)
  if (tid >= NTH) __builtin_unreachable();
  const int32_t nx = (int32_t)a.nx, ny = (int32_t)a.ny;
  const int32_t x0 = (int32_t)txi * TX - RG, y0 = (int32_t)tyi * TY - RG;
  const size_t pb = (size_t)a.plane * sizeof(R);
  const Rel2<R> rc = const_rel2<R>(a);
  const R phi_ref = (R)a.phi_ref;
  // separable velocity: component c at (x, y) is ((t_c[0] t_c[1+x]) t_c[1+nx+y]) t_c[1+nx+ny]
  const R* tab = (const R*)a.u_tab;
  const int32_t tstride = 1 + nx + ny + (int32_t)a.nz;
  R ta0 = (R)0, ta1 = (R)0, tz0 = (R)0, tz1 = (R)0;
  if constexpr (UK == 1) {  // read here, before any store, as scalars
    ta0 = tab[0];
    ta1 = tab[tstride];
    tz0 = tab[1 + nx + ny];
    tz1 = tab[tstride + 1 + nx + ny];
  }

  // row of the widened tile -> row of the grid (periodic image; with walls the
  // row itself, which may lie beyond a wall and is then skipped)
  auto grid_row = [&](int ly) -> int32_t { return WY ? y0 + ly : wrap_once(y0 + ly, ny); };
  auto outside = [&](int32_t y) { return WY && (y < 0 || y >= ny); };
  // LDS gather of the nine populations of local node (lx, ly), grid row y
  auto gather = [&](R(&f)[9], int lx, int ly, int32_t y) {
    // rows 1 .. ny - 2 pull from rows inside the walls: there the wall rule
    // is the plain pull, and only the two rows next to a wall need it
    if (!WY || (y >= 1 && y < ny - 1)) {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = lds[i * C0 + (ly - kEy9[i]) * W0 + (lx - kEx9[i])];
    } else {
#define LBM_FUSED_WALL_PULL(I)                                     \
  {                                                                \
    int pop, dx;                                                   \
    int32_t sy;                                                    \
    wall_source<I>(a, y, ny, pop, sy, dx);                         \
    f[I] = lds[pop * C0 + (ly + (sy - y)) * W0 + (lx + dx)];       \
  }
      LBM_FUSED_WALL_PULL(0)
      LBM_FUSED_WALL_PULL(1)
      LBM_FUSED_WALL_PULL(2)
      LBM_FUSED_WALL_PULL(3)
      LBM_FUSED_WALL_PULL(4)
      LBM_FUSED_WALL_PULL(5)
      LBM_FUSED_WALL_PULL(6)
      LBM_FUSED_WALL_PULL(7)
      LBM_FUSED_WALL_PULL(8)
#undef LBM_FUSED_WALL_PULL
    }
  };

  // v of one node of the tile itself at the launch's step st
  auto store_v = [&](const R(&f)[9], R ux, R uy, const Rel2<R>& rel, int32_t x, int32_t y, int lx, int ly, int st) {
    if constexpr (VOUT) {
      if (lx < RG || lx >= RG + TX || ly < RG || ly >= RG + TY || x0 + lx >= nx || y0 + ly >= ny) return;
      R vx, vy;
      adjoint_v<R>(f, ux, uy, phi_ref, rel, vx, vy);
      const uint32_t o = (__umul24((uint32_t)y, (uint32_t)nx) + x) * (uint32_t)sizeof(R);
      char* vb = vout + st * vstep;
      gst<R, true>(vb, o, vx);
      gst<R, true>(vb + (size_t)nx * ny * sizeof(R), o, vy);
    }
  };
  // collision of one node at periodic image (x, y); (lx, ly) in the widened
  // tile; st = the launch's step
  auto collide = [&](R(&f)[9], int32_t x, int32_t y, int lx, int ly, int st) {
    R ux, uy;
    if constexpr (UK == 0) {
      ux = (R)a.u_const[0];
      uy = (R)a.u_const[1];
    } else if constexpr (UK == 1) {
      ux = (ucol[lx] * urow[ly]) * tz0;
      uy = (ucol[W0 + lx] * urow[H0 + ly]) * tz1;
    } else {
      velocity2<R>(a, x, y, ux, uy);
    }
    if constexpr (NP) {  // per-node relaxation parameters (a D field)
      const Rel2<R> rn = node_rel2<R>(a, (int64_t)y * nx + x);
      store_v(f, ux, uy, rn, x, y, lx, ly, st);
      collide_d2q9<R, 1>(f, ux, uy, phi_ref, rn);
    } else {
      store_v(f, ux, uy, rc, x, y, lx, ly, st);
      collide_d2q9<R, 1>(f, ux, uy, phi_ref, rc);
    }
  };

  // step 1: HBM -> LDS over the whole widened tile
  {
    // the nine source planes as scalar base addresses (as the destination
    // planes of the last step, below)
    const char* spl[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      spl[i] = (const char*)a.src + i * pb;
      asm volatile("" : "+s"(spl[i]));
    }
    const uint32_t rlast = (uint32_t)(ny - 1) * (uint32_t)nx;  // offset of the last row
    R f[K0][9];
    constexpr uint32_t E = sizeof(R);
    // separable velocity: the widened tile's column and row factors are read
    // before the populations and staged in LDS after them, so that the
    // barrier which publishes them waits for these few loads only
    R sc0 = (R)0, sc1 = (R)0, sr0 = (R)0, sr1 = (R)0;
    if constexpr (UK == 1) {
      if (tid < W0) {
        const int32_t x = wrap_once(x0 + tid, nx);
        sc0 = tab[1 + x];
        sc1 = tab[tstride + 1 + x];
      }
      if (tid < H0) {
        // rows beyond a wall are never collided; clamp to stay inside the table
        const int32_t yy = grid_row(tid), y = WY ? (yy < 0 ? 0 : (yy >= ny ? ny - 1 : yy)) : yy;
        sr0 = tab[1 + nx + y];
        sr1 = tab[tstride + 1 + nx + y];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    // the loads of slot k (node tid + k NTH of the widened tile)
    auto load_slot = [&](const int k) {
      const int j = tid + k * NTH;
      if (K0 * NTH > C0 && j >= C0) return;
      const int ly = j / W0, lx = j - ly * W0;
      const int32_t x = wrap_once(x0 + lx, nx), y = grid_row(ly);
      if (outside(y)) return;
      const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x + 1 == nx ? 0 : x + 1;
      if (!WY || (y >= 1 && y < ny - 1)) {  // the plain pull (as in gather)
        const uint32_t r0 = __umul24((uint32_t)y, (uint32_t)nx), rm = y == 0 ? rlast : r0 - nx,
                       rp = y + 1 == ny ? 0u : r0 + nx;
        f[k][0] = gld<R>(spl[0], (r0 + x) * E);
        f[k][1] = gld<R>(spl[1], (r0 + xm) * E);
        f[k][2] = gld<R>(spl[2], (rm + x) * E);
        f[k][3] = gld<R>(spl[3], (r0 + xp) * E);
        f[k][4] = gld<R>(spl[4], (rp + x) * E);
        f[k][5] = gld<R>(spl[5], (rm + xm) * E);
        f[k][6] = gld<R>(spl[6], (rm + xp) * E);
        f[k][7] = gld<R>(spl[7], (rp + xp) * E);
        f[k][8] = gld<R>(spl[8], (rp + xm) * E);
      } else {
#define LBM_FUSED_WALL_LOAD(I)                                                                  \
  {                                                                                             \
    int pop, dx;                                                                                \
    int32_t sy;                                                                                 \
    wall_source<I>(a, y, ny, pop, sy, dx);                                                      \
    const uint32_t sx = dx < 0 ? xm : (dx > 0 ? xp : (uint32_t)x);                              \
    const uint32_t so = (__umul24((uint32_t)sy, (uint32_t)nx) + sx) * E;                        \
    f[k][I] = gld<R>((const char*)a.src + (size_t)pop * pb, so);                                \
  }
        LBM_FUSED_WALL_LOAD(0)
        LBM_FUSED_WALL_LOAD(1)
        LBM_FUSED_WALL_LOAD(2)
        LBM_FUSED_WALL_LOAD(3)
        LBM_FUSED_WALL_LOAD(4)
        LBM_FUSED_WALL_LOAD(5)
        LBM_FUSED_WALL_LOAD(6)
        LBM_FUSED_WALL_LOAD(7)
        LBM_FUSED_WALL_LOAD(8)
#undef LBM_FUSED_WALL_LOAD
      }
    };
    // Issue order: the slot that only some threads fill first, then the full
    // slots in order, each kept together (sched_barrier), so that the wait
    // before slot k's collision covers only the loads issued up to slot k:
    // slot 0 collides while the later slots' loads are still in flight.
    constexpr int KF = C0 / NTH;  // slots that every thread fills
    if constexpr (K0 > KF) load_slot(KF);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      load_slot(k);
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (UK == 1) {
      if (tid < W0) {
        ucol[tid] = ta0 * sc0;
        ucol[W0 + tid] = ta1 * sc1;
      }
      if (tid < H0) {
        urow[tid] = sr0;
        urow[H0 + tid] = sr1;
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      const int j = tid + k * NTH;
      if (K0 * NTH > C0 && j >= C0) continue;
      const int ly = j / W0, lx = j - ly * W0;
      const int32_t y = grid_row(ly);
      if (outside(y)) continue;
      collide(f[k], wrap_once(x0 + lx, nx), y, lx, ly, 0);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[i * C0 + j] = f[k][i];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();

  // steps 2 .. T-1: in place in LDS over the ring of width T - s.  Slot k
  // keeps step 1's node (tid + k NTH of the widened tile), whose coordinates
  // are computed once; a step takes the slots inside its ring.
  int slx[K0], sly[K0];
#pragma unroll
  for (int k = 0; k < K0; ++k) {
    const int j = tid + k * NTH;
    sly[k] = j / W0;
    slx[k] = j - sly[k] * W0;
    if (K0 * NTH > C0 && j >= C0) sly[k] = H0;  // past the tile: in no ring
  }
#pragma unroll
  for (int s = 2; s < T; ++s) {
    const int off = RG - (T - s);  // the ring's first row and column
    R f[K0][9];
    bool in[K0];
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      const int lx = slx[k], ly = sly[k];
      in[k] = (uint32_t)(lx - off) < (uint32_t)(W0 - 2 * off) && (uint32_t)(ly - off) < (uint32_t)(H0 - 2 * off);
      if (!in[k]) continue;
      const int32_t y = grid_row(ly);
      if (outside(y)) {
        in[k] = false;
        continue;
      }
      gather(f[k], lx, ly, y);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K0; ++k) {
      if (!in[k]) continue;
      const int lx = slx[k], ly = sly[k];
      collide(f[k], wrap_once(x0 + lx, nx), grid_row(ly), lx, ly, s - 1);
#pragma unroll
      for (int i = 0; i < 9; ++i) lds[i * C0 + ly * W0 + lx] = f[k][i];
    }
    __syncthreads();
  }

  // step T: LDS -> HBM for the tile's own nodes
  // the nine destination planes as scalar base addresses (the empty asm keeps
  // each in scalar registers and out of the per-node address arithmetic, so
  // a store takes the base-plus-32-bit-offset form with no vector add)
  char* dpl[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    dpl[i] = (char*)a.dst + i * pb;
    asm volatile("" : "+s"(dpl[i]));
  }
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    const int lx = threadIdx.x + RG, ly = threadIdx.y + k * BY + RG;
    const int32_t x = x0 + lx, y = y0 + ly;
    if (x >= nx || y >= ny) continue;
    R g[9];
    gather(g, lx, ly, y);
    collide(g, x, y, lx, ly, T - 1);
    if (VOUT && !store_end) continue;
    const uint32_t off = (__umul24((uint32_t)y, (uint32_t)nx) + x) * (uint32_t)sizeof(R);
#pragma unroll
    for (int i = 0; i < 9; ++i) gst<R, true>(dpl[i], off, g[i]);
  }
}

// One run: one block per tile, in the chosen block order.  NP: the run has
// per-node relaxation parameters (a D field; the branch is resolved at compile
// time, so runs without them pay nothing for it).
template <typename R, int BX, int BY, int NY, int T, int UK, bool WY, bool NP>
__global__ __launch_bounds__(BX * BY) void k_fused_d2q9(const RunArgs a) {
  const uint32_t b = tile_of_block32(blockIdx.x, gridDim.x, a.tiles_x, a.xcd_remap);
  const uint32_t tyi = fdiv(b, a.tiles_x);
  fused_tile<R, BX, BY, NY, T, UK, WY, false, NP>(a, b - tyi * a.tiles_x.d, tyi);
}

// The arguments of one step of a batched run (its compact record), for the
// multi-step tile: what fused_tile reads, in the one-run kernel's form.
template <typename R>
LBM_FORCEINLINE RunArgs batch_run_args(const BatchRun& br, int par) {
  RunArgs a;
  a.src = br.pop[par];
  a.dst = (void*)br.pop[par ^ 1];
  a.nx = br.nx;
  a.ny = br.ny;
  a.nz = 1;
  a.plane = br.pb / (uint32_t)sizeof(R);
  a.bc[0] = LBM_CDE_PERIODIC;
  a.bc[1] = br.bc_y;
  a.bc[2] = LBM_CDE_PERIODIC;
  a.model = br.model;
  a.u_kind = br.u_kind;
  a.u_const[0] = br.u_const[0];
  a.u_const[1] = br.u_const[1];
  a.u_tab = br.u_tab;
  a.node_par = nullptr;
  a.phi_ref = br.phi_ref;
  a.s[1] = br.s1;
  a.s[2] = br.s2;
  a.s[7] = br.s7;
  a.s[8] = br.s8;
  a.A[0][0] = br.axx;
  a.A[0][1] = br.axy;
  a.A[1][1] = br.ayy;
  a.heat[0] = br.s4;
  a.heat[1] = br.s6;
  if constexpr (sizeof(R) == sizeof(float)) a.relf = rel2_of_rates<float>(a);
  else a.reld = rel2_of_rates<double>(a);
  return a;
}

// T steps of every active run of a batch (runs periodic in x, walls or not
// in y, constant or separable velocity) in one launch: block b takes tile b
// of a flat list of BX x (BY * NY) tiles over the runs (in order of
// decreasing budget; blocks past the active runs' tiles exit, and the host
// launches this kernel only while no run's budget ends inside the launch).
// The buffer parity is clock[2], which every launch of a batched kernel
// flips (the one-step kernel's parity, t & 1, equals it between launches of
// this kernel taken in pairs).
template <typename R, int BX, int BY, int NY, int T, int UK, bool WY>
__global__ __launch_bounds__(BX * BY) void k_batch_fused_d2q9(const BatchRun* __restrict__ runs,
                                                             const uint32_t* __restrict__ tile_start, int nruns,
                                                             const int64_t* __restrict__ clock) {
  const uint32_t t = blockIdx.x;
  // active runs: a prefix of the list (runs are stored by decreasing budget)
  const int64_t t_global = clock[0];
  int na;
  {
    int l = 0, h = nruns;
    while (l < h) {
      const int mid = (l + h) / 2;
      const int64_t ms = runs[mid].max_steps;
      if (ms >= 0 && t_global >= ms) h = mid;
      else l = mid + 1;
    }
    na = l;
  }
  if (na == 0 || t >= tile_start[na]) return;
  int lo = 0, hi = na - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (tile_start[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const BatchRun& br = runs[lo];
  const RunArgs a = batch_run_args<R>(br, (int)(clock[2] & 1));
  const uint32_t ntx = (br.nx + BX - 1) / BX, local = t - tile_start[lo];
  const uint32_t tyi = local / ntx;
  fused_tile<R, BX, BY, NY, T, UK, WY>(a, local - tyi * ntx, tyi);
}

}  // namespace lbm
