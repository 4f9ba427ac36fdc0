// Shared device-side definitions of the gfx950 lattice Boltzmann kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm_cde.h"

#ifndef LBM_FORCEINLINE
#define LBM_FORCEINLINE __device__ __forceinline__
#endif

namespace lbm {

// n / d for n < 2^31 with one multiply-high: m = floor(2^(31+s) / d) + 1,
// s = ceil(log2 d) (s = 0 for d = 1).  For 2^(s-1) < d <= 2^s the error of
// m / 2^(31+s) against 1/d keeps floor(n m / 2^(31+s)) = floor(n / d) for
// every n < 2^31.  Computed on the host; the kernels' tile decompositions
// then need no integer division.
struct FastDiv {
  uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 0u, 0u};
  if (d <= 1) return f;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)(((uint64_t)1 << (31 + s)) / d + 1);
  return f;
}

// Velocity description in the precision R of the arithmetic.
enum UKind : int32_t { U_CONST = 0, U_SEPARABLE = 1, U_FIELD = 2 };

// Compiled for the host and the device alike.
#define LBM_HD __host__ __device__ __forceinline__

// Relaxation coefficients of the D2Q9 collision (Eq. 31) in the precision R
// of the arithmetic; make_rel2_vals computes them.
template <typename R>
struct Rel2 {
  R s1, s2, s7, s8, s4, s6;
  R axx, axy, ayy;
  R c34, c36, c54, c56;  // coupling coefficients of Eq. (31); zero for the standard S (Eq. 24)
  R nl;                  // 1 for the equilibria with u^2 terms (Eq. 38, 39), else 0
  R c2;                  // m2_eq(phi, 0) / phi: 1 for Eq. (38), else 2
  // the rows of S divided by the squared norms of the rows of M (Eq. 12):
  // the collision applies M^-1 = M^T diag(1/|M_k|^2) to S n
  R k1, k2, k4, k6, k7, k8;
  R g33, g34, g35, g36, g53, g54, g55, g56;
  bool lin;  // equilibrium linear in phi and phi u (Eq. 37): no u^2 terms, m2_eq = 2 phi
};

// Everything one kernel launch needs about one run.  Passed by value as a
// kernel argument (and stored in device memory for batched launches).
struct RunArgs {
  const void* src;          // populations read this step  (Q planes)
  void* dst;                // populations written          (Q planes)
  const void* src_phi;      // FP16 split: phi plane read
  void* dst_phi;            // FP16 split: phi plane written
  int64_t nx, ny, nz;
  int64_t plane;            // elements between two population planes
  int32_t bc[3];
  int32_t model;            // LBM_CDE_MRT_A (modified) or an unmodified MRT-B variant
  int32_t u_kind;
  double u_const[3];
  const void* u_tab;        // SEPARABLE: per component: amp, X[nx], Y[ny], Z[nz] (type R)
  int32_t u_z_unit;         // SEPARABLE 2D: Z[0] == 1 exactly for both components
  const double* const* u_slot;  // FIELD: device slot holding the current FP64 field [dim][nodes]
  unsigned* u_flag;         // FIELD: set to 1 where |u| >= c_s = 1/sqrt(3) (sticky)
  const void* node_par;     // per-node relaxation parameters (type R) or null
  int32_t node_heat_const;  // node_par's heat-flux rates equal heat[] at every node (not read)
  double phi_ref;
  double fp16_scale, fp16_inv_scale;
  void* fp16_flags;         // 16-bit storage: set to 1 when a value saturates
  // relaxation (constant D): diagonal rates and the flux block
  double s[15];             // s[k] by moment index (flux-row entries unused)
  double A[3][3];           // flux block s_ab
  double heat[3];           // s4, s6, s8
  // the D2Q9 collision's coefficients for the constant rates above, rounded
  // on the host by the kernels' own formulas (make_rel2_vals), so that a
  // block reads them instead of deriving them again
  Rel2<float> relf;
  Rel2<double> reld;
  // FP16 split storage (MRT-A, constant D), rounded once on the host: the
  // rows of (I - S) times the storage scale over |M_k|^2 (see
  // collide_neq_d2q9) and 1/scale
  float split_g[14];
  float split_inv;
  void* split_dst[9];       // base of each destination half plane (periodic split step)
  int32_t xcd_remap;        // block order (see tile_of_block32)
  FastDiv tiles_x;          // x tiles of the launch's block shape
  FastDiv tiles_y;          // tile rows per z plane (D3Q15)
  int32_t rows32;           // D2Q9 batch: x periodic, constant D, every byte offset < 4 GiB
  int32_t active;           // 0: run has used its step budget
  int64_t max_steps;        // step budget (< 0: unlimited), used by batched launches
  double xref0, xref_drift; // sampled x-moments: x_ref(t) = xref0 + xref_drift * t
};

// Block id remapping for the 8 XCDs of MI355X: consecutive hardware block ids
// go round-robin to the XCDs, so give XCD k the k-th contiguous range of
// logical tiles; neighbouring tiles then share that XCD's L2.
LBM_FORCEINLINE int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t nx = 8;
  const int64_t xcd = b % nx, local = b / nx;
  const int64_t per = nb / nx, rem = nb % nx;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Row-interleaved order: tile row r goes to XCD r mod 8 with all its x-tiles,
// so the cache lines that x-neighbouring tiles share (the x-shifted
// populations) are fetched into one L2.  Needs a multiple of 8 tile rows.
LBM_FORCEINLINE int64_t xcd_rows(int64_t b, int64_t ntx) {
  const int64_t xcd = b % 8, local = b / 8;
  const int64_t tx = local % ntx, group = local / ntx;
  return (group * 8 + xcd) * ntx + tx;
}

// Block order: 0 = hardware order, 1 = XCD-contiguous ranges, 2 = row-interleaved.
LBM_FORCEINLINE int64_t tile_of_block(int64_t b, int64_t nb, int64_t ntx, int mode) {
  if (mode == 1) return xcd_tile(b, nb);
  if (mode == 2) return xcd_rows(b, ntx);
  return b;
}

LBM_FORCEINLINE uint32_t fdiv(uint32_t n, const FastDiv& f) { return f.s == 0 ? n : __umulhi(n, f.m) >> (f.s - 1); }

// tile_of_block in 32 bits with the host's division by the x-tile count.
LBM_FORCEINLINE uint32_t tile_of_block32(uint32_t b, uint32_t nb, const FastDiv& ntx, int mode) {
  if (mode == 1) {
    const uint32_t xcd = b & 7u, local = b >> 3, per = nb >> 3, rem = nb & 7u;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
  }
  if (mode == 2) {
    const uint32_t xcd = b & 7u, local = b >> 3;
    const uint32_t group = fdiv(local, ntx), tx = local - group * ntx.d;
    return (group * 8u + xcd) * ntx.d + tx;
  }
  return b;
}

template <typename R>
LBM_FORCEINLINE R load_ro(const R* p) { return __builtin_nontemporal_load(p); }

// Load / store through a global-address-space base and a 32-bit byte offset
// (the base-plus-offset addressing of the memory instructions).
template <typename T>
LBM_FORCEINLINE T gld(const char* base, uint32_t off) {
  return *(const __attribute__((address_space(1))) T*)(base + off);
}

template <typename T, bool NT>
LBM_FORCEINLINE void gst(char* base, uint32_t off, T v) {
  __attribute__((address_space(1))) T* p = (__attribute__((address_space(1))) T*)(base + off);
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// A per-node velocity read from a FIELD run: flag speeds at or above the
// lattice sound speed (the step is unstable there).
LBM_FORCEINLINE void check_speed(const RunArgs& a, double u2) {
  if (u2 >= 1.0 / 3.0) *a.u_flag = 1u;
}

template <typename R, bool NT>
LBM_FORCEINLINE void store_pop(R* p, R v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Periodic neighbour index.
LBM_FORCEINLINE int64_t wrap_m(int64_t i, int64_t n) { return i == 0 ? n - 1 : i - 1; }
LBM_FORCEINLINE int64_t wrap_p(int64_t i, int64_t n) { return i == n - 1 ? 0 : i + 1; }

}  // namespace lbm
