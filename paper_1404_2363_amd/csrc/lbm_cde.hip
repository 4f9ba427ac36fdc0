// Host runtime and C ABI of the gfx950 modified-MRT lattice Boltzmann solver.
//
// The library owns no device memory: every buffer lives in the caller's
// workspace, laid out per run as
//   [populations A][populations B][velocity tables or field][node params]
//   [reduction partials][reduction result][flags]
// each piece 256-byte aligned.  Populations are structure-of-arrays: plane i
// holds f_i of every node, x fastest, planes `plane` elements apart.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm_cde.h"
#include "aux_kernels.hpp"
#include "common.hpp"
#include "d2q9.hpp"
#include "d3q15.hpp"
#include "adjoint_d2q9.hpp"
#include "fp16_d2q9.hpp"
#include "fused_d2q9.hpp"
#include "adjoint_fused_d2q9.hpp"
#include "stability.hpp"

using namespace lbm;

// Reduction partials of lbm_cde_reduce_noalloc (4 doubles per partial), for
// callers that cannot allocate.  One copy per GPU, held until the process
// ends; host code reaches it only through the address that
// hipGetSymbolAddress returns on that GPU (see scratch_address).
constexpr int64_t kScratchPartials = 32768;     // 1 MiB
constexpr int64_t kNodesPerPartial = 16384;     // nodes reduced into one partial
static __device__ __align__(256) double scratch[4 * kScratchPartials];

namespace {

thread_local std::string g_init_error;

constexpr size_t kAlign = 256;
constexpr int kGraphSteps = 32;   // steps per captured graph (an even number)
constexpr size_t kMaxAdjGraphs = 16;  // captured adjoint-segment parts kept per handle
constexpr int kBatchRedBlocks = 64;  // reduction blocks per run in batched sampling

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Extra bytes between population planes (a multiple of 256).
size_t plane_skew() {
  static const size_t skew = [] {
    if (const char* t = std::getenv("LBM_CDE_PAD")) return align_up((size_t)std::strtoull(t, nullptr, 10));
    return (size_t)16640;  // 16 KiB + 256 B
  }();
  return skew;
}

// A launch variant of the step kernel: tile shape, store kind, block order,
// for the batched persistent launch its number of blocks, and the number of
// steps one launch takes (more than one: the LDS-blocked D2Q9 kernel).
struct Variant {
  int bx, by, ny;
  bool nt;       // non-temporal (streaming) stores
  int xcd;       // block order: 0 hardware, 1 XCD-contiguous ranges, 2 rows interleaved over XCDs
  int grid = 0;  // batched launch: blocks walking the tile list (0: one block per tile)
  int fuse = 1;  // steps per launch
  bool operator==(const Variant& o) const {
    return bx == o.bx && by == o.by && ny == o.ny && nt == o.nt && xcd == o.xcd && grid == o.grid &&
           fuse == o.fuse;
  }
};

struct Run {
  lbm_cde_run_desc d;
  int Q = 9, dim = 2;
  int64_t nodes = 0;
  int64_t plane = 0;            // elements between population planes
  size_t elem = 8;              // bytes per stored population value
  bool dbl = true;              // arithmetic and storage in double
  // workspace pieces
  char* pop[2] = {nullptr, nullptr};
  char* phi[2] = {nullptr, nullptr};   // split 16-bit storage: phi planes
  bool half = false;                   // 16-bit population storage
  bool split = false;                  // ... with phi stored apart
  double fp16_scale = 1.0;
  char* utab = nullptr;
  int32_t u_z_unit = 0;      // SEPARABLE 2D: every component's z factor is exactly 1
  char* ufield = nullptr;    // FP64 copy of the initial velocity field
  char* uslot = nullptr;     // device pointer to the field the steps read
  char* node_par = nullptr;
  double* red_partial = nullptr;
  double* red_out = nullptr;
  unsigned long long* flags = nullptr;
  // derived constants
  double kappa = 1.0 / 3.0;
  double A[3][3] = {{0}};
  double heat[3] = {0, 0, 0};
  double s[15] = {0};
  int64_t steps = 0;
  int cur = 0;         // population buffer (0/1) that holds the current state
  bool walls = false;
  Variant var{256, 1, 1, true, false};
  Variant var1{256, 1, 1, true, false};  // one-step launches (the steps a multi-step variant leaves over)
};

}  // namespace

struct lbm_cde {
  std::vector<Run> runs;
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  bool graph_off = false;  // the runs' steps cannot be replayed from graph[] (odd launch counts)
  std::string err;
  int64_t sample_rows = 0;
  // batched mode: one persistent launch steps every run (same lattice and precision)
  bool batched = false;
  RunArgs* dev_runs = nullptr;       // per-run arguments (parity 0) in the workspace
  int64_t* dev_tiles = nullptr;      // tile_start[nruns + 1] of the flat tile list
  int32_t* dev_order = nullptr;      // run of each tile-list position (decreasing step budget)
  int64_t* dev_clock = nullptr;      // [0] global steps, [1] history rows written
  std::vector<int32_t> batch_order;  // host copy of dev_order
  bool batch_lean = false;           // every run takes the row-tile path: compact records
  BatchRun* dev_brun = nullptr;      // compact records in tile-list order
  uint32_t* dev_tiles32 = nullptr;   // 32-bit tile starts of the compact launch
  double* batch_partial = nullptr;   // reduction partials [nruns][kBatchRedBlocks][3]
  int64_t global_steps = 0;
  Variant batch_var{256, 1, 1, true, 0, 0};  // row-tile width, stores and grid of the batched launch
  int64_t batch_tiles = 0;           // tiles of the flat list at batch_var.bx
  unsigned batch_grid = 0;
  // captured batched steps (and sampled blocks) per launch grid: late in an
  // ensemble the grid shrinks with the active prefix of the tile list
  std::map<unsigned, hipGraphExec_t> batch_graphs, sample_graphs;
  // captured parts of adjoint segments: (run, K, seg, mu, mu_tmp, grad, part)
  std::map<std::tuple<int32_t, int32_t, const void*, const void*, const void*, const void*, int>, hipGraphExec_t>
      adj_graphs;
  std::vector<int64_t> batch_prefix;  // tile-list prefix, in batch order (host copy)
  // several steps per launch for the whole batch (fuse > 1), used for every
  // kGraphSteps block in which no run's budget ends; batch_var steps the rest
  Variant batch_fuse{64, 8, 2, true, 0, 0, 1};
  uint32_t* dev_tiles_f = nullptr;     // tile starts of the multi-step launch, batch order
  std::vector<int64_t> batch_prefix_f; // host copy
  std::map<unsigned, hipGraphExec_t> batch_fgraphs;
  std::map<uint64_t, hipGraphExec_t> sample_fgraphs;
  int64_t sample_every = 0;
  double* sample_hist = nullptr;
  bool env_variant = false;   // LBM_CDE_TILE / _NT / _XCD override every run
  Variant env{256, 1, 1, true, 0};
  Variant env3{128, 1, 1, true, 0};
  bool env16_set = false;     // LBM_CDE_TILE16 = BXxBY[xNT[xORDER]]: split 16-bit launch variant
  Variant env16{64, 4, 1, false, 0};
  double* scratch_dev = nullptr;  // device address of `scratch` on the handle's GPU
  int adj_bx = 256;                // row-tile width of the reverse (adjoint) kernel
  bool adj_nt = true;              // streaming stores in the reverse kernel
};

namespace {

int fail_init(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_init_error = buf;
  return code;
}

int fail(lbm_cde* h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  else g_init_error = buf;
  return code;
}

#define HIP_TRY(h, expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((h), LBM_CDE_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

// ---- parameter derivation (Eq. 36, A.6) -----------------------------------

// Prefactor kappa of D = kappa (I - A/2) A^-1 for the model's alpha1, alpha2.
double kappa_of(int lattice) {
  if (lattice == LBM_CDE_D2Q9) {
    const double a1 = -8.0, a2 = 8.0;             // Eq. (37)
    return 2.0 / 3.0 + a1 / 8.0 + a2 / 12.0;      // Eq. (36)
  }
  const double a1 = -6.0 / 5.0, a2 = 192.0;        // 3D analog of the 2D choice
  return 2.0 / 3.0 + 55.0 * a1 / 54.0 + a2 / 216.0; // Eq. (A.6)
}

void sym_from_components(int dim, const double* c, double M[3][3]) {
  // components xx, yy, zz, xy, xz, yz
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i][j] = 0.0;
  M[0][0] = c[0];
  M[1][1] = c[1];
  M[0][1] = M[1][0] = c[3];
  if (dim == 3) {
    M[2][2] = c[2];
    M[0][2] = M[2][0] = c[4];
    M[1][2] = M[2][1] = c[5];
  }
}

bool is_spd(int dim, double M[3][3]) {
  if (!(M[0][0] > 0.0)) return false;
  const double m2 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
  if (!(m2 > 0.0)) return false;
  if (dim == 2) return true;
  const double m3 = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                    M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                    M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  return m3 > 0.0;
}

void invert(int dim, double B[3][3], double out[3][3]) {
  if (dim == 2) {
    const double det = B[0][0] * B[1][1] - B[0][1] * B[1][0];
    out[0][0] = B[1][1] / det;
    out[1][1] = B[0][0] / det;
    out[0][1] = -B[0][1] / det;
    out[1][0] = -B[1][0] / det;
    return;
  }
  double C[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      C[i][j] = B[i1][j1] * B[i2][j2] - B[i1][j2] * B[i2][j1];
    }
  const double det = B[0][0] * C[0][0] + B[0][1] * C[0][1] + B[0][2] * C[0][2];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[i][j] = C[j][i] / det;
}

// Smallest eigenvalue of a symmetric 2x2 or 3x3 matrix (closed forms; the
// 3x3 one is the trigonometric solution of the characteristic cubic).
double lambda_min(int dim, double M[3][3]) {
  if (dim == 2) {
    const double m = 0.5 * (M[0][0] + M[1][1]), d = 0.5 * (M[0][0] - M[1][1]);
    return m - std::sqrt(d * d + M[0][1] * M[0][1]);
  }
  const double p1 = M[0][1] * M[0][1] + M[0][2] * M[0][2] + M[1][2] * M[1][2];
  const double q = (M[0][0] + M[1][1] + M[2][2]) / 3.0;
  if (p1 == 0.0) return std::min(M[0][0], std::min(M[1][1], M[2][2]));
  const double p2 = (M[0][0] - q) * (M[0][0] - q) + (M[1][1] - q) * (M[1][1] - q) +
                    (M[2][2] - q) * (M[2][2] - q) + 2.0 * p1;
  const double p = std::sqrt(p2 / 6.0);
  double B[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[i][j] = (M[i][j] - (i == j ? q : 0.0)) / p;
  const double detB = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                      B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                      B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
  double r = detB / 2.0;
  r = std::max(-1.0, std::min(1.0, r));
  const double phi = std::acos(r) / 3.0;
  const double pi = 3.14159265358979323846;
  return q + 2.0 * p * std::cos(phi + 2.0 * pi / 3.0);
}

double default_rate(int lattice, int k) {
  if (k == 1 || k == 2) return 1.1;
  if (lattice == LBM_CDE_D2Q9) return (k == 7 || k == 8) ? 1.2 : 0.0;
  return k >= 9 ? 1.2 : 0.0;
}

int validate(const lbm_cde_run_desc& d, int idx) {
  if (d.lattice != LBM_CDE_D2Q9 && d.lattice != LBM_CDE_D3Q15)
    return fail_init(LBM_CDE_EINVAL, "run %d: unknown lattice %d", idx, d.lattice);
  if (d.precision < LBM_CDE_FP64 || d.precision > LBM_CDE_FP16_SHIFTED)
    return fail_init(LBM_CDE_EINVAL, "run %d: unknown precision %d", idx, d.precision);
  if (d.nx < 1 || d.ny < 1 || d.nz < 1)
    return fail_init(LBM_CDE_EINVAL, "run %d: grid %lld x %lld x %lld has an empty axis", idx, (long long)d.nx,
                     (long long)d.ny, (long long)d.nz);
  if (d.lattice == LBM_CDE_D2Q9 && d.nz != 1)
    return fail_init(LBM_CDE_EINVAL, "run %d: D2Q9 needs nz = 1", idx);
  if (d.nx > (1ll << 40) || d.ny > (1ll << 40) || d.nz > (1ll << 40) ||
      (double)d.nx * (double)d.ny * (double)d.nz > 9.0e15)
    return fail_init(LBM_CDE_EINVAL, "run %d: grid too large", idx);
  const int dim = d.lattice == LBM_CDE_D2Q9 ? 2 : 3;
  for (int a = 0; a < dim; ++a)
    if (d.bc[a] < LBM_CDE_PERIODIC || d.bc[a] > LBM_CDE_NODE_MIRROR)
      return fail_init(LBM_CDE_EINVAL, "run %d: unknown boundary kind %d on axis %d", idx, d.bc[a], a);
  if (d.model < LBM_CDE_MRT_A || d.model > LBM_CDE_MRT_B3)
    return fail_init(LBM_CDE_EINVAL, "run %d: unknown collision model %d", idx, d.model);
  int plates = 0, other_walls = 0;
  for (int a = 0; a < dim; ++a) {
    plates += d.bc[a] == LBM_CDE_NODE_MIRROR;
    other_walls += d.bc[a] != LBM_CDE_NODE_MIRROR && d.bc[a] != LBM_CDE_PERIODIC;
  }
  const bool half16 = d.precision == LBM_CDE_FP16_SPLIT || d.precision == LBM_CDE_FP16_SHIFTED;
  if (plates && (d.lattice != LBM_CDE_D2Q9 || plates > 1 || other_walls || half16))
    return fail_init(LBM_CDE_EUNSUPPORTED,
                     "run %d: the on-node plate rule is built for D2Q9, FP64/FP32, on one axis with the other periodic",
                     idx);
  if ((d.bc[0] == LBM_CDE_NODE_MIRROR && d.nx < 2) || (d.bc[1] == LBM_CDE_NODE_MIRROR && d.ny < 2))
    return fail_init(LBM_CDE_EINVAL, "run %d: the plate rule needs at least 2 nodes across", idx);
  if (d.model != LBM_CDE_MRT_A && (d.lattice != LBM_CDE_D2Q9 || half16))
    return fail_init(LBM_CDE_EUNSUPPORTED, "run %d: the unmodified MRT-B models are built for D2Q9, FP64/FP32", idx);
  if (d.u_kind < LBM_CDE_U_CONST || d.u_kind > LBM_CDE_U_FIELD)
    return fail_init(LBM_CDE_EINVAL, "run %d: unknown velocity kind %d", idx, d.u_kind);
  if (d.u_kind == LBM_CDE_U_SEPARABLE && !d.u_tables)
    return fail_init(LBM_CDE_EINVAL, "run %d: separable velocity without tables", idx);
  if (d.u_kind == LBM_CDE_U_FIELD && !d.u_field)
    return fail_init(LBM_CDE_EINVAL, "run %d: velocity field pointer is NULL", idx);
  if (d.heat_rule < LBM_CDE_HEAT_LAMBDA_MIN || d.heat_rule > LBM_CDE_HEAT_EXPLICIT)
    return fail_init(LBM_CDE_EINVAL, "run %d: unknown heat-flux rate rule %d", idx, d.heat_rule);
  if (!std::isfinite(d.phi_ref)) return fail_init(LBM_CDE_EINVAL, "run %d: phi_ref is not finite", idx);
  const bool half = d.precision == LBM_CDE_FP16_SPLIT || d.precision == LBM_CDE_FP16_SHIFTED;
  if (half && d.lattice == LBM_CDE_D3Q15)
    return fail_init(LBM_CDE_EUNSUPPORTED, "run %d: 16-bit storage is built for D2Q9 only", idx);
  if (half && (d.D_field || d.u_kind == LBM_CDE_U_FIELD))
    return fail_init(LBM_CDE_EUNSUPPORTED, "run %d: 16-bit storage needs constant D and a constant or separable u",
                     idx);
  if (half && (d.fp16_scale < 0.0 || !std::isfinite(d.fp16_scale)))
    return fail_init(LBM_CDE_EINVAL, "run %d: fp16_scale must be >= 0", idx);
  if (d.lattice == LBM_CDE_D3Q15 && d.D_field)
    return fail_init(LBM_CDE_EUNSUPPORTED, "run %d: per-node D fields are built for D2Q9 only", idx);
  return LBM_CDE_OK;
}

// Derive A, heat rates and diagonal rates of a run with constant D.
int derive(Run& r, int idx) {
  const lbm_cde_run_desc& d = r.d;
  r.kappa = kappa_of(d.lattice);
  for (int k = 0; k < 15; ++k) {
    const double v = d.rates[k] != 0.0 ? d.rates[k] : default_rate(d.lattice, k);
    r.s[k] = v;
  }
  static const int used2[] = {1, 2, 7, 8, -1, -1, -1, -1, -1};
  static const int used3[] = {1, 2, 9, 10, 11, 12, 13, 14, -1};
  const int* used = d.lattice == LBM_CDE_D2Q9 ? used2 : used3;
  for (int j = 0; j < 9 && used[j] >= 0; ++j) {
    const double v = r.s[used[j]];
    if (!(v > 0.0 && v < 2.0))
      return fail_init(LBM_CDE_EUNSTABLE, "run %d: rate s%d = %g outside (0, 2)", idx, used[j], v);
  }
  if (d.heat_rule == LBM_CDE_HEAT_EXPLICIT)
    for (int a = 0; a < r.dim; ++a)
      if (!(d.heat_rates[a] > 0.0 && d.heat_rates[a] < 2.0))
        return fail_init(LBM_CDE_EUNSTABLE, "run %d: heat-flux rate %g outside (0, 2)", idx, d.heat_rates[a]);
  if (d.D_field) {
    for (int a = 0; a < 3; ++a) r.heat[a] = d.heat_rates[a];
    return LBM_CDE_OK;  // A per node, derived on the GPU
  }
  double D[3][3], B[3][3];
  sym_from_components(r.dim, d.D, D);
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(d.D[i])) return fail_init(LBM_CDE_EINVAL, "run %d: D has a non-finite entry", idx);
  if (!is_spd(r.dim, D)) return fail_init(LBM_CDE_ENOTSPD, "run %d: D is not symmetric positive definite", idx);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[i][j] = D[i][j] / r.kappa + (i == j ? 0.5 : 0.0);
  invert(r.dim, B, r.A);
  const double lmin = lambda_min(r.dim, r.A);
  for (int a = 0; a < r.dim; ++a) {
    if (d.heat_rule == LBM_CDE_HEAT_LAMBDA_MIN) r.heat[a] = lmin;
    else if (d.heat_rule == LBM_CDE_HEAT_PAPER) r.heat[a] = r.A[a][a];
    else r.heat[a] = d.heat_rates[a];
    if (!(r.heat[a] > 0.0 && r.heat[a] < 2.0))
      return fail_init(LBM_CDE_EUNSTABLE, "run %d: heat-flux rate %g outside (0, 2)", idx, r.heat[a]);
  }
  return LBM_CDE_OK;
}

// |u| < c_s check for constant and separable velocities (a bound for the latter).
int check_velocity(const Run& r, int idx) {
  const lbm_cde_run_desc& d = r.d;
  double bound2 = 0.0;
  if (d.u_kind == LBM_CDE_U_CONST) {
    for (int c = 0; c < r.dim; ++c) {
      if (!std::isfinite(d.u_const[c])) return fail_init(LBM_CDE_EINVAL, "run %d: u is not finite", idx);
      bound2 += d.u_const[c] * d.u_const[c];
    }
  } else if (d.u_kind == LBM_CDE_U_SEPARABLE) {
    const int64_t stride = 1 + d.nx + d.ny + d.nz;
    for (int c = 0; c < r.dim; ++c) {
      const double* t = d.u_tables + c * stride;
      double mx[3] = {0, 0, 0};
      const int64_t len[3] = {d.nx, d.ny, d.nz};
      const double* seg = t + 1;
      for (int a = 0; a < 3; ++a) {
        for (int64_t i = 0; i < len[a]; ++i) {
          if (!std::isfinite(seg[i])) return fail_init(LBM_CDE_EINVAL, "run %d: u table not finite", idx);
          mx[a] = std::max(mx[a], std::fabs(seg[i]));
        }
        seg += len[a];
      }
      const double b = std::fabs(t[0]) * mx[0] * mx[1] * mx[2];
      bound2 += b * b;
    }
  } else {
    return LBM_CDE_OK;  // per-node field: not checked
  }
  if (!(std::sqrt(bound2) < 1.0 / std::sqrt(3.0)))
    return fail_init(LBM_CDE_EUNSTABLE, "run %d: |u| reaches the lattice sound speed 1/sqrt(3)", idx);
  return LBM_CDE_OK;
}

// The relaxation matrix S of a run with constant D, row-major Q x Q: Eq. (31)
// / (A.5) for MRT-A, Eq. (24) for the MRT-B models.
void relaxation_matrix_of(const Run& r, double* S) {
  const int Q = r.Q;
  for (int i = 0; i < Q * Q; ++i) S[i] = 0.0;
  const int flux[3] = {3, 5, 7}, heatrow[3] = {4, 6, 8};
  for (int k = 0; k < Q; ++k) S[k * Q + k] = r.s[k];
  for (int a = 0; a < r.dim; ++a) S[heatrow[a] * Q + heatrow[a]] = r.heat[a];
  for (int a = 0; a < r.dim; ++a)
    for (int b = 0; b < r.dim; ++b) {
      S[flux[a] * Q + flux[b]] = r.A[a][b];
      if (r.d.model == LBM_CDE_MRT_A)  // the coupling of Eq. (31); Eq. (24) has none
        S[flux[a] * Q + heatrow[b]] = (a == b ? r.A[a][b] / 2.0 - 1.0 : r.A[a][b] / 2.0) * r.heat[b];
    }
}

// Upper bound of the spectral radius of the linearised step of a run with
// constant D and u (a 48^2 or 10^3 k-grid), remembered per parameter set.
double spectral_radius_of(const Run& r) {
  static std::mutex mu;
  static std::map<std::string, double> cache;
  double S[225];
  relaxation_matrix_of(r, S);
  std::string key = std::to_string(r.d.lattice) + ":" + std::to_string(r.d.model);
  char buf[32];
  for (int i = 0; i < r.Q * r.Q; ++i) {
    std::snprintf(buf, sizeof buf, ":%a", S[i]);
    key += buf;
  }
  for (int c = 0; c < r.dim; ++c) {
    std::snprintf(buf, sizeof buf, ":%a", r.d.u_const[c]);
    key += buf;
  }
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const double u[3] = {r.d.u_const[0], r.d.u_const[1], r.dim == 3 ? r.d.u_const[2] : 0.0};
  const double rho = stability::spectral_radius(r.d.lattice, r.d.model, S, u, r.dim == 2 ? 48 : 10);
  std::lock_guard<std::mutex> lock(mu);
  cache[key] = rho;
  return rho;
}

constexpr double kStabilityTol = 1e-5;  // accepted excess of the spectral-radius bound over 1

// Linear stability of a run with constant D and u (unless the descriptor
// asks to skip the check): EUNSTABLE if a Fourier mode grows.
int check_stability(const Run& r, int idx) {
  if (r.d.D_field || r.d.u_kind != LBM_CDE_U_CONST || r.d.skip_stability_check) return LBM_CDE_OK;
  const double rho = spectral_radius_of(r);
  if (rho > 1.0 + kStabilityTol)
    return fail_init(LBM_CDE_EUNSTABLE,
                     "run %d: the linearised step amplifies a Fourier mode by up to %.6f per step (the heat-flux "
                     "rates, D and u give a spectral radius above 1)",
                     idx, rho);
  return LBM_CDE_OK;
}

// Workspace layout of one run; with base == nullptr only sizes are computed.
size_t layout(Run& r, char* base) {
  const lbm_cde_run_desc& d = r.d;
  r.dim = d.lattice == LBM_CDE_D2Q9 ? 2 : 3;
  r.Q = d.lattice == LBM_CDE_D2Q9 ? 9 : 15;
  r.dbl = d.precision == LBM_CDE_FP64;
  r.half = d.precision == LBM_CDE_FP16_SPLIT || d.precision == LBM_CDE_FP16_SHIFTED;
  r.split = d.precision == LBM_CDE_FP16_SPLIT;
  r.elem = r.dbl ? 8 : (r.half ? 2 : 4);
  r.nodes = d.nx * d.ny * d.nz;
  // planes padded to a multiple of 256 bytes plus a skew, so that the same
  // node of consecutive planes does not fall on the same HBM channel and bank
  r.plane = (int64_t)((align_up((size_t)r.nodes * r.elem) + plane_skew()) / r.elem);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const size_t popbytes = (size_t)r.plane * r.elem * r.Q;
  r.pop[0] = take(popbytes);
  r.pop[1] = take(popbytes);
  r.phi[0] = r.phi[1] = nullptr;
  if (r.split) {
    r.phi[0] = take(sizeof(float) * (size_t)r.nodes);
    r.phi[1] = take(sizeof(float) * (size_t)r.nodes);
  }
  r.utab = nullptr;
  r.ufield = nullptr;
  r.uslot = nullptr;
  r.node_par = nullptr;
  const size_t relem = r.dbl ? 8 : 4;  // arithmetic precision of tables and parameters
  if (d.u_kind == LBM_CDE_U_SEPARABLE) r.utab = take((size_t)r.dim * (1 + d.nx + d.ny + d.nz) * relem);
  if (d.u_kind == LBM_CDE_U_FIELD) {
    r.ufield = take((size_t)r.dim * r.nodes * sizeof(double));
    r.uslot = take(sizeof(double*));
  }
  if (d.D_field) r.node_par = take((size_t)(r.dim == 2 ? 5 : 9) * r.nodes * relem);
  r.red_partial = (double*)take(sizeof(double) * 4 * RED_BLOCKS);
  r.red_out = (double*)take(sizeof(double) * 4);
  r.flags = (unsigned long long*)take(sizeof(unsigned long long) * 4);
  return off;
}

// Number of tile rows of a launch (y tiles times z planes).
int64_t tile_rows(const Run& r, const Variant& v) {
  return (r.d.ny + (int64_t)v.by * v.ny - 1) / ((int64_t)v.by * v.ny) * r.d.nz;
}

// Bytes of one state: the population planes (and, split storage, phi).
size_t state_size(const Run& r) {
  const size_t pb = (size_t)r.Q * r.plane * r.elem;
  return r.split ? align_up(pb) + sizeof(float) * r.nodes : pb;
}

RunArgs make_args(const lbm_cde* h, const Run& r, int parity, const Variant* launch = nullptr) {
  const Variant& var = launch ? *launch : r.var;
  RunArgs a;
  std::memset(&a, 0, sizeof a);
  a.src = r.pop[parity];
  a.dst = r.pop[parity ^ 1];
  a.src_phi = r.phi[parity];
  a.dst_phi = r.phi[parity ^ 1];
  a.fp16_scale = r.half ? r.fp16_scale : 1.0;
  a.fp16_inv_scale = r.half ? 1.0 / r.fp16_scale : 1.0;
  a.split_inv = (float)a.fp16_inv_scale;
  if (r.half && a.dst)
    for (int i = 0; i < 9; ++i) a.split_dst[i] = (char*)a.dst + (size_t)i * (size_t)r.plane * 2u;
  a.fp16_flags = r.flags ? (void*)&r.flags[1] : nullptr;
  a.nx = r.d.nx;
  a.ny = r.d.ny;
  a.nz = r.d.nz;
  a.plane = r.plane;
  for (int i = 0; i < 3; ++i) a.bc[i] = r.d.bc[i];
  a.model = r.d.model;
  a.u_kind = r.d.u_kind;
  for (int i = 0; i < 3; ++i) a.u_const[i] = r.d.u_const[i];
  a.u_tab = r.utab;
  a.u_z_unit = r.u_z_unit;
  a.u_slot = (const double* const*)r.uslot;
  a.u_flag = r.flags ? (unsigned*)&r.flags[2] : nullptr;
  a.node_par = r.node_par;
  a.node_heat_const = r.node_par && r.d.heat_rule == LBM_CDE_HEAT_EXPLICIT;
  a.phi_ref = (r.dbl || r.split) ? 0.0 : r.d.phi_ref;
  for (int k = 0; k < 15; ++k) a.s[k] = r.s[k];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a.A[i][j] = r.A[i][j];
  for (int i = 0; i < 3; ++i) a.heat[i] = r.heat[i];
  a.relf = rel2_of_rates<float>(a);
  a.reld = rel2_of_rates<double>(a);
  if (r.split) {
    // rows of (I - S) of MRT-A (Eq. 31) times scale / |M_k|^2, in FP64, rounded once
    const double sc = a.fp16_scale, k36 = sc / 36.0, k12 = sc / 12.0, k6 = sc / 6.0, k4 = sc / 4.0;
    const double s4 = r.heat[0], s6 = r.heat[1];
    const double axx = r.A[0][0], axy = r.A[0][1], ayy = r.A[1][1];
    const double c34 = (axx * 0.5 - 1.0) * s4, c36 = (axy * 0.5) * s6;
    const double c54 = (axy * 0.5) * s4, c56 = (ayy * 0.5 - 1.0) * s6;
    const double g[14] = {(1.0 - r.s[1]) * k36, (1.0 - r.s[2]) * k36, (1.0 - s4) * k12, (1.0 - s6) * k12,
                          (1.0 - r.s[7]) * k4,  (1.0 - r.s[8]) * k4,  (1.0 - axx) * k6, -c34 * k6,
                          -axy * k6,            -c36 * k6,            -axy * k6,        -c54 * k6,
                          (1.0 - ayy) * k6,     -c56 * k6};
    for (int i = 0; i < 14; ++i) a.split_g[i] = (float)g[i];
  }
  a.max_steps = r.d.max_steps;
  a.xref0 = r.d.xref0;
  a.xref_drift = r.d.xref_drift;
  a.xcd_remap = var.xcd;
  // tile counts of the launch's block shape (16-bit runs: the split kernels
  // tile BX x BY nodes; the literal kernel 256 x 1)
  const int64_t tbx = r.half && !r.split ? 256 : var.bx;
  const int64_t tby = r.half && !r.split ? 1 : (int64_t)var.by * (r.half ? 1 : var.ny);
  a.tiles_x = make_fastdiv((uint32_t)((r.d.nx + tbx - 1) / tbx));
  a.tiles_y = make_fastdiv((uint32_t)((r.d.ny + tby - 1) / tby));
  a.rows32 = r.d.lattice == LBM_CDE_D2Q9 && !r.half && r.d.bc[0] == LBM_CDE_PERIODIC && !r.node_par &&
             (double)r.plane * r.Q * r.elem < 4294967296.0 && r.d.nx < (1ll << 31) && r.d.ny < (1ll << 31) &&
             (r.d.u_kind != LBM_CDE_U_FIELD || 16.0 * (double)r.nodes < 4294967296.0);
  if (a.xcd_remap == 2 && tile_rows(r, var) % 8 != 0) a.xcd_remap = 0;
  a.active = 1;
  return a;
}

// A batch of runs is stepped by one persistent launch when every run is D2Q9
// in the same FP64 or FP32 precision.
bool batch_eligible(const lbm_cde_run_desc* runs, int32_t nruns) {
  if (nruns < 2) return false;
  for (int i = 0; i < nruns; ++i)
    if (runs[i].lattice != LBM_CDE_D2Q9 || runs[i].precision != runs[0].precision ||
        runs[i].precision == LBM_CDE_FP16_SPLIT || runs[i].precision == LBM_CDE_FP16_SHIFTED)
      return false;
  return true;
}

size_t batch_bytes(int32_t nruns) {
  return align_up(sizeof(RunArgs) * nruns) + align_up(sizeof(int64_t) * (nruns + 1)) +
         align_up(sizeof(int32_t) * nruns) + align_up(3 * sizeof(int64_t)) +
         align_up(sizeof(double) * 3 * kBatchRedBlocks * nruns) + align_up(sizeof(BatchRun) * nruns) +
         2 * align_up(sizeof(uint32_t) * (nruns + 1));
}

// ---- kernel dispatch ------------------------------------------------------

// Default launch variants, from sweeps on MI355X: wide one-row tiles with
// streaming stores and the hardware's round-robin XCD order were fastest
// (the XCD-contiguous remap was 5-10% slower on 4096^2 D2Q9).
Variant default_variant(int lattice, int precision) {
  if (lattice == LBM_CDE_D3Q15) return Variant{128, 1, 1, true, 0};
  if (precision == LBM_CDE_FP16_SPLIT) return Variant{128, 4, 1, false, 0};
  if (precision == LBM_CDE_FP16_SHIFTED) return Variant{256, 1, 1, false, 0};
  return precision == LBM_CDE_FP64 ? Variant{128, 2, 1, true, 0} : Variant{256, 1, 1, true, 0};
}

using StepFn = void (*)(const RunArgs, hipStream_t);

template <typename R, int BX, int BY, int NY, bool WALLS, bool NT>
void launch_d2q9(const RunArgs a, hipStream_t s) {
  const int64_t ntx = (a.nx + BX - 1) / BX;
  const int64_t nty = (a.ny + BY * NY - 1) / (BY * NY);
  hipLaunchKernelGGL((k_step_d2q9<R, BX, BY, NY, WALLS, NT>), dim3((unsigned)(ntx * nty)), dim3(BX, BY), 0, s, a);
}

template <typename R, int BX, int BY, int NY, bool WALLS, bool NT>
void launch_d3q15(const RunArgs a, hipStream_t s) {
  const int64_t ntx = (a.nx + BX - 1) / BX;
  const int64_t nty = (a.ny + BY * NY - 1) / (BY * NY);
  hipLaunchKernelGGL((k_step_d3q15<R, BX, BY, NY, WALLS, NT>), dim3((unsigned)(ntx * nty * a.nz)), dim3(BX, BY), 0,
                     s, a);
}

struct Step3Entry {
  int bx, by, ny;
  bool nt;
  StepFn fn[2][2];
};

#define STEP3_ENTRY(BX, BY, NY, NT)                                                      \
  Step3Entry {                                                                           \
    BX, BY, NY, NT, {                                                                    \
      {launch_d3q15<float, BX, BY, NY, false, NT>, launch_d3q15<float, BX, BY, NY, true, NT>}, \
      {launch_d3q15<double, BX, BY, NY, false, NT>, launch_d3q15<double, BX, BY, NY, true, NT>} \
    }                                                                                    \
  }

const Step3Entry kSteps3[] = {
    STEP3_ENTRY(64, 4, 1, false), STEP3_ENTRY(128, 2, 1, false), STEP3_ENTRY(256, 1, 1, false),
    STEP3_ENTRY(64, 2, 2, false), STEP3_ENTRY(128, 1, 1, false), STEP3_ENTRY(64, 4, 1, true),
    STEP3_ENTRY(128, 2, 1, true), STEP3_ENTRY(256, 1, 1, true), STEP3_ENTRY(64, 2, 2, true),
    STEP3_ENTRY(128, 1, 1, true),
};

struct StepEntry {
  int bx, by, ny;
  bool nt;
  StepFn fn[2][2];  // [double?][walls?]
};

#define STEP_ENTRY(BX, BY, NY, NT)                                                     \
  StepEntry {                                                                          \
    BX, BY, NY, NT, {                                                                  \
      {launch_d2q9<float, BX, BY, NY, false, NT>, launch_d2q9<float, BX, BY, NY, true, NT>}, \
      {launch_d2q9<double, BX, BY, NY, false, NT>, launch_d2q9<double, BX, BY, NY, true, NT>} \
    }                                                                                  \
  }

const StepEntry kSteps[] = {
    STEP_ENTRY(64, 4, 1, false),  STEP_ENTRY(64, 4, 2, false),  STEP_ENTRY(128, 2, 1, false),
    STEP_ENTRY(256, 1, 1, false), STEP_ENTRY(256, 1, 2, false), STEP_ENTRY(64, 2, 4, false),
    STEP_ENTRY(128, 2, 2, false), STEP_ENTRY(512, 1, 1, false), STEP_ENTRY(128, 1, 1, false),
    STEP_ENTRY(64, 4, 1, true),   STEP_ENTRY(64, 4, 2, true),   STEP_ENTRY(128, 2, 1, true),
    STEP_ENTRY(256, 1, 1, true),  STEP_ENTRY(256, 1, 2, true),  STEP_ENTRY(64, 2, 4, true),
    STEP_ENTRY(128, 2, 2, true),  STEP_ENTRY(512, 1, 1, true),  STEP_ENTRY(128, 1, 1, true),
};

// A periodic split run takes the 32-bit-offset kernel when its grid covers a
// tile and every byte offset (phi plane, nine half planes) fits 32 bits.
bool split_fast_ok(const RunArgs& a, int bx, int by) {
  return a.nx >= bx && a.ny >= by && 4 * a.nx * a.ny < (1ll << 32) && 18 * a.plane < (1ll << 32);
}

template <int BX, int BY, bool WALLS, bool NT>
void launch_split(const RunArgs a, hipStream_t s) {
  const int64_t ntx = (a.nx + BX - 1) / BX, nty = (a.ny + BY - 1) / BY;
  if (!WALLS && split_fast_ok(a, BX, BY)) {
    const dim3 g((unsigned)(ntx * nty)), b(BX, BY);
    if (a.u_kind == U_CONST)
      hipLaunchKernelGGL((k_step_d2q9_split_p<BX, BY, NT, 0>), g, b, 0, s, a, (unsigned*)a.fp16_flags);
    else if (a.u_z_unit)
      hipLaunchKernelGGL((k_step_d2q9_split_p<BX, BY, NT, 2>), g, b, 0, s, a, (unsigned*)a.fp16_flags);
    else
      hipLaunchKernelGGL((k_step_d2q9_split_p<BX, BY, NT, 1>), g, b, 0, s, a, (unsigned*)a.fp16_flags);
  }
  else
    hipLaunchKernelGGL((k_step_d2q9_split<BX, BY, WALLS>), dim3((unsigned)(ntx * nty)), dim3(BX, BY), 0, s, a,
                       (unsigned*)a.fp16_flags);
}

template <bool WALLS>
void launch_half(const RunArgs a, hipStream_t s) {
  const int64_t ntx = (a.nx + 255) / 256;
  hipLaunchKernelGGL((k_step_d2q9_half<256, WALLS>), dim3((unsigned)(ntx * a.ny)), dim3(256), 0, s, a,
                     (unsigned*)a.fp16_flags);
}

struct SplitEntry {
  int bx, by;
  StepFn fn[2][2];  // [walls?][streaming stores? (periodic kernel only)]
};
#define SPLIT_ENTRY(BX, BY)                                                                 \
  SplitEntry {                                                                              \
    BX, BY, {{launch_split<BX, BY, false, false>, launch_split<BX, BY, false, true>},       \
             {launch_split<BX, BY, true, false>, launch_split<BX, BY, true, false>}}        \
  }
const SplitEntry kSplit[] = {SPLIT_ENTRY(64, 4), SPLIT_ENTRY(128, 2), SPLIT_ENTRY(256, 1), SPLIT_ENTRY(64, 8),
                             SPLIT_ENTRY(128, 4), SPLIT_ENTRY(256, 2)};


// Several steps per launch (fused_d2q9.hpp): D2Q9 in FP64 or FP32, periodic
// on both axes, streaming stores; tile BX x (BY * NY) nodes; the velocity
// kind is a template argument.  A shape whose LDS (nine planes of the tile
// widened by T - 1 nodes on every side) would exceed the 160 KiB of a CU is
// not built for that precision.
template <typename R, int BX, int BY, int NY, int T>
void launch_fused(const RunArgs a, hipStream_t s) {
  const int64_t ntx = (a.nx + BX - 1) / BX, nty = (a.ny + BY * NY - 1) / (BY * NY);
  const dim3 g((unsigned)(ntx * nty)), b(BX, BY);
  if (a.node_par) {  // a D field (periodic, velocity constant or separable: fused_ok)
    if (a.u_kind == U_CONST) hipLaunchKernelGGL((k_fused_d2q9<R, BX, BY, NY, T, 0, false, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_fused_d2q9<R, BX, BY, NY, T, 1, false, true>), g, b, 0, s, a);
  } else if (a.bc[1] != LBM_CDE_PERIODIC) {  // walls in y (velocity constant or separable)
    if (a.u_kind == U_CONST) hipLaunchKernelGGL((k_fused_d2q9<R, BX, BY, NY, T, 0, true, false>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_fused_d2q9<R, BX, BY, NY, T, 1, true, false>), g, b, 0, s, a);
  } else if (a.u_kind == U_CONST) {
    hipLaunchKernelGGL((k_fused_d2q9<R, BX, BY, NY, T, 0, false, false>), g, b, 0, s, a);
  } else if (a.u_kind == U_SEPARABLE) {
    hipLaunchKernelGGL((k_fused_d2q9<R, BX, BY, NY, T, 1, false, false>), g, b, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_fused_d2q9<R, BX, BY, NY, T, 2, false, false>), g, b, 0, s, a);
  }
}

template <typename R, int BX, int BY, int NY, int T>
constexpr StepFn fused_fn() {
  if constexpr (9 * (BX + 2 * (T - 1)) * (BY * NY + 2 * (T - 1)) * sizeof(R) <= 160 * 1024)
    return launch_fused<R, BX, BY, NY, T>;
  else
    return nullptr;
}

struct FusedEntry {
  int bx, by, ny, T;
  StepFn fn[2];  // [double?]
};
#define FUSED_ENTRY(BX, BY, NY, T) \
  FusedEntry { BX, BY, NY, T, {fused_fn<float, BX, BY, NY, T>(), fused_fn<double, BX, BY, NY, T>()} }
const FusedEntry kFused[] = {FUSED_ENTRY(128, 4, 2, 2), FUSED_ENTRY(128, 4, 2, 3), FUSED_ENTRY(128, 4, 2, 4),
                             FUSED_ENTRY(128, 4, 2, 5), FUSED_ENTRY(64, 4, 2, 3),  FUSED_ENTRY(64, 4, 2, 4),
                             FUSED_ENTRY(64, 8, 2, 3),  FUSED_ENTRY(64, 8, 2, 4),  FUSED_ENTRY(64, 8, 2, 5),
                             FUSED_ENTRY(64, 8, 3, 4),  FUSED_ENTRY(64, 12, 2, 4)};

// A run can take T steps per launch when it is D2Q9 in FP64 or FP32 with an
// equilibrium linear in phi and phi u (MRT-A or MRT-B3), periodic in x, each
// periodic axis spans the tile plus T - 1 nodes on both sides (halo nodes are
// periodic images taken with one wrap), a run with walls in y or a D field
// (per-node rates, periodic only) has a constant or separable velocity,
// byte offsets within a population plane fit 32 bits and node coordinates 24
// bits (row offsets are 24-bit products).
bool fused_ok(const Run& r, const Variant& v) {
  const bool wy = r.d.bc[1] != LBM_CDE_PERIODIC;
  return r.d.lattice == LBM_CDE_D2Q9 && !r.half && !r.split && r.d.bc[0] == LBM_CDE_PERIODIC && r.d.nz == 1 &&
         (r.d.model == LBM_CDE_MRT_A || r.d.model == LBM_CDE_MRT_B3) && !(wy && r.d.u_kind == LBM_CDE_U_FIELD) &&
         !(r.node_par && (wy || r.d.u_kind == LBM_CDE_U_FIELD)) &&
         r.d.nx >= (int64_t)v.bx + 2 * (v.fuse - 1) && (wy || r.d.ny >= (int64_t)v.by * v.ny + 2 * (v.fuse - 1)) &&
         (double)r.nodes * (double)r.elem < 4294967296.0 && r.d.nx < (1ll << 24) && r.d.ny < (1ll << 24) &&
         v.grid == 0;
}

StepFn find_step(const Run& r, const Variant& v) {
  const int p = r.dbl ? 1 : 0, w = r.walls ? 1 : 0;
  if (v.fuse != 1) {
    if (v.fuse < 2 || !v.nt || !fused_ok(r, v)) return nullptr;
    for (const auto& e : kFused)
      if (e.bx == v.bx && e.by == v.by && e.ny == v.ny && e.T == v.fuse) return e.fn[p];
    return nullptr;
  }
  if (r.split) {
    for (const auto& e : kSplit)
      if (e.bx == v.bx && e.by == v.by && v.ny == 1) return e.fn[w][v.nt && !r.walls ? 1 : 0];
    return nullptr;
  }
  if (r.half) return (v.bx == 256 && v.by == 1 && v.ny == 1) ? (r.walls ? launch_half<true> : launch_half<false>)
                                                             : nullptr;
  if (r.d.lattice == LBM_CDE_D3Q15) {
    for (const auto& e : kSteps3)
      if (e.bx == v.bx && e.by == v.by && e.ny == v.ny && e.nt == v.nt) return e.fn[p][w];
    return nullptr;
  }
  for (const auto& e : kSteps)
    if (e.bx == v.bx && e.by == v.by && e.ny == v.ny && e.nt == v.nt) return e.fn[p][w];
  return nullptr;
}

// One launch of variant v (validated when it was set) on run r: reads buffer
// cur, writes the other, advances the run by v.fuse steps.
void launch_variant(lbm_cde* h, Run& r, const Variant& v, hipStream_t s) {
  find_step(r, v)(make_args(h, r, r.cur, &v), s);
  r.cur ^= 1;
  r.steps += v.fuse;
}

// Enqueue n steps of run r (fewer where its budget ends first): launches of
// its variant while they fit, one-step launches for the rest.  With `even`,
// one multi-step launch is traded for one-step launches where that makes the
// number of launches even (a captured graph must leave the state in the
// buffer it started from).  Returns the number of launches.
int64_t enqueue_run(lbm_cde* h, Run& r, int64_t n, hipStream_t s, bool even = false) {
  if (r.d.max_steps >= 0) n = std::min<int64_t>(n, std::max<int64_t>(r.d.max_steps - r.steps, 0));
  const int T = r.var.fuse;
  int64_t q = T > 1 ? n / T : 0, rest = n - q * T;
  if (even && T > 1 && q > 0 && ((q + rest) & 1)) {
    q -= 1;
    rest += T;
  }
  for (int64_t k = 0; k < q; ++k) launch_variant(h, r, r.var, s);
  const Variant& v1 = T > 1 ? r.var1 : r.var;
  for (int64_t k = 0; k < rest; ++k) launch_variant(h, r, v1, s);
  return q + rest;
}

int launch_steps(lbm_cde* h, hipStream_t s, int64_t n) {
  for (auto& r : h->runs) enqueue_run(h, r, n, s);
  HIP_TRY(h, hipGetLastError());
  return LBM_CDE_OK;
}

void drop_graphs(lbm_cde* h) {
  for (auto& g : h->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  h->graph_off = false;
  for (auto* m : {&h->batch_graphs, &h->sample_graphs, &h->batch_fgraphs}) {
    for (auto& kv : *m) (void)hipGraphExecDestroy(kv.second);
    m->clear();
  }
  for (auto& kv : h->sample_fgraphs) (void)hipGraphExecDestroy(kv.second);
  h->sample_fgraphs.clear();
  for (auto& kv : h->adj_graphs) (void)hipGraphExecDestroy(kv.second);
  h->adj_graphs.clear();
}

// Capture kGraphSteps steps of every run, each starting from buffer p, on
// the private stream.  Callers make sure that every run has kGraphSteps
// steps of budget left.  A run whose steps take an odd number of launches
// would end in the other buffer: then no graph is kept (graph_off) and the
// steps are launched one call at a time.
int build_graph(lbm_cde* h, int p) {
  std::vector<std::pair<int64_t, int>> saved;
  for (auto& r : h->runs) {
    saved.emplace_back(r.steps, r.cur);
    r.cur = p;
  }
  bool even = true;
  HIP_TRY(h, hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
  for (auto& r : h->runs) even = (enqueue_run(h, r, kGraphSteps, h->capture, true) % 2 == 0) && even;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->capture, &g);
  for (size_t i = 0; i < h->runs.size(); ++i) std::tie(h->runs[i].steps, h->runs[i].cur) = saved[i];
  if (e != hipSuccess) return fail(h, LBM_CDE_EHIP, "graph capture: %s", hipGetErrorString(e));
  if (even) e = hipGraphInstantiate(&h->graph[p], g, nullptr, nullptr, 0);
  else h->graph_off = true;
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(h, LBM_CDE_EHIP, "graph instantiate: %s", hipGetErrorString(e));
  return LBM_CDE_OK;
}

Run* get_run(lbm_cde* h, int32_t run) {
  if (!h || run < 0 || run >= (int32_t)h->runs.size()) return nullptr;
  return &h->runs[run];
}

template <typename R>
void launch_init(const Run& r, const RunArgs& a, const double* phi0, hipStream_t s) {
  const int64_t N = r.nodes;
  const unsigned blocks = (unsigned)((N + 255) / 256);
  if (r.d.lattice == LBM_CDE_D2Q9) hipLaunchKernelGGL(k_init_d2q9<R>, dim3(blocks), dim3(256), 0, s, a, phi0);
  else hipLaunchKernelGGL(k_init_d3q15<R>, dim3(blocks), dim3(256), 0, s, a, phi0);
}

int reduce_into(lbm_cde* h, Run& r, int kind, double x_ref, double* out_dev) {
  RunArgs a = make_args(h, r, r.cur);
  if (r.dbl)
    hipLaunchKernelGGL(k_reduce_partial<double>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, h->stream, a, r.Q, kind,
                       x_ref, r.red_partial);
  else if (r.half)
    hipLaunchKernelGGL(k_reduce_partial<__half>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, h->stream, a, r.Q, kind,
                       x_ref, r.red_partial);
  else
    hipLaunchKernelGGL(k_reduce_partial<float>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, h->stream, a, r.Q, kind,
                       x_ref, r.red_partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, h->stream, r.red_partial, RED_BLOCKS, out_dev);
  HIP_TRY(h, hipGetLastError());
  return LBM_CDE_OK;
}

// Device address of `scratch` on the current GPU, looked up once per device.
int scratch_address(double** out) {
  static std::mutex mu;
  static double* addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_init(LBM_CDE_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= 64) return fail_init(LBM_CDE_EUNSUPPORTED, "device %d: at most 64 GPUs are supported", dev);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail_init(LBM_CDE_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    addr[dev] = (double*)p;
  }
  *out = addr[dev];
  return LBM_CDE_OK;
}

void parse_env(lbm_cde* h) {
  const char* t2 = std::getenv("LBM_CDE_TILE");
  const char* t3 = std::getenv("LBM_CDE_TILE3");
  const char* nt = std::getenv("LBM_CDE_NT");
  const char* xcd = std::getenv("LBM_CDE_XCD");
  const char* t16 = std::getenv("LBM_CDE_TILE16");
  int bx16, by16, nt16 = 0, xcd16 = 0;
  if (const char* adj = std::getenv("LBM_CDE_ADJ")) {  // "BX[xNT]": reverse-kernel tile width, stores
    int bx = 256, ntv = 0;
    if (std::sscanf(adj, "%dx%d", &bx, &ntv) >= 1 && (bx == 64 || bx == 128 || bx == 256 || bx == 512)) {
      h->adj_bx = bx;
      h->adj_nt = ntv != 0;
    }
  }
  if (t16 && std::sscanf(t16, "%dx%dx%dx%d", &bx16, &by16, &nt16, &xcd16) >= 2) {
    h->env16_set = true;
    h->env16 = Variant{bx16, by16, 1, nt16 != 0, xcd16};
  }
  if (!t2 && !t3 && !nt && !xcd) return;
  h->env_variant = true;
  int bx, by, ny;
  int fuse = 1;
  if (t2 && std::sscanf(t2, "%dx%dx%dx%d", &bx, &by, &ny, &fuse) >= 3)
    h->env = Variant{bx, by, ny, false, 0, 0, fuse};
  if (t3 && std::sscanf(t3, "%dx%dx%d", &bx, &by, &ny) == 3) h->env3 = Variant{bx, by, ny, false, 0};
  h->env.nt = h->env3.nt = nt ? std::atoi(nt) != 0 : false;
  h->env.xcd = h->env3.xcd = xcd ? std::atoi(xcd) : 0;
}

// Power-of-two scale of 16-bit storage: the given one, or one that puts the
// largest magnitude to store at about 1/256 of the half range.  Half is a
// floating-point format, so the headroom costs no relative precision for
// values in the normal range; it absorbs later growth of the stored part
// (the non-equilibrium part grows as gradients build up in compressive
// flows).  The reduction partials of the run serve as scratch.
int choose_fp16_scale(Run& r, lbm_cde* h, const double* phi0, hipStream_t s) {
  if (r.d.fp16_scale > 0.0) {
    r.fp16_scale = r.d.fp16_scale;
    return LBM_CDE_OK;
  }
  const RunArgs a = make_args(h, r, 0);
  float* partial = (float*)r.red_partial;
  float* out = (float*)r.red_out;
  hipLaunchKernelGGL(k_fp16_probe, dim3(RED_BLOCKS), dim3(256), 0, s, a, phi0, r.split ? 1 : 0, partial);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, (const float*)partial, RED_BLOCKS, out);
  float m = 0.0f;
  HIP_TRY(nullptr, hipMemcpyAsync(&m, out, sizeof m, hipMemcpyDeviceToHost, s));
  HIP_TRY(nullptr, hipStreamSynchronize(s));
  if (!std::isfinite(m)) return fail_init(LBM_CDE_EINVAL, "init: non-finite initial state");
  const double target = kHalfMax / 256.0;
  int e = m > 0.0f ? (int)std::floor(std::log2(target / (double)m)) : 24;
  e = std::max(-24, std::min(60, e));
  r.fp16_scale = std::ldexp(1.0, e);
  return LBM_CDE_OK;
}

// Batched launch variants (row-tile width, streaming stores) compiled into the library.
using BatchFn = void (*)(const lbm_cde*, hipStream_t, unsigned);
struct BatchEntry {
  int bx;
  bool nt;
  BatchFn fn[2];  // [double?]
};
template <typename R, int BX, bool NT>
void launch_batch(const lbm_cde* h, hipStream_t s, unsigned grid) {
  if (h->batch_lean)
    hipLaunchKernelGGL((k_batch_rows_d2q9<R, BX, NT>), dim3(grid), dim3(BX), 0, s, h->dev_brun, h->dev_tiles32,
                       (int)h->runs.size(), h->dev_clock);
  else
    hipLaunchKernelGGL((k_batch_d2q9<R, BX, NT>), dim3(grid), dim3(BX), 0, s, h->dev_runs, h->dev_tiles,
                       h->dev_order, (int)h->runs.size(), h->dev_clock);
}
#define BATCH_ENTRY(BX, NT) \
  BatchEntry { BX, NT, {launch_batch<float, BX, NT>, launch_batch<double, BX, NT>} }
const BatchEntry kBatch[] = {BATCH_ENTRY(128, true), BATCH_ENTRY(256, true), BATCH_ENTRY(512, true),
                             BATCH_ENTRY(128, false), BATCH_ENTRY(256, false), BATCH_ENTRY(512, false)};

const BatchEntry* find_batch(const Variant& v) {
  if (v.by != 1 || v.ny != 1 || v.xcd != 0 || v.grid < 0 || v.fuse != 1) return nullptr;
  for (const auto& e : kBatch)
    if (e.bx == v.bx && e.nt == v.nt) return &e;
  return nullptr;
}

int compute_units() {
  int dev = 0, cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    cus = prop.multiProcessorCount;
  return cus;
}

// Candidates of the batched launch: every compiled row-tile width and store
// kind, with one block per tile or a persistent grid of 8..64 blocks per CU.
std::vector<Variant> batch_candidates() {
  std::vector<Variant> out;
  const int cus = compute_units();
  for (const auto& e : kBatch)
    for (int per_cu : {0, 8, 16, 32, 64}) out.push_back(Variant{e.bx, 1, 1, e.nt, 0, per_cu * cus});
  return out;
}

BatchFn find_batch_fused(const lbm_cde* h, const Variant& v);

// The multi-step launches every run of the batch allows.
std::vector<Variant> batch_fused_candidates(const lbm_cde* h);

// Every candidate of a batched handle: the one-step launches, then the
// multi-step ones.
std::vector<Variant> batch_all_candidates(const lbm_cde* h) {
  std::vector<Variant> out = batch_candidates();
  for (const Variant& c : batch_fused_candidates(h)) out.push_back(c);
  return out;
}

// Make v the batched launch variant: the flat tile list (runs in order of
// decreasing step budget, ceil(nx / bx) tiles per row) is rewritten in the
// workspace and the captured graphs are dropped.  tiles_out, if given,
// receives the host copy.
int apply_batch_variant(lbm_cde* h, const Variant& v, std::vector<int64_t>* tiles_out) {
  if (!find_batch(v)) return fail(h, LBM_CDE_EINVAL, "batch variant %dx%dx%d nt=%d order=%d grid=%d not built", v.bx,
                                  v.by, v.ny, (int)v.nt, v.xcd, v.grid);
  const int32_t nruns = (int32_t)h->runs.size();
  std::vector<int64_t> tiles(1, 0);
  for (int32_t k = 0; k < nruns; ++k) {
    const Run& r = h->runs[h->batch_order[k]];
    tiles.push_back(tiles.back() + (r.d.nx + v.bx - 1) / v.bx * r.d.ny);
  }
  if (tiles.back() >= ((int64_t)1 << 31)) return fail(h, LBM_CDE_EINVAL, "batch: too many tiles");
  HIP_TRY(h, hipMemcpyAsync(h->dev_tiles, tiles.data(), sizeof(int64_t) * (nruns + 1), hipMemcpyHostToDevice,
                            h->stream));
  // compact records of the lean launch, in tile-list order
  std::vector<BatchRun> br(nruns);
  std::vector<uint32_t> t32(nruns + 1);
  for (int32_t k = 0; k <= nruns; ++k) t32[k] = (uint32_t)tiles[k];
  for (int32_t k = 0; k < nruns; ++k) {
    const Run& r = h->runs[h->batch_order[k]];
    const RunArgs a = make_args(h, r, 0);
    BatchRun& b = br[k];
    std::memset(&b, 0, sizeof b);
    b.pop[0] = (const char*)r.pop[0];
    b.pop[1] = (const char*)r.pop[1];
    b.u_tab = (const char*)a.u_tab;
    b.u_slot = a.u_slot;
    b.u_flag = a.u_flag;
    b.nx = (uint32_t)r.d.nx;
    b.ny = (uint32_t)r.d.ny;
    b.pb = (uint32_t)(r.plane * (int64_t)r.elem);
    b.ntx = (uint32_t)((r.d.nx + v.bx - 1) / v.bx);
    b.inv_ntx = 1.0 / (double)b.ntx;
    b.tile0 = t32[k];
    b.bc_y = r.d.bc[1];
    b.u_kind = r.d.u_kind;
    b.model = r.d.model;
    b.max_steps = r.d.max_steps;
    b.u_const[0] = a.u_const[0];
    b.u_const[1] = a.u_const[1];
    b.phi_ref = a.phi_ref;
    b.s1 = a.s[1];
    b.s2 = a.s[2];
    b.s7 = a.s[7];
    b.s8 = a.s[8];
    b.axx = a.A[0][0];
    b.axy = a.A[0][1];
    b.ayy = a.A[1][1];
    b.s4 = a.heat[0];
    b.s6 = a.heat[1];
  }
  HIP_TRY(h, hipMemcpyAsync(h->dev_brun, br.data(), sizeof(BatchRun) * nruns, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->dev_tiles32, t32.data(), sizeof(uint32_t) * (nruns + 1), hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  drop_graphs(h);
  h->batch_var = v;
  h->batch_tiles = tiles.back();
  h->batch_grid = (unsigned)(v.grid > 0 ? std::min<int64_t>(v.grid, tiles.back()) : tiles.back());
  h->batch_prefix = tiles;
  if (tiles_out) *tiles_out = tiles;
  return LBM_CDE_OK;
}

// Several steps per launch for a whole batch (k_batch_fused_d2q9): every run
// periodic in x, of a linear equilibrium, without per-node fields, all with
// the same velocity kind (constant or separable) and all with walls in y or
// none; T divides kGraphSteps an even number of times, so that a captured
// block of multi-step launches leaves the state in the buffer that the
// step count's parity names.
template <typename R, int BX, int BY, int NY, int T>
void launch_batch_fused(const lbm_cde* h, hipStream_t s, unsigned grid) {
  const Run& r0 = h->runs[0];
  const int nr = (int)h->runs.size();
  const dim3 g(grid), b(BX, BY);
  if (r0.d.bc[1] != LBM_CDE_PERIODIC) {
    if (r0.d.u_kind == LBM_CDE_U_CONST)
      hipLaunchKernelGGL((k_batch_fused_d2q9<R, BX, BY, NY, T, 0, true>), g, b, 0, s, h->dev_brun, h->dev_tiles_f,
                         nr, h->dev_clock);
    else
      hipLaunchKernelGGL((k_batch_fused_d2q9<R, BX, BY, NY, T, 1, true>), g, b, 0, s, h->dev_brun, h->dev_tiles_f,
                         nr, h->dev_clock);
  } else if (r0.d.u_kind == LBM_CDE_U_CONST) {
    hipLaunchKernelGGL((k_batch_fused_d2q9<R, BX, BY, NY, T, 0, false>), g, b, 0, s, h->dev_brun, h->dev_tiles_f, nr,
                       h->dev_clock);
  } else {
    hipLaunchKernelGGL((k_batch_fused_d2q9<R, BX, BY, NY, T, 1, false>), g, b, 0, s, h->dev_brun, h->dev_tiles_f, nr,
                       h->dev_clock);
  }
}

template <typename R, int BX, int BY, int NY, int T>
constexpr BatchFn batch_fused_fn() {
  if constexpr (9 * (BX + 2 * (T - 1)) * (BY * NY + 2 * (T - 1)) * sizeof(R) <= 160 * 1024)
    return launch_batch_fused<R, BX, BY, NY, T>;
  else
    return nullptr;
}

struct BatchFusedEntry {
  int bx, by, ny, T;
  BatchFn fn[2];  // [double?]
};
#define BATCH_FUSED_ENTRY(BX, BY, NY, T)                                                           \
  BatchFusedEntry {                                                                                \
    BX, BY, NY, T, {batch_fused_fn<float, BX, BY, NY, T>(), batch_fused_fn<double, BX, BY, NY, T>()} \
  }
const BatchFusedEntry kBatchFused[] = {BATCH_FUSED_ENTRY(64, 8, 2, 4), BATCH_FUSED_ENTRY(64, 4, 2, 4),
                                       BATCH_FUSED_ENTRY(128, 4, 2, 4), BATCH_FUSED_ENTRY(64, 8, 2, 2),
                                       BATCH_FUSED_ENTRY(64, 12, 2, 4)};

// The multi-step batched launch of variant v, or null where it is not built
// or some run does not allow it.
BatchFn find_batch_fused(const lbm_cde* h, const Variant& v) {
  if (!h->batch_lean || v.fuse < 2 || (kGraphSteps / v.fuse) % 2 != 0 || kGraphSteps % v.fuse != 0 || !v.nt ||
      v.xcd != 0 || v.grid != 0 || h->runs.empty())
    return nullptr;
  const Run& r0 = h->runs[0];
  for (const Run& r : h->runs)
    if (!fused_ok(r, v) || r.node_par || r.d.u_kind == LBM_CDE_U_FIELD || r.d.u_kind != r0.d.u_kind ||
        (r.d.bc[1] == LBM_CDE_PERIODIC) != (r0.d.bc[1] == LBM_CDE_PERIODIC) || r.dbl != r0.dbl)
      return nullptr;
  for (const auto& e : kBatchFused)
    if (e.bx == v.bx && e.by == v.by && e.ny == v.ny && e.T == v.fuse) return e.fn[r0.dbl ? 1 : 0];
  return nullptr;
}

std::vector<Variant> batch_fused_candidates(const lbm_cde* h) {
  std::vector<Variant> out;
  for (const auto& e : kBatchFused) {
    const Variant c{e.bx, e.by, e.ny, true, 0, 0, e.T};
    if (find_batch_fused(h, c)) out.push_back(c);
  }
  return out;
}

// Make v the multi-step batched launch (v.fuse > 1; validated by the caller
// with find_batch_fused) or switch it off (v.fuse == 1): the flat list of
// BX x (BY * NY) tiles over the runs, in batch order, goes to the workspace.
int apply_batch_fused(lbm_cde* h, const Variant& v) {
  if (v.fuse > 1) {
    const int32_t nruns = (int32_t)h->runs.size();
    std::vector<int64_t> tiles(1, 0);
    const int64_t th = (int64_t)v.by * v.ny;
    for (int32_t k = 0; k < nruns; ++k) {
      const Run& r = h->runs[h->batch_order[k]];
      tiles.push_back(tiles.back() + (r.d.nx + v.bx - 1) / v.bx * ((r.d.ny + th - 1) / th));
    }
    if (tiles.back() >= ((int64_t)1 << 31)) return fail(h, LBM_CDE_EINVAL, "batch: too many tiles");
    std::vector<uint32_t> t32(nruns + 1);
    for (int32_t k = 0; k <= nruns; ++k) t32[k] = (uint32_t)tiles[k];
    HIP_TRY(h, hipMemcpyAsync(h->dev_tiles_f, t32.data(), sizeof(uint32_t) * (nruns + 1), hipMemcpyHostToDevice,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->batch_prefix_f = tiles;
  }
  drop_graphs(h);
  h->batch_fuse = v;
  return LBM_CDE_OK;
}

// Launch grid of the multi-step batched launch from step t on: the tiles of
// the runs still active, rounded up to a power of two (blocks past them exit).
unsigned batch_fgrid_at(const lbm_cde* h, int64_t t) {
  int64_t active = 0;
  for (size_t k = 0; k < h->batch_order.size(); ++k) {
    const int64_t ms = h->runs[h->batch_order[k]].d.max_steps;
    if (ms >= 0 && t >= ms) break;
    active = h->batch_prefix_f[k + 1];
  }
  const int64_t total = h->batch_prefix_f.back();
  int64_t g = 64;
  while (g < active && g < total) g *= 2;
  return (unsigned)std::max<int64_t>(1, std::min(g, total));
}

// Whether steps t .. t + n of a batch may take the multi-step launch: it is
// on, and no run's budget ends strictly inside the span.
bool batch_fused_span(const lbm_cde* h, int64_t t, int64_t n) {
  if (h->batch_fuse.fuse < 2 || n < 2 * h->batch_fuse.fuse) return false;
  for (const Run& r : h->runs) {
    const int64_t ms = r.d.max_steps;
    if (ms >= 0 && ms > t && ms < t + n) return false;
  }
  return true;
}

// Per-run set-up of lbm_cde_init (errors go to the thread's init error text).
int init_runs(lbm_cde* h, const lbm_cde_run_desc* runs, int32_t nruns, const double* const* phi0, char* workspace,
              size_t ws_bytes) {
  size_t off = 0;
  for (int i = 0; i < nruns; ++i) {
    int rc = validate(runs[i], i);
    if (rc) return rc;
    if (!phi0[i]) return fail_init(LBM_CDE_EINVAL, "run %d: phi0 is NULL", i);
    Run r;
    r.d = runs[i];
    const size_t need = layout(r, nullptr);
    if (off + need > ws_bytes) return fail_init(LBM_CDE_ENOSPC, "init: workspace of %zu bytes is too small", ws_bytes);
    layout(r, workspace + off);
    off += need;
    if ((rc = derive(r, i)) || (rc = check_velocity(r, i)) || (rc = check_stability(r, i))) return rc;
    r.walls = false;
    for (int a = 0; a < r.dim; ++a) r.walls |= r.d.bc[a] != LBM_CDE_PERIODIC;
    r.var = default_variant(r.d.lattice, r.d.precision);
    {
      // runs that can take several steps per launch do so by default (64 x 24
      // tiles, 4 steps, XCD-contiguous order in FP32, else 64 x 16; 64 x 8,
      // 4 steps, XCD-contiguous order in FP64)
      const Variant multi = r.dbl ? Variant{64, 4, 2, true, 1, 0, 4} : Variant{64, 12, 2, true, 1, 0, 4};
      const Variant multi16 = Variant{64, 8, 2, true, 0, 0, 4};
      if (r.d.lattice == LBM_CDE_D2Q9 && !r.half && find_step(r, multi)) r.var = multi;
      else if (r.d.lattice == LBM_CDE_D2Q9 && !r.half && !r.dbl && find_step(r, multi16)) r.var = multi16;
    }
    if (r.split && h->env16_set) r.var = h->env16;
    if (h->env_variant && !r.half) r.var = r.d.lattice == LBM_CDE_D3Q15 ? h->env3 : h->env;
    if (r.var.fuse == 1) r.var1 = r.var;
    else r.var1 = default_variant(r.d.lattice, r.d.precision);
    if (!find_step(r, r.var) || !find_step(r, r.var1))
      return fail_init(LBM_CDE_EINVAL, "run %d: launch variant not built", i);
    // host tables are copied during init; keep no pointer to caller memory
    r.d.u_tables = nullptr;
    r.d.u_field = nullptr;
    r.d.D_field = nullptr;
    const lbm_cde_run_desc& orig = runs[i];
    hipStream_t s = h->stream;
    if (orig.u_kind == LBM_CDE_U_SEPARABLE) {
      const size_t n = (size_t)r.dim * (1 + orig.nx + orig.ny + orig.nz);
      if (r.dim == 2) {
        const size_t st = 1 + orig.nx + orig.ny + orig.nz;
        r.u_z_unit = orig.u_tables[st - 1] == 1.0 && orig.u_tables[2 * st - 1] == 1.0;
      }
      if (r.dbl) {
        HIP_TRY(nullptr, hipMemcpyAsync(r.utab, orig.u_tables, n * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(nullptr, hipStreamSynchronize(s));  // the caller's table may go away after init
      } else {
        std::vector<float> tmp(n);
        for (size_t k = 0; k < n; ++k) tmp[k] = (float)orig.u_tables[k];
        HIP_TRY(nullptr, hipMemcpyAsync(r.utab, tmp.data(), n * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(nullptr, hipStreamSynchronize(s));
      }
    } else if (orig.u_kind == LBM_CDE_U_FIELD) {
      // the steps read the field through the slot: first the library's copy,
      // later whatever lbm_cde_set_velocity points it at
      const int64_t n = r.dim * r.nodes;
      const unsigned blocks = (unsigned)((n + 255) / 256);
      hipLaunchKernelGGL(k_convert<double>, dim3(blocks), dim3(256), 0, s, orig.u_field, (double*)r.ufield, n);
      hipLaunchKernelGGL(k_store_ptr, dim3(1), dim3(64), 0, s, (const double**)r.uslot, (const double*)r.ufield);
      HIP_TRY(nullptr, hipMemsetAsync(&r.flags[2], 0, sizeof(unsigned long long), s));
      hipLaunchKernelGGL(k_check_speed, dim3((unsigned)((r.nodes + 255) / 256)), dim3(256), 0, s,
                         (const double*)r.ufield, r.dim, r.nodes, (unsigned*)&r.flags[2]);
      unsigned long long fast = 0;
      HIP_TRY(nullptr, hipMemcpyAsync(&fast, &r.flags[2], sizeof fast, hipMemcpyDeviceToHost, s));
      HIP_TRY(nullptr, hipStreamSynchronize(s));
      if (fast) return fail_init(LBM_CDE_EUNSTABLE, "run %d: |u| reaches the lattice sound speed 1/sqrt(3)", i);
    }
    if (orig.D_field) {
      HIP_TRY(nullptr, hipMemsetAsync(r.flags, 0, sizeof(unsigned long long), s));
      const unsigned blocks = (unsigned)((r.nodes + 255) / 256);
      if (r.dbl)
        hipLaunchKernelGGL(k_node_params_2d<double>, dim3(blocks), dim3(256), 0, s, orig.D_field, r.nodes, r.kappa,
                           orig.heat_rule, orig.heat_rates[0], orig.heat_rates[1], (double*)r.node_par, r.flags);
      else
        hipLaunchKernelGGL(k_node_params_2d<float>, dim3(blocks), dim3(256), 0, s, orig.D_field, r.nodes, r.kappa,
                           orig.heat_rule, orig.heat_rates[0], orig.heat_rates[1], (float*)r.node_par, r.flags);
      unsigned long long bad = 0;
      HIP_TRY(nullptr, hipMemcpyAsync(&bad, r.flags, sizeof bad, hipMemcpyDeviceToHost, s));
      HIP_TRY(nullptr, hipStreamSynchronize(s));
      if (bad) return fail_init(LBM_CDE_ENOTSPD, "run %d: %llu nodes of D_field are not SPD", i, bad);
    }
    HIP_TRY(nullptr, hipMemsetAsync(&r.flags[1], 0, sizeof(unsigned long long), s));
    if (r.half) {
      int rc2 = choose_fp16_scale(r, h, phi0[i], s);
      if (rc2) return rc2;
    }
    // initial populations: the equilibrium of phi0, written to buffer 0
    const RunArgs a = make_args(h, r, 1);
    if (r.half) {
      const unsigned blocks = (unsigned)((r.nodes + 255) / 256);
      hipLaunchKernelGGL(k_init_d2q9_fp16, dim3(blocks), dim3(256), 0, s, a, phi0[i], r.split ? 1 : 0,
                         (unsigned*)&r.flags[1]);
    } else if (r.dbl) {
      launch_init<double>(r, a, phi0[i], s);
    } else {
      launch_init<float>(r, a, phi0[i], s);
    }
    HIP_TRY(nullptr, hipGetLastError());
    h->runs.push_back(r);
  }
  if (batch_eligible(runs, nruns)) {
    if (off + batch_bytes(nruns) > ws_bytes)
      return fail_init(LBM_CDE_ENOSPC, "init: workspace of %zu bytes is too small", ws_bytes);
    char* p = workspace + off;
    h->dev_runs = (RunArgs*)p;
    p += align_up(sizeof(RunArgs) * nruns);
    h->dev_tiles = (int64_t*)p;
    p += align_up(sizeof(int64_t) * (nruns + 1));
    h->dev_order = (int32_t*)p;
    p += align_up(sizeof(int32_t) * nruns);
    h->dev_clock = (int64_t*)p;
    p += align_up(3 * sizeof(int64_t));
    h->batch_partial = (double*)p;
    p += align_up(sizeof(double) * 3 * kBatchRedBlocks * nruns);
    h->dev_brun = (BatchRun*)p;
    p += align_up(sizeof(BatchRun) * nruns);
    h->dev_tiles32 = (uint32_t*)p;
    p += align_up(sizeof(uint32_t) * (nruns + 1));
    h->dev_tiles_f = (uint32_t*)p;
    std::vector<RunArgs> args;
    h->batch_lean = true;
    for (auto& r : h->runs) {
      args.push_back(make_args(h, r, 0));
      h->batch_lean = h->batch_lean && args.back().rows32;
    }
    if (std::getenv("LBM_CDE_BATCH_GENERAL")) h->batch_lean = false;  // the general kernel for every batch
    // tile list in order of decreasing step budget (unlimited first), so that
    // the active runs always own a prefix of it
    std::vector<int32_t> order(nruns);
    for (int32_t i = 0; i < nruns; ++i) order[i] = i;
    auto budget = [&](int32_t i) {
      const int64_t m = h->runs[i].d.max_steps;
      return m < 0 ? INT64_MAX : m;
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return budget(x) > budget(y); });
    h->batch_order = order;
    hipStream_t s = h->stream;
    HIP_TRY(nullptr, hipMemcpyAsync(h->dev_runs, args.data(), sizeof(RunArgs) * nruns, hipMemcpyHostToDevice, s));
    HIP_TRY(nullptr, hipMemcpyAsync(h->dev_order, order.data(), sizeof(int32_t) * nruns, hipMemcpyHostToDevice, s));
    HIP_TRY(nullptr, hipMemsetAsync(h->dev_clock, 0, 3 * sizeof(int64_t), s));
    HIP_TRY(nullptr, hipStreamSynchronize(s));
    h->batched = true;
    Variant bv = h->batch_var;
    int bx = bv.bx, nt = 1, grid = 0;
    if (const char* e = std::getenv("LBM_CDE_BATCH"))  // "BX[xNT[xGRID]]" fixes the batched launch variant
      if (std::sscanf(e, "%dx%dx%d", &bx, &nt, &grid) >= 1) bv = Variant{bx, 1, 1, nt != 0, 0, grid};
    if (apply_batch_variant(h, bv, nullptr)) return fail_init(LBM_CDE_EINVAL, "init: %s", h->err.c_str());
    // several steps per launch by default where every run allows it (not
    // when LBM_CDE_BATCH fixes the one-step launch); LBM_CDE_BATCH_FUSE =
    // "BXxBYxNYxT" fixes the multi-step one
    Variant fv = h->runs[0].dbl ? Variant{64, 4, 2, true, 0, 0, 4} : Variant{64, 12, 2, true, 0, 0, 4};
    if (!find_batch_fused(h, fv)) fv = Variant{64, 8, 2, true, 0, 0, 4};
    int fbx, fby, fny, ft;
    if (const char* e = std::getenv("LBM_CDE_BATCH_FUSE"))
      if (std::sscanf(e, "%dx%dx%dx%d", &fbx, &fby, &fny, &ft) == 4) fv = Variant{fbx, fby, fny, true, 0, 0, ft};
    if (!std::getenv("LBM_CDE_BATCH") && find_batch_fused(h, fv) && apply_batch_fused(h, fv))
      return fail_init(LBM_CDE_EINVAL, "init: %s", h->err.c_str());
  }
  HIP_TRY(nullptr, hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking));
  return LBM_CDE_OK;
}

// Launch grid for steps from global step t on: the variant's grid, but no
// more blocks than the tiles of the runs still active at t (the runs are
// listed by decreasing budget, so they own a prefix of the tile list; the
// count only falls as t grows), rounded up to a power of two so that few
// distinct graphs are captured.  The kernel finds the active prefix itself
// every step, so any grid of at least one block is correct; this only keeps
// the finished runs' tiles from costing blocks that exit at once.
unsigned batch_grid_at(const lbm_cde* h, int64_t t) {
  int64_t active = 0;
  for (size_t k = 0; k < h->batch_order.size(); ++k) {
    const int64_t ms = h->runs[h->batch_order[k]].d.max_steps;
    if (ms >= 0 && t >= ms) break;
    active = h->batch_prefix[k + 1];
  }
  unsigned g = 64;
  while ((int64_t)g < active && g < h->batch_grid) g *= 2;
  return std::min(g, h->batch_grid);
}

// One batched step: the persistent kernel, then the clock tick.
void launch_batch_step(lbm_cde* h, hipStream_t s, unsigned grid) {
  find_batch(h->batch_var)->fn[h->runs[0].dbl ? 1 : 0](h, s, grid);
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, h->dev_clock, 0, 1);
}

// Sample the x-moments of every run into hist[row], then advance the row clock.
void launch_batch_sample(lbm_cde* h, hipStream_t s, double* hist) {
  const int nr = (int)h->runs.size();
  const int Q = h->runs[0].Q;
  if (h->runs[0].dbl)
    hipLaunchKernelGGL(k_batch_xmom_partial<double>, dim3(kBatchRedBlocks, nr), dim3(RED_THREADS), 0, s,
                       h->dev_runs, Q, h->dev_clock, h->batch_partial);
  else
    hipLaunchKernelGGL(k_batch_xmom_partial<float>, dim3(kBatchRedBlocks, nr), dim3(RED_THREADS), 0, s,
                       h->dev_runs, Q, h->dev_clock, h->batch_partial);
  hipLaunchKernelGGL(k_batch_xmom_final, dim3(nr), dim3(RED_THREADS), 0, s, h->batch_partial, kBatchRedBlocks, nr,
                     h->dev_clock, hist);
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, h->dev_clock, 1, 1);
}

// Capture `steps` batched steps of the given grid (and, with hist, one
// sample) as a graph.  With gridf > 0 the steps go in pairs of multi-step
// launches of that grid as far as they fit, the rest one per launch.
int capture_batch(lbm_cde* h, int64_t steps, double* hist, unsigned grid, hipGraphExec_t* out, unsigned gridf = 0) {
  HIP_TRY(h, hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
  int64_t one = steps;
  if (gridf > 0) {
    const int T = h->batch_fuse.fuse;
    const int64_t q = steps / (2 * T) * 2;
    const BatchFn fn = find_batch_fused(h, h->batch_fuse);
    for (int64_t k = 0; k < q; ++k) {
      fn(h, h->capture, gridf);
      hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, h->capture, h->dev_clock, 2, T);
    }
    one = steps - q * T;
  }
  for (int64_t t = 0; t < one; ++t) launch_batch_step(h, h->capture, grid);
  if (hist) launch_batch_sample(h, h->capture, hist);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->capture, &g);
  if (e != hipSuccess) return fail(h, LBM_CDE_EHIP, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(h, LBM_CDE_EHIP, "graph instantiate: %s", hipGetErrorString(e));
  return LBM_CDE_OK;
}

void advance_host_clock(lbm_cde* h, int64_t n) {
  h->global_steps += n;
  for (auto& r : h->runs) {
    r.steps = (r.d.max_steps >= 0 && h->global_steps > r.d.max_steps) ? r.d.max_steps : h->global_steps;
    r.cur = (int)(r.steps & 1);  // the batched kernels take the buffer from the step's parity
  }
}

int batch_step(lbm_cde* h, int64_t n) {
  int64_t done = 0;
  while (done < n) {
    const unsigned grid = batch_grid_at(h, h->global_steps);
    if (n - done >= kGraphSteps) {
      const bool fused = batch_fused_span(h, h->global_steps, kGraphSteps);
      const unsigned gridf = fused ? batch_fgrid_at(h, h->global_steps) : 0;
      auto& graphs = fused ? h->batch_fgraphs : h->batch_graphs;
      const unsigned key = fused ? gridf : grid;
      hipGraphExec_t& g = graphs[key];
      if (!g) {
        const int rc = capture_batch(h, kGraphSteps, nullptr, grid, &g, gridf);
        if (rc) {
          graphs.erase(key);
          return rc;
        }
      }
      HIP_TRY(h, hipGraphLaunch(g, h->stream));
      advance_host_clock(h, kGraphSteps);
      done += kGraphSteps;
    } else {
      launch_batch_step(h, h->stream, grid);
      HIP_TRY(h, hipGetLastError());
      advance_host_clock(h, 1);
      done += 1;
    }
  }
  return LBM_CDE_OK;
}

// ---- autotuner -------------------------------------------------------------

std::string tune_key(const Run& r) {
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s:%s:%s:%lldx%lldx%lld:%d%d%d", arch.c_str(),
                r.d.lattice == LBM_CDE_D2Q9 ? "d2q9" : "d3q15",
                r.dbl ? "fp64" : r.split ? "fp16split" : r.half ? "fp16" : "fp32", (long long)r.d.nx,
                (long long)r.d.ny, (long long)r.d.nz, r.d.bc[0], r.d.bc[1], r.d.bc[2]);
  return buf;
}

bool cache_lookup(const std::string& key, Variant& v) {
  const char* path = std::getenv("LBM_CDE_TUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512], k[256];
  int bx, by, ny, nt, xcd, grid, fuse;
  double ms;
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    fuse = 1;  // lines without the steps-per-launch field are one-step variants
    if (std::sscanf(line, "%255s %d %d %d %d %d %d %lf %d", k, &bx, &by, &ny, &nt, &xcd, &grid, &ms, &fuse) >= 8 &&
        key == k) {
      v = Variant{bx, by, ny, nt != 0, xcd, grid, fuse};
      found = true;  // the last entry wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, const Variant& v, double ms) {
  const char* path = std::getenv("LBM_CDE_TUNE_CACHE");
  if (!path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%s %d %d %d %d %d %d %.6f %d\n", key.c_str(), v.bx, v.by, v.ny, (int)v.nt, v.xcd, v.grid, ms,
                 v.fuse);
    std::fclose(f);
  }
}

// Time `trials` launches of variant v on run r.  Every launch reads the
// current state and writes the other buffer, so the state is not changed.
int time_variant(lbm_cde* h, Run& r, const Variant& v, int trials, double* ms) {
  StepFn fn = find_step(r, v);
  if (!fn) return LBM_CDE_EINVAL;
  const RunArgs a = make_args(h, r, r.cur, &v);
  hipEvent_t e0, e1;
  HIP_TRY(h, hipEventCreate(&e0));
  HIP_TRY(h, hipEventCreate(&e1));
  fn(a, h->stream);  // warm-up
  HIP_TRY(h, hipEventRecord(e0, h->stream));
  for (int t = 0; t < trials; ++t) fn(a, h->stream);
  HIP_TRY(h, hipEventRecord(e1, h->stream));
  HIP_TRY(h, hipEventSynchronize(e1));
  float elapsed = 0.f;
  HIP_TRY(h, hipEventElapsedTime(&elapsed, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(h, hipGetLastError());
  *ms = elapsed / trials / v.fuse;  // per step
  return LBM_CDE_OK;
}

// Time `trials` launches of the batched step kernel (or of the multi-step
// one, per step) without advancing the clock: each reads the current buffers
// and writes the other ones, so the state of every run is unchanged.
int time_batch(lbm_cde* h, int trials, double* ms, const Variant* fused = nullptr) {
  const BatchFn fn = fused ? find_batch_fused(h, *fused) : find_batch(h->batch_var)->fn[h->runs[0].dbl ? 1 : 0];
  const unsigned grid = fused ? (unsigned)h->batch_prefix_f.back() : h->batch_grid;
  hipEvent_t e0, e1;
  HIP_TRY(h, hipEventCreate(&e0));
  HIP_TRY(h, hipEventCreate(&e1));
  fn(h, h->stream, grid);  // warm-up
  HIP_TRY(h, hipEventRecord(e0, h->stream));
  for (int t = 0; t < trials; ++t) fn(h, h->stream, grid);
  HIP_TRY(h, hipEventRecord(e1, h->stream));
  HIP_TRY(h, hipEventSynchronize(e1));
  float elapsed = 0.f;
  HIP_TRY(h, hipEventElapsedTime(&elapsed, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(h, hipGetLastError());
  *ms = elapsed / trials / (fused ? fused->fuse : 1);  // per step
  return LBM_CDE_OK;
}

// Launch variants of a run stepped alone: every compiled tile shape and store
// kind in every block order (the row-interleaved one only with a multiple of
// 8 tile rows).
std::vector<Variant> run_candidates(const Run& r) {
  std::vector<Variant> out;
  auto add = [&](const Variant& c) {
    if (c.xcd == 2 && tile_rows(r, c) % 8 != 0) return;
    out.push_back(c);
  };
  for (int xcd = 0; xcd < 3; ++xcd) {
    if (r.split) {
      for (const auto& e : kSplit)
        for (int nt = 0; nt < (r.walls ? 1 : 2); ++nt) add(Variant{e.bx, e.by, 1, nt != 0, xcd});
    } else if (r.half) {
      add(Variant{256, 1, 1, false, xcd});
    } else if (r.d.lattice == LBM_CDE_D3Q15) {
      for (const auto& e : kSteps3) add(Variant{e.bx, e.by, e.ny, e.nt, xcd});
    } else {
      for (const auto& e : kSteps) add(Variant{e.bx, e.by, e.ny, e.nt, xcd});
      for (const auto& e : kFused) {
        const Variant c{e.bx, e.by, e.ny, true, xcd, 0, e.T};
        if (find_step(r, c)) add(c);
      }
    }
  }
  return out;
}

// Tuning-cache key of a batch: architecture, precision and every run's grid,
// boundaries and step budget (FNV-1a).
std::string batch_tune_key(const lbm_cde* h) {
  uint64_t fnv = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int b = 0; b < 8; ++b) {
      fnv ^= (uint64_t)((v >> (8 * b)) & 0xff);
      fnv *= 1099511628211ull;
    }
  };
  for (const auto& r : h->runs) {
    mix(r.d.nx);
    mix(r.d.ny);
    mix(r.d.bc[0] * 16 + r.d.bc[1]);
    mix(r.d.max_steps);
  }
  const std::string first = tune_key(h->runs[0]);
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s:batch%zu:%016llx", first.substr(0, first.find(':')).c_str(), h->runs.size(),
                (unsigned long long)fnv);
  return std::string(buf) + (h->runs[0].dbl ? ":fp64" : ":fp32");
}

// Variant as the six integers of the C ABI.
void variant_out(const Variant& v, int grid, int32_t* out) {
  out[0] = v.bx;
  out[1] = v.by;
  out[2] = v.ny;
  out[3] = v.nt ? 1 : 0;
  out[4] = v.xcd;
  out[5] = grid;
  out[6] = v.fuse;
}

}  // namespace

namespace {

int check_adjoint_run(lbm_cde* h, Run* r) {
  if (!r) return fail(h, LBM_CDE_EINVAL, "adjoint: bad handle or run");
  if (r->d.lattice != LBM_CDE_D2Q9 || r->half)
    return fail(h, LBM_CDE_EUNSUPPORTED, "adjoint: built for D2Q9 in FP64 or FP32 storage");
  if (r->d.model != LBM_CDE_MRT_A)
    return fail(h, LBM_CDE_EUNSUPPORTED, "adjoint: built for the modified model MRT-A");
  for (int a = 0; a < 2; ++a)
    if (r->d.bc[a] == LBM_CDE_NODE_MIRROR)
      return fail(h, LBM_CDE_EUNSUPPORTED, "adjoint: the plate rule is not a permutation, no adjoint is built");
  if (r->d.heat_rule != LBM_CDE_HEAT_EXPLICIT)
    return fail(h, LBM_CDE_EUNSUPPORTED,
                "adjoint: needs explicit heat-flux rates (the other rules make them depend on D)");
  return LBM_CDE_OK;
}

// The buffers of one reverse step.
struct AdjBufs {
  const void* v;      // v_t of the forward step, [2][N]
  const void* mu_in;  // mu_{t+1}
  const double* inj;  // dL/dphi_{t+1} or null
  void* mu_out;       // mu_t
  double* grad;       // FP64 output [3][N]
  float* part;        // FP32 partial [3][N]
};

template <typename R, bool WALLS, int GMODE, bool NT>
void launch_adjoint_g(const RunArgs& a, unsigned blocks, unsigned bx, const AdjBufs& b, double inv_kappa,
                      hipStream_t s) {
  const FastDiv ntx = make_fastdiv((uint32_t)((a.nx + bx - 1) / bx));
  if (b.inj)
    hipLaunchKernelGGL((k_adjoint_d2q9<R, WALLS, GMODE, true, NT>), dim3(blocks), dim3(bx), 0, s, a, (const R*)b.v,
                       (const R*)b.mu_in, b.inj, (R*)b.mu_out, b.grad, b.part, inv_kappa, ntx);
  else
    hipLaunchKernelGGL((k_adjoint_d2q9<R, WALLS, GMODE, false, NT>), dim3(blocks), dim3(bx), 0, s, a, (const R*)b.v,
                       (const R*)b.mu_in, b.inj, (R*)b.mu_out, b.grad, b.part, inv_kappa, ntx);
}

template <typename R, bool WALLS, bool NT>
void launch_adjoint_w(const RunArgs& a, unsigned blocks, unsigned bx, const AdjBufs& b, int gmode,
                      double inv_kappa, hipStream_t s) {
  if constexpr (sizeof(R) == 4) {
    if (gmode == GRAD_F32_SET) return launch_adjoint_g<R, WALLS, GRAD_F32_SET, NT>(a, blocks, bx, b, inv_kappa, s);
    if (gmode == GRAD_F32_ADD) return launch_adjoint_g<R, WALLS, GRAD_F32_ADD, NT>(a, blocks, bx, b, inv_kappa, s);
    if (gmode == GRAD_F32_FOLD) return launch_adjoint_g<R, WALLS, GRAD_F32_FOLD, NT>(a, blocks, bx, b, inv_kappa, s);
  }
  launch_adjoint_g<R, WALLS, GRAD_F64, NT>(a, blocks, bx, b, inv_kappa, s);
}

// Every byte offset of the wall-free reverse kernel fits 32 bits: the Q
// population planes and the three FP64 gradient planes.
bool adjoint_offsets32(const Run& r) {
  return (double)r.Q * r.plane * r.elem < 4294967296.0 && 24.0 * (double)r.nodes < 4294967296.0;
}

template <typename R>
void launch_adjoint(const lbm_cde* h, const Run& r, const RunArgs& a, const AdjBufs& b, int gmode, double inv_kappa,
                    hipStream_t s) {
  const unsigned bx = (unsigned)h->adj_bx;
  const unsigned blocks = (unsigned)((r.d.nx + bx - 1) / bx * r.d.ny);  // bx-wide row tiles
  // periodic runs whose offsets do not fit 32 bits take the general kernel
  const bool walls = r.walls || !adjoint_offsets32(r);
  if (h->adj_nt) {
    if (walls) launch_adjoint_w<R, true, true>(a, blocks, bx, b, gmode, inv_kappa, s);
    else launch_adjoint_w<R, false, true>(a, blocks, bx, b, gmode, inv_kappa, s);
  } else {
    if (walls) launch_adjoint_w<R, true, false>(a, blocks, bx, b, gmode, inv_kappa, s);
    else launch_adjoint_w<R, false, false>(a, blocks, bx, b, gmode, inv_kappa, s);
  }
}

// One recomputed forward step of a segment: state and v, or only v (STORE false).
template <typename R>
void launch_step_v(const Run& r, const RunArgs& a, void* v, bool store, hipStream_t s) {
  const unsigned blocks = (unsigned)((r.d.nx + 255) / 256 * r.d.ny);
  const FastDiv ntx = make_fastdiv((uint32_t)((r.d.nx + 255) / 256));
  if (r.walls) {
    if (store) hipLaunchKernelGGL((k_step_v_d2q9<R, true, true>), dim3(blocks), dim3(256), 0, s, a, (R*)v, ntx);
    else hipLaunchKernelGGL((k_step_v_d2q9<R, true, false>), dim3(blocks), dim3(256), 0, s, a, (R*)v, ntx);
  } else {
    if (store) hipLaunchKernelGGL((k_step_v_d2q9<R, false, true>), dim3(blocks), dim3(256), 0, s, a, (R*)v, ntx);
    else hipLaunchKernelGGL((k_step_v_d2q9<R, false, false>), dim3(blocks), dim3(256), 0, s, a, (R*)v, ntx);
  }
}

// Several steps per launch in a checkpoint segment (adjoint_fused_d2q9.hpp):
// the forward recomputation with v, and the reverse sweep.
template <typename R, int BX, int BY, int NY, int T>
void launch_fused_v(const RunArgs& a, char* vout, int64_t vstep, bool store, hipStream_t s) {
  const unsigned blocks = (unsigned)(((a.nx + BX - 1) / BX) * ((a.ny + BY * NY - 1) / (BY * NY)));
  const dim3 g(blocks), b(BX, BY);
  if (a.node_par) {  // velocity constant or separable (fused_ok)
    if (a.u_kind == U_CONST)
      hipLaunchKernelGGL((k_fused_v_d2q9<R, BX, BY, NY, T, 0, true>), g, b, 0, s, a, vout, vstep, (int)store);
    else
      hipLaunchKernelGGL((k_fused_v_d2q9<R, BX, BY, NY, T, 1, true>), g, b, 0, s, a, vout, vstep, (int)store);
  } else if (a.u_kind == U_CONST) {
    hipLaunchKernelGGL((k_fused_v_d2q9<R, BX, BY, NY, T, 0, false>), g, b, 0, s, a, vout, vstep, (int)store);
  } else if (a.u_kind == U_SEPARABLE) {
    hipLaunchKernelGGL((k_fused_v_d2q9<R, BX, BY, NY, T, 1, false>), g, b, 0, s, a, vout, vstep, (int)store);
  } else {
    hipLaunchKernelGGL((k_fused_v_d2q9<R, BX, BY, NY, T, 2, false>), g, b, 0, s, a, vout, vstep, (int)store);
  }
}

template <typename R, int BX, int BY, int NY, int T>
void launch_fused_adj(const RunArgs& a, const char* v_hi, int64_t vstep, const void* mu_in, void* mu_out,
                      double* grad, float* part, double inv_kappa, bool fold, hipStream_t s) {
  const unsigned blocks = (unsigned)(((a.nx + BX - 1) / BX) * ((a.ny + BY * NY - 1) / (BY * NY)));
  if (a.node_par)
    hipLaunchKernelGGL((k_fused_adj_d2q9<R, BX, BY, NY, T, true>), dim3(blocks), dim3(BX, BY), 0, s, a, v_hi, vstep,
                       (const R*)mu_in, (R*)mu_out, grad, part, inv_kappa, (int)fold);
  else
    hipLaunchKernelGGL((k_fused_adj_d2q9<R, BX, BY, NY, T, false>), dim3(blocks), dim3(BX, BY), 0, s, a, v_hi,
                       vstep, (const R*)mu_in, (R*)mu_out, grad, part, inv_kappa, (int)fold);
}

// The shape of the multi-step adjoint launches: FP32 64 x 16 tiles with 4
// steps, FP64 64 x 8 tiles with 3 (the reverse kernel adds the tile's
// running gradient sums to the LDS of the forward one).
Variant adjoint_multi_variant(const Run& r) {
  return r.dbl ? Variant{64, 4, 2, true, 0, 0, 3} : Variant{64, 8, 2, true, 0, 0, 4};
}

// Scratch of a segment of K steps: two ping-pong states, v of every step
// ([K][2][N] in the storage precision) and the FP32 gradient partial [3][N].
struct SegLayout {
  size_t state, v_step, v, part, total;
};
SegLayout seg_layout(const Run& r, int64_t K) {
  SegLayout L;
  L.state = align_up((size_t)r.Q * r.plane * r.elem);
  L.v_step = align_up(2 * (size_t)r.nodes * r.elem);
  L.v = 2 * L.state;
  L.part = L.v + (size_t)K * L.v_step;
  L.total = L.part + align_up(3 * sizeof(float) * (size_t)r.nodes);
  return L;
}

}  // namespace

// ---- C ABI ----------------------------------------------------------------

extern "C" {

int lbm_cde_workspace_bytes(const lbm_cde_run_desc* runs, int32_t nruns, size_t* bytes) {
  if (!runs || nruns < 1 || !bytes) return fail_init(LBM_CDE_EINVAL, "workspace_bytes: null argument or nruns < 1");
  size_t total = 0;
  for (int i = 0; i < nruns; ++i) {
    int rc = validate(runs[i], i);
    if (rc) return rc;
    Run r;
    r.d = runs[i];
    total += layout(r, nullptr);
    if ((rc = derive(r, i)) || (rc = check_velocity(r, i)) || (rc = check_stability(r, i))) return rc;
  }
  if (batch_eligible(runs, nruns)) total += batch_bytes(nruns);
  *bytes = total;
  return LBM_CDE_OK;
}

int lbm_cde_init(const lbm_cde_run_desc* runs, int32_t nruns, const double* const* phi0, void* workspace,
                 size_t ws_bytes, void* hip_stream, lbm_cde_handle* out) {
  if (out) *out = nullptr;
  if (!runs || nruns < 1 || !phi0 || !workspace || !out)
    return fail_init(LBM_CDE_EINVAL, "init: null argument or nruns < 1");
  if ((uintptr_t)workspace % kAlign) return fail_init(LBM_CDE_EINVAL, "init: workspace not 256-byte aligned");
  lbm_cde* h = new lbm_cde();
  h->stream = (hipStream_t)hip_stream;
  parse_env(h);
  int rc = scratch_address(&h->scratch_dev);
  if (!rc) rc = init_runs(h, runs, nruns, phi0, (char*)workspace, ws_bytes);
  if (rc) {
    if (h->capture) (void)hipStreamDestroy(h->capture);
    delete h;
    return rc;
  }
  *out = h;
  return LBM_CDE_OK;
}

int lbm_cde_step(lbm_cde_handle h, int64_t n) {
  if (!h) return fail_init(LBM_CDE_EINVAL, "step: null handle");
  if (n < 0) return fail(h, LBM_CDE_EINVAL, "step: negative step count %lld", (long long)n);
  if (h->batched) return batch_step(h, n);
  int64_t done = 0;
  while (done < n) {
    // a captured graph is valid while every run takes all kGraphSteps steps
    bool uniform = n - done >= kGraphSteps;
    int parity = -1;
    for (auto& r : h->runs) {
      if (r.d.max_steps >= 0 && r.steps + kGraphSteps > r.d.max_steps) uniform = false;
      const int p = r.cur;
      if (parity < 0) parity = p;
      else if (parity != p) uniform = false;
    }
    if (uniform && parity >= 0 && !h->graph[parity] && !h->graph_off) {
      const int rc = build_graph(h, parity);
      if (rc) return rc;
    }
    if (uniform && parity >= 0 && h->graph[parity]) {
      HIP_TRY(h, hipGraphLaunch(h->graph[parity], h->stream));
      for (auto& r : h->runs) r.steps += kGraphSteps;
      done += kGraphSteps;
    } else {
      const int64_t chunk = std::min<int64_t>(n - done, kGraphSteps);
      const int rc = launch_steps(h, h->stream, chunk);
      if (rc) return rc;
      done += chunk;
    }
  }
  return LBM_CDE_OK;
}

int lbm_cde_steps_done(lbm_cde_handle h, int32_t run, int64_t* steps) {
  Run* r = get_run(h, run);
  if (!r || !steps) return fail(h, LBM_CDE_EINVAL, "steps_done: bad handle, run or pointer");
  *steps = r->steps;
  return LBM_CDE_OK;
}

int lbm_cde_moments(lbm_cde_handle h, int32_t run, double* phi_out) {
  Run* r = get_run(h, run);
  if (!r || !phi_out) return fail(h, LBM_CDE_EINVAL, "moments: bad handle, run or pointer");
  const RunArgs a = make_args(h, *r, r->cur);
  const unsigned blocks = (unsigned)((r->nodes + 255) / 256);
  if (r->dbl) hipLaunchKernelGGL(k_moments<double>, dim3(blocks), dim3(256), 0, h->stream, a, r->Q, phi_out);
  else if (r->half) hipLaunchKernelGGL(k_moments<__half>, dim3(blocks), dim3(256), 0, h->stream, a, r->Q, phi_out);
  else hipLaunchKernelGGL(k_moments<float>, dim3(blocks), dim3(256), 0, h->stream, a, r->Q, phi_out);
  HIP_TRY(h, hipGetLastError());
  return LBM_CDE_OK;
}

int lbm_cde_reduce(lbm_cde_handle h, int32_t run, int32_t kind, double x_ref, double* out) {
  Run* r = get_run(h, run);
  if (!r || !out) return fail(h, LBM_CDE_EINVAL, "reduce: bad handle, run or pointer");
  if (kind < LBM_CDE_RED_MASS || kind > LBM_CDE_RED_NONFINITE)
    return fail(h, LBM_CDE_EINVAL, "reduce: unknown kind %d", kind);
  if (kind == LBM_CDE_RED_XMOMENTS && !std::isfinite(x_ref))
    return fail(h, LBM_CDE_EINVAL, "reduce: x_ref is not finite");
  int rc = reduce_into(h, *r, kind, x_ref, r->red_out);
  if (rc) return rc;
  double res[4];
  unsigned long long fl[3] = {0, 0, 0};
  HIP_TRY(h, hipMemcpyAsync(res, r->red_out, sizeof res, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(fl, r->flags, sizeof fl, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  const unsigned long long over = fl[1], fast = r->uslot ? fl[2] : 0;
  if (kind == LBM_CDE_RED_NONFINITE) {
    out[0] = res[3];
    out[1] = out[2] = 0.0;
  } else {
    out[0] = res[0];
    out[1] = kind == LBM_CDE_RED_XMOMENTS ? res[1] : 0.0;
    out[2] = kind == LBM_CDE_RED_XMOMENTS ? res[2] : 0.0;
    if (res[3] != 0.0) return fail(h, LBM_CDE_ENONFINITE, "reduce: %g non-finite values in the state", res[3]);
  }
  if (over) return fail(h, LBM_CDE_EOVERFLOW, "reduce: 16-bit storage of run %d saturated", run);
  if (fast) return fail(h, LBM_CDE_EUNSTABLE, "reduce: a velocity field of run %d reached |u| >= 1/sqrt(3)", run);
  return LBM_CDE_OK;
}

int lbm_cde_reduce_noalloc(lbm_cde_handle h, int32_t run, int32_t kind, double x_ref, double* out) {
  Run* r = get_run(h, run);
  if (!r || !out) return fail(h, LBM_CDE_EINVAL, "reduce_noalloc: bad handle, run or pointer");
  if (kind < LBM_CDE_RED_MASS || kind > LBM_CDE_RED_NONFINITE)
    return fail(h, LBM_CDE_EINVAL, "reduce_noalloc: unknown kind %d", kind);
  if (kind == LBM_CDE_RED_XMOMENTS && !std::isfinite(x_ref))
    return fail(h, LBM_CDE_EINVAL, "reduce_noalloc: x_ref is not finite");
  const int64_t nb = std::max<int64_t>(1, (r->nodes + kNodesPerPartial - 1) / kNodesPerPartial);
  if (nb > kScratchPartials)
    return fail(h, LBM_CDE_EINVAL,
                "reduce_noalloc: run %d has %lld nodes; the static scratch holds the partials of at most %lld nodes",
                run, (long long)r->nodes, (long long)(kScratchPartials * kNodesPerPartial));
  const RunArgs a = make_args(h, *r, r->cur);
  double* partial = h->scratch_dev;  // every partial in [0, nb) is written before it is read
  if (r->dbl)
    hipLaunchKernelGGL(k_reduce_partial<double>, dim3((unsigned)nb), dim3(RED_THREADS), 0, h->stream, a, r->Q, kind,
                       x_ref, partial);
  else if (r->half)
    hipLaunchKernelGGL(k_reduce_partial<__half>, dim3((unsigned)nb), dim3(RED_THREADS), 0, h->stream, a, r->Q, kind,
                       x_ref, partial);
  else
    hipLaunchKernelGGL(k_reduce_partial<float>, dim3((unsigned)nb), dim3(RED_THREADS), 0, h->stream, a, r->Q, kind,
                       x_ref, partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, h->stream, (const double*)partial, (int)nb, out);
  HIP_TRY(h, hipGetLastError());
  return LBM_CDE_OK;
}

int lbm_cde_run_sampled(lbm_cde_handle h, int64_t n, int64_t every, double* hist, int64_t capacity) {
  if (!h) return fail_init(LBM_CDE_EINVAL, "run_sampled: null handle");
  if (!hist || every < 1 || n < 0 || n % every)
    return fail(h, LBM_CDE_EINVAL, "run_sampled: need hist != NULL, every >= 1 and n a multiple of every");
  const int64_t rows = n / every;
  if (h->sample_rows + rows > capacity)
    return fail(h, LBM_CDE_EINVAL, "run_sampled: history capacity %lld exceeded", (long long)capacity);
  const int64_t nr = (int64_t)h->runs.size();
  if (h->batched) {
    if (h->sample_every != every || h->sample_hist != hist) {
      for (auto& kv : h->sample_graphs) (void)hipGraphExecDestroy(kv.second);
      h->sample_graphs.clear();
      for (auto& kv : h->sample_fgraphs) (void)hipGraphExecDestroy(kv.second);
      h->sample_fgraphs.clear();
      h->sample_every = every;
      h->sample_hist = hist;
    }
    for (int64_t k = 0; k < rows; ++k) {
      const unsigned grid = batch_grid_at(h, h->global_steps);
      const bool fused = batch_fused_span(h, h->global_steps, every);
      const unsigned gridf = fused ? batch_fgrid_at(h, h->global_steps) : 0;
      hipGraphExec_t* gp;
      if (fused) gp = &h->sample_fgraphs[((uint64_t)gridf << 32) | grid];
      else gp = &h->sample_graphs[grid];
      hipGraphExec_t& g = *gp;
      if (!g) {
        const int rc = capture_batch(h, every, hist, grid, &g, gridf);
        if (rc) {
          if (fused) h->sample_fgraphs.erase(((uint64_t)gridf << 32) | grid);
          else h->sample_graphs.erase(grid);
          return rc;
        }
      }
      HIP_TRY(h, hipGraphLaunch(g, h->stream));
      advance_host_clock(h, every);
    }
    h->sample_rows += rows;
    return LBM_CDE_OK;
  }
  for (int64_t k = 0; k < rows; ++k) {
    int rc = lbm_cde_step(h, every);
    if (rc) return rc;
    for (int64_t i = 0; i < nr; ++i) {
      Run& r = h->runs[i];
      double x_ref = r.d.xref0 + r.d.xref_drift * (double)r.steps;
      x_ref -= (double)r.d.nx * std::floor(x_ref / (double)r.d.nx);
      rc = reduce_into(h, r, LBM_CDE_RED_XMOMENTS, x_ref, r.red_out);
      if (rc) return rc;
      HIP_TRY(h, hipMemcpyAsync(hist + ((h->sample_rows + k) * nr + i) * 3, r.red_out, 3 * sizeof(double),
                                hipMemcpyDeviceToDevice, h->stream));
    }
  }
  h->sample_rows += rows;
  return LBM_CDE_OK;
}

int lbm_cde_samples_written(lbm_cde_handle h, int64_t* rows) {
  if (!h || !rows) return fail(h, LBM_CDE_EINVAL, "samples_written: null argument");
  *rows = h->sample_rows;
  return LBM_CDE_OK;
}

int lbm_cde_relaxation_matrix(lbm_cde_handle h, int32_t run, double* S_out) {
  Run* r = get_run(h, run);
  if (!r || !S_out) return fail(h, LBM_CDE_EINVAL, "relaxation_matrix: bad handle, run or pointer");
  if (r->node_par) return fail(h, LBM_CDE_EINVAL, "relaxation_matrix: run has a per-node D field");
  relaxation_matrix_of(*r, S_out);
  return LBM_CDE_OK;
}

int lbm_cde_spectral_radius(const lbm_cde_run_desc* d, double* rho) {
  if (!d || !rho) return fail_init(LBM_CDE_EINVAL, "spectral_radius: null argument");
  int rc = validate(*d, 0);
  if (rc) return rc;
  Run r;
  r.d = *d;
  layout(r, nullptr);
  if ((rc = derive(r, 0)) || (rc = check_velocity(r, 0))) return rc;
  if (d->D_field || d->u_kind != LBM_CDE_U_CONST)
    return fail_init(LBM_CDE_EUNSUPPORTED, "spectral_radius: needs a constant D and a constant u");
  *rho = spectral_radius_of(r);
  return LBM_CDE_OK;
}

int lbm_cde_set_velocity(lbm_cde_handle h, int32_t run, const double* u) {
  Run* r = get_run(h, run);
  if (!r || !u) return fail(h, LBM_CDE_EINVAL, "set_velocity: bad handle, run or pointer");
  if (r->d.u_kind != LBM_CDE_U_FIELD || !r->uslot)
    return fail(h, LBM_CDE_EINVAL, "set_velocity: run %d was not initialised with a velocity field", run);
  hipLaunchKernelGGL(k_store_ptr, dim3(1), dim3(64), 0, h->stream, (const double**)r->uslot, u);
  HIP_TRY(h, hipGetLastError());
  return LBM_CDE_OK;
}

int lbm_cde_destroy(lbm_cde_handle h) {
  if (!h) return LBM_CDE_EINVAL;
  drop_graphs(h);
  if (h->capture) (void)hipStreamDestroy(h->capture);
  delete h;
  return LBM_CDE_OK;
}

int lbm_cde_tune(lbm_cde_handle h, int32_t trials) {
  if (!h) return fail_init(LBM_CDE_EINVAL, "tune: null handle");
  if (trials < 1) return fail(h, LBM_CDE_EINVAL, "tune: trials must be >= 1");
  if (h->batched) {
    const std::string key = batch_tune_key(h);
    const Variant off{64, 8, 2, true, 0, 0, 1};
    Variant v, v1;
    if (cache_lookup(key, v)) {
      if (v.fuse == 1 && find_batch(v)) {
        const int rc = apply_batch_variant(h, v, nullptr);
        return rc ? rc : apply_batch_fused(h, off);
      }
      if (v.fuse > 1 && cache_lookup(key + "/1", v1) && find_batch(v1) && find_batch_fused(h, v)) {
        const int rc = apply_batch_variant(h, v1, nullptr);
        return rc ? rc : apply_batch_fused(h, v);
      }
    }
    // one-step launches (kept for the blocks in which a budget ends), then
    // the multi-step ones, per step
    double best1 = 1e300;
    Variant best_v1 = h->batch_var;
    for (const Variant& c : batch_candidates()) {
      double ms = 0.0;
      int rc = apply_batch_variant(h, c, nullptr);
      if (!rc) rc = time_batch(h, trials, &ms);
      if (rc) return rc;
      if (ms < best1) {
        best1 = ms;
        best_v1 = c;
      }
    }
    int rc = apply_batch_variant(h, best_v1, nullptr);
    if (rc) return rc;
    double best = best1;
    Variant best_v = best_v1;
    for (const Variant& c : batch_fused_candidates(h)) {
      double ms = 0.0;
      rc = apply_batch_fused(h, c);
      if (!rc) rc = time_batch(h, trials, &ms, &c);
      if (rc) return rc;
      if (ms < best) {
        best = ms;
        best_v = c;
      }
    }
    cache_store(key, best_v, best);
    if (best_v.fuse > 1) cache_store(key + "/1", best_v1, best1);
    return apply_batch_fused(h, best_v.fuse > 1 ? best_v : off);
  }
  for (auto& r : h->runs) {
    const std::string key = tune_key(r);
    Variant v;
    Variant v1;
    if (cache_lookup(key, v) && find_step(r, v) &&
        (v.fuse == 1 || (cache_lookup(key + "/1", v1) && v1.fuse == 1 && find_step(r, v1)))) {
      r.var = v;
      r.var1 = v.fuse == 1 ? v : v1;
      continue;
    }
    // time every candidate (per step), then rank by the time of a captured
    // kGraphSteps-step block: a multi-step variant leaves kGraphSteps mod T
    // steps to the fastest one-step variant
    const std::vector<Variant> cands = run_candidates(r);
    std::vector<double> per_step(cands.size());
    double best1 = 1e300;
    Variant best_v1 = r.var1;
    for (size_t i = 0; i < cands.size(); ++i) {
      const int rc = time_variant(h, r, cands[i], trials, &per_step[i]);
      if (rc) return rc;
      if (cands[i].fuse == 1 && per_step[i] < best1) {
        best1 = per_step[i];
        best_v1 = cands[i];
      }
    }
    double best = 1e300;
    Variant best_v = r.var;
    for (size_t i = 0; i < cands.size(); ++i) {
      const int T = cands[i].fuse, left = kGraphSteps % T;
      const double block = per_step[i] * (kGraphSteps - left) + best1 * left;
      if (block / kGraphSteps < best) {
        best = block / kGraphSteps;
        best_v = cands[i];
      }
    }
    r.var = best_v;
    r.var1 = best_v1;
    cache_store(key, best_v, best);
    if (best_v.fuse != 1) cache_store(key + "/1", best_v1, best1);
  }
  drop_graphs(h);  // captured graphs hold the previous kernels
  return LBM_CDE_OK;
}

int lbm_cde_get_variant(lbm_cde_handle h, int32_t run, int32_t* out) {
  Run* r = get_run(h, run);
  if (!r || !out) return fail(h, LBM_CDE_EINVAL, "get_variant: bad handle, run or pointer");
  if (h->batched) {
    if (h->batch_fuse.fuse > 1) variant_out(h->batch_fuse, (int)h->batch_prefix_f.back(), out);
    else variant_out(h->batch_var, h->batch_grid, out);
    return LBM_CDE_OK;
  }
  Variant v = r->var;
  if (v.xcd == 2 && tile_rows(*r, v) % 8 != 0) v.xcd = 0;  // the launch falls back to the hardware order
  variant_out(v, 0, out);
  return LBM_CDE_OK;
}

int lbm_cde_variant_count(lbm_cde_handle h, int32_t run, int32_t* count) {
  Run* r = get_run(h, run);
  if (!r || !count) return fail(h, LBM_CDE_EINVAL, "variant_count: bad handle, run or pointer");
  *count = (int32_t)(h->batched ? batch_all_candidates(h).size() : run_candidates(*r).size());
  return LBM_CDE_OK;
}

int lbm_cde_variant_at(lbm_cde_handle h, int32_t run, int32_t index, int32_t* out) {
  Run* r = get_run(h, run);
  if (!r || !out) return fail(h, LBM_CDE_EINVAL, "variant_at: bad handle, run or pointer");
  const std::vector<Variant> c = h->batched ? batch_all_candidates(h) : run_candidates(*r);
  if (index < 0 || index >= (int32_t)c.size())
    return fail(h, LBM_CDE_EINVAL, "variant_at: index %d outside [0, %zu)", index, c.size());
  variant_out(c[index], c[index].grid, out);
  return LBM_CDE_OK;
}

int lbm_cde_set_variant(lbm_cde_handle h, int32_t run, const int32_t* v) {
  Run* r = get_run(h, run);
  if (!r || !v) return fail(h, LBM_CDE_EINVAL, "set_variant: bad handle, run or pointer");
  const Variant c{v[0], v[1], v[2], v[3] != 0, v[4], v[5], v[6]};
  if (h->batched) {
    if (c.fuse > 1) {
      if (!find_batch_fused(h, c))
        return fail(h, LBM_CDE_EINVAL, "set_variant: %dx%dx%d with %d steps per launch is not built for this batch",
                    c.bx, c.by, c.ny, c.fuse);
      return apply_batch_fused(h, c);
    }
    const int rc = apply_batch_variant(h, c, nullptr);
    return rc ? rc : apply_batch_fused(h, Variant{64, 8, 2, true, 0, 0, 1});
  }
  if (c.grid != 0 || c.xcd < 0 || c.xcd > 2 || !find_step(*r, c))
    return fail(h, LBM_CDE_EINVAL,
                "set_variant: variant %dx%dx%d nt=%d order=%d grid=%d steps=%d is not built for run %d", c.bx, c.by,
                c.ny, (int)c.nt, c.xcd, c.grid, c.fuse, run);
  if (c.xcd == 2 && tile_rows(*r, c) % 8 != 0)
    return fail(h, LBM_CDE_EINVAL, "set_variant: the row-interleaved order needs a multiple of 8 tile rows");
  r->var = c;
  if (c.fuse == 1) r->var1 = c;
  drop_graphs(h);
  return LBM_CDE_OK;
}

int lbm_cde_state_bytes(lbm_cde_handle h, int32_t run, size_t* bytes) {
  Run* r = get_run(h, run);
  if (!r || !bytes) return fail(h, LBM_CDE_EINVAL, "state_bytes: bad handle, run or pointer");
  *bytes = state_size(*r);
  return LBM_CDE_OK;
}

int lbm_cde_get_state(lbm_cde_handle h, int32_t run, void* dst) {
  Run* r = get_run(h, run);
  if (!r || !dst) return fail(h, LBM_CDE_EINVAL, "get_state: bad handle, run or pointer");
  const size_t pb = (size_t)r->Q * r->plane * r->elem;
  HIP_TRY(h, hipMemcpyAsync(dst, r->pop[r->cur], pb, hipMemcpyDeviceToDevice, h->stream));
  if (r->split)
    HIP_TRY(h, hipMemcpyAsync((char*)dst + align_up(pb), r->phi[r->cur], sizeof(float) * r->nodes,
                              hipMemcpyDeviceToDevice, h->stream));
  return LBM_CDE_OK;
}

int lbm_cde_set_state(lbm_cde_handle h, int32_t run, const void* src, int64_t steps) {
  Run* r = get_run(h, run);
  if (!r || !src || steps < 0) return fail(h, LBM_CDE_EINVAL, "set_state: bad handle, run, pointer or step count");
  if (h->batched) return fail(h, LBM_CDE_EUNSUPPORTED, "set_state: not available for batched handles");
  if (r->d.max_steps >= 0 && steps > r->d.max_steps)
    return fail(h, LBM_CDE_EINVAL, "set_state: step count beyond the run's budget");
  r->steps = steps;
  const size_t pb = (size_t)r->Q * r->plane * r->elem;
  HIP_TRY(h, hipMemcpyAsync(r->pop[r->cur], src, pb, hipMemcpyDeviceToDevice, h->stream));
  if (r->split)
    HIP_TRY(h, hipMemcpyAsync(r->phi[r->cur], (const char*)src + align_up(pb), sizeof(float) * r->nodes,
                              hipMemcpyDeviceToDevice, h->stream));
  return LBM_CDE_OK;
}

int lbm_cde_adjoint_scratch_bytes(lbm_cde_handle h, int32_t run, int32_t nsteps, size_t* bytes) {
  Run* r = get_run(h, run);
  int rc = check_adjoint_run(h, r);
  if (rc) return rc;
  if (nsteps < 1 || !bytes) return fail(h, LBM_CDE_EINVAL, "adjoint_scratch_bytes: nsteps < 1 or null pointer");
  *bytes = seg_layout(*r, nsteps).total;
  return LBM_CDE_OK;
}

int lbm_cde_adjoint_segment(lbm_cde_handle h, int32_t run, const void* ckpt, int32_t nsteps, void* seg,
                            const double* const* inj, void* mu, void* mu_tmp, double* grad) {
  Run* r = get_run(h, run);
  int rc = check_adjoint_run(h, r);
  if (rc) return rc;
  if (!ckpt || nsteps < 1 || !seg || !mu || !mu_tmp || !grad)
    return fail(h, LBM_CDE_EINVAL, "adjoint_segment: null buffer or nsteps < 1");
  const SegLayout L = seg_layout(*r, nsteps);
  char* segc = (char*)seg;
  char* P[2] = {segc, segc + L.state};
  float* part = (float*)(segc + L.part);
  const int K = nsteps;
  const double inv_kappa = 1.0 / r->kappa;
  // Launch plans.  A run periodic on both axes that spans the tile takes
  // several steps per launch (unless a snapshot falls inside the segment, or
  // LBM_CDE_ADJ_FUSED=0): forward chunks of T steps from the checkpoint, the
  // remaining steps one per launch; after the first reverse step (the one
  // that takes the injection, one per launch), reverse chunks of T steps down
  // to the segment's start, the rest one per launch.
  bool mid_inj = false;
  if (inj)
    for (int k = 0; k + 1 < K; ++k) mid_inj = mid_inj || inj[k];
  const Variant av = adjoint_multi_variant(*r);
  bool multi = K >= 2 && !mid_inj && !r->walls && fused_ok(*r, av);
  if (const char* e = std::getenv("LBM_CDE_ADJ_FUSED")) multi = multi && std::atoi(e) != 0;
  const int TA = multi ? av.fuse : 1;
  std::vector<std::pair<int, int>> fw, rv;  // (first / highest step, steps)
  for (int k = 0; k < K;) {
    const int n = k + TA <= K ? TA : 1;
    fw.emplace_back(k, n);
    k += n;
  }
  for (int k = K - 2; k >= 0;) {
    const int n = k - TA + 1 >= 0 ? TA : 1;
    rv.emplace_back(k, n);
    k -= n;
  }
  // forward launch: steps k .. k+n-1 from src into dst, v of every step
  // (the segment's last step stores no state)
  auto fwd = [&](int k, int n, const void* src, void* dst, hipStream_t s) {
    RunArgs a = make_args(h, *r, 0);
    a.src = src;
    a.dst = dst;
    char* v = segc + L.v + (size_t)k * L.v_step;
    const bool store = k + n < K;
    if (n == 1) {
      if (r->dbl) launch_step_v<double>(*r, a, v, store, s);
      else launch_step_v<float>(*r, a, v, store, s);
    } else if (r->dbl) {
      launch_fused_v<double, 64, 4, 2, 3>(a, v, (int64_t)L.v_step, store, s);
    } else {
      launch_fused_v<float, 64, 8, 2, 4>(a, v, (int64_t)L.v_step, store, s);
    }
  };
  // reverse launch: steps k, k-1, .., k-n+1: mu_{k+1} (cur) -> mu_{k-n+1}
  // (nxt).  FP32 storage gathers the segment's gradient in the FP32 partial
  // (set by the first reverse step) and folds it into the FP64 output in the
  // last reverse step.
  auto rev = [&](int k, int n, void* cur, void* nxt, const double* injk, hipStream_t s) {
    const RunArgs a = make_args(h, *r, 0);
    if (n == 1) {
      const AdjBufs b{segc + L.v + (size_t)k * L.v_step, cur, injk, nxt, grad, part};
      int gmode = GRAD_F64;
      if (!r->dbl && K >= 2) gmode = k == K - 1 ? GRAD_F32_SET : (k == 0 ? GRAD_F32_FOLD : GRAD_F32_ADD);
      if (r->dbl) launch_adjoint<double>(h, *r, a, b, gmode, inv_kappa, s);
      else launch_adjoint<float>(h, *r, a, b, gmode, inv_kappa, s);
    } else {
      const char* v_hi = segc + L.v + (size_t)k * L.v_step;
      const bool fold = k - n + 1 == 0;
      if (r->dbl)
        launch_fused_adj<double, 64, 4, 2, 3>(a, v_hi, (int64_t)L.v_step, cur, nxt, grad, part, inv_kappa, fold, s);
      else
        launch_fused_adj<float, 64, 8, 2, 4>(a, v_hi, (int64_t)L.v_step, cur, nxt, grad, part, inv_kappa, fold, s);
    }
  };
  // the forward launches after the first, from buffer P[1]
  auto fwd_rest = [&](hipStream_t s) {
    int p = 1;
    for (size_t j = 1; j < fw.size(); ++j) {
      fwd(fw[j].first, fw[j].second, P[p], P[p ^ 1], s);
      p ^= 1;
    }
  };
  // the reverse launches after the first, mu_{K-1} in mu_tmp; the result ends in mu
  auto rev_rest = [&](hipStream_t s) -> void* {
    void* cur = mu_tmp;
    void* nxt = mu;
    for (const auto& c : rv) {
      rev(c.first, c.second, cur, nxt, nullptr, s);
      std::swap(cur, nxt);
    }
    return cur;
  };
  const size_t sb = (size_t)r->Q * r->plane * r->elem;
  // Graphs: with K >= 2 and no injection before the segment's last step,
  // everything but the first forward launch (which reads the caller's
  // checkpoint) and the first reverse step (which reads the injection) has
  // the same arguments in every call with the same K and buffers: those two
  // are launched directly and the rest replayed from two captured graphs.
  bool graphs = K >= 2 && !mid_inj;
  if (const char* e = std::getenv("LBM_CDE_ADJ_GRAPHS")) graphs = graphs && std::atoi(e) != 0;
  if (!graphs) {
    fwd(fw[0].first, fw[0].second, ckpt, P[1], h->stream);
    fwd_rest(h->stream);
    rev(K - 1, 1, mu, mu_tmp, inj ? inj[K - 1] : nullptr, h->stream);
    void* cur = mu_tmp;
    void* nxt = mu;
    for (const auto& c : rv) {
      rev(c.first, c.second, cur, nxt, inj ? inj[c.first] : nullptr, h->stream);
      std::swap(cur, nxt);
    }
    if (cur != mu) HIP_TRY(h, hipMemcpyAsync(mu, cur, sb, hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(h, hipGetLastError());
    return LBM_CDE_OK;
  }
  auto graph = [&](int which, auto body) -> hipGraphExec_t {
    const auto key = std::make_tuple(run, K, (const void*)seg, (const void*)mu, (const void*)mu_tmp,
                                     (const void*)grad, which + 2 * TA);
    auto it = h->adj_graphs.find(key);
    if (it != h->adj_graphs.end()) return it->second;
    if (h->adj_graphs.size() >= kMaxAdjGraphs) {  // callers that change buffers every call
      if (hipStreamSynchronize(h->stream) != hipSuccess) return nullptr;
      for (auto& kv : h->adj_graphs) (void)hipGraphExecDestroy(kv.second);
      h->adj_graphs.clear();
    }
    if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    body(h->capture);
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    const hipError_t e = hipStreamEndCapture(h->capture, &g);
    if (e == hipSuccess && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess) h->adj_graphs[key] = x;
    if (g) (void)hipGraphDestroy(g);
    return x;
  };
  hipGraphExec_t ga = graph(0, [&](hipStream_t s) { fwd_rest(s); });
  hipGraphExec_t gb = graph(1, [&](hipStream_t s) {
    void* cur = rev_rest(s);
    if (cur != mu) (void)hipMemcpyAsync(mu, cur, sb, hipMemcpyDeviceToDevice, s);
  });
  if (!ga || !gb) return fail(h, LBM_CDE_EHIP, "adjoint_segment: graph capture failed");
  fwd(fw[0].first, fw[0].second, ckpt, P[1], h->stream);
  HIP_TRY(h, hipGraphLaunch(ga, h->stream));
  rev(K - 1, 1, mu, mu_tmp, inj ? inj[K - 1] : nullptr, h->stream);
  HIP_TRY(h, hipGraphLaunch(gb, h->stream));
  HIP_TRY(h, hipGetLastError());
  return LBM_CDE_OK;
}

int lbm_cde_adjoint_phi0(lbm_cde_handle h, int32_t run, const void* mu0, const double* inj0, double* dphi0) {
  Run* r = get_run(h, run);
  int rc = check_adjoint_run(h, r);
  if (rc) return rc;
  if (!mu0 || !dphi0) return fail(h, LBM_CDE_EINVAL, "adjoint_phi0: null buffer");
  const RunArgs a = make_args(h, *r, 0);
  const unsigned blocks = (unsigned)((r->nodes + 255) / 256);
  if (r->dbl) {
    if (r->walls)
      hipLaunchKernelGGL((k_adjoint_phi0_d2q9<double, true>), dim3(blocks), dim3(256), 0, h->stream, a,
                         (const double*)mu0, inj0, dphi0);
    else
      hipLaunchKernelGGL((k_adjoint_phi0_d2q9<double, false>), dim3(blocks), dim3(256), 0, h->stream, a,
                         (const double*)mu0, inj0, dphi0);
  } else {
    if (r->walls)
      hipLaunchKernelGGL((k_adjoint_phi0_d2q9<float, true>), dim3(blocks), dim3(256), 0, h->stream, a,
                         (const float*)mu0, inj0, dphi0);
    else
      hipLaunchKernelGGL((k_adjoint_phi0_d2q9<float, false>), dim3(blocks), dim3(256), 0, h->stream, a,
                         (const float*)mu0, inj0, dphi0);
  }
  HIP_TRY(h, hipGetLastError());
  return LBM_CDE_OK;
}

const char* lbm_cde_last_error(lbm_cde_handle h) { return h ? h->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
