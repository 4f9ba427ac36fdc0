/*
 * lbm_cde.h - C ABI of the MI355X (gfx950) modified-MRT lattice Boltzmann
 * solver for the anisotropic convection-diffusion equation
 *
 *     d_t phi + div(phi u) = div(D grad phi)                      (Eq. 1)
 *
 * following Huang & Wu, "A modified multiple-relaxation-time lattice
 * Boltzmann model for convection-diffusion equation".  One time step is the
 * fused collide-and-stream update of every node: moments m = M f (Eq. 11,
 * Eq. 12 / A.2), relaxation m' = m - S (m - m_eq) with the modified,
 * non-diagonal S of Eq. (31) / (A.5) and the equilibrium of Eq. (37) /
 * (A.3)-(A.4), back-transform f' = M^-1 m' (Eq. 14) and streaming (Eq. 5).
 * D enters through A, the flux block of S, as D = kappa (I - A/2) A^-1 with
 * kappa = 1/3 (Eq. 36, A.6).
 *
 * Units are lattice units: dx = dt = 1, node x has integer coordinates
 * 0..n-1 per axis.
 *
 * Memory and ownership
 *   The caller owns every byte of device memory: a workspace sized by
 *   lbm_cde_workspace_bytes(), the initial fields and every output buffer.
 *   The library never allocates or frees device memory.  Handles are host
 *   objects; one handle must not be used from two host threads at once.
 *   Host tables passed in a descriptor are copied during lbm_cde_init().
 *
 * Streams
 *   Every call enqueues its GPU work on the stream given to lbm_cde_init()
 *   (a hipStream_t; NULL = the null stream) and returns without waiting,
 *   except lbm_cde_init() (which waits for its initialisation), lbm_cde_reduce()
 *   (which copies results to host memory) and lbm_cde_tune() (which times
 *   launches); these wait for that stream.
 *
 * Errors
 *   Every function returns LBM_CDE_OK (0) or a negative status.  The text of
 *   the last error of a handle is returned by lbm_cde_last_error(h); errors
 *   of lbm_cde_init()/lbm_cde_workspace_bytes(), where no handle exists yet,
 *   are returned by lbm_cde_last_error(NULL) (per host thread).  A failed
 *   call leaves the simulation state as it was.
 */
#ifndef LBM_CDE_H
#define LBM_CDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_CDE_ABI_VERSION 2

/* ---- status codes -------------------------------------------------------- */
enum {
  LBM_CDE_OK = 0,
  LBM_CDE_EINVAL = -1,      /* bad argument: null pointer, size, enum, step count   */
  LBM_CDE_ENOTSPD = -2,     /* D (or a node of D_field) is not symmetric positive definite */
  LBM_CDE_EUNSTABLE = -3,   /* a rate outside (0, 2), |u| >= c_s = 1/sqrt(3), or a
                               linearised step that amplifies a Fourier mode           */
  LBM_CDE_EHIP = -4,        /* HIP runtime error; the runtime's message is kept      */
  LBM_CDE_ENONFINITE = -5,  /* a reduction met NaN or Inf in the state               */
  LBM_CDE_ENOSPC = -6,      /* workspace smaller than lbm_cde_workspace_bytes()       */
  LBM_CDE_EUNSUPPORTED = -7, /* a valid combination the library does not provide      */
  LBM_CDE_EOVERFLOW = -8     /* 16-bit storage saturated at least once (sticky)         */
};

/* ---- enumerations -------------------------------------------------------- */
/* Lattices: D2Q9 of Eq. (2) with M of Eq. (12); D3Q15 of Eq. (A.1) with M of
 * Eq. (A.2), velocities ordered as the columns of that M. */
enum { LBM_CDE_D2Q9 = 0, LBM_CDE_D3Q15 = 1 };

/* Storage precision of the populations (arithmetic is FP64 for FP64 and FP32
 * otherwise):
 *   FP64          f_i stored as double.
 *   FP32_SHIFTED  g_i = f_i - w_i phi_ref stored as float, w_i the weights of
 *                 the model's equilibrium at rest (D2Q9: 5/9, 1/18; D3Q15:
 *                 8/15, 1/30).  The collision is done exactly on g.
 *   FP16_SPLIT    per node phi (float) and the non-equilibrium part
 *                 f_i - f_i^eq(phi, u) of the populations (half, times a
 *                 power-of-two scale).  D2Q9, constant D only.
 *   FP16_SHIFTED  g_i = f_i - w_i phi_ref as half times a power-of-two scale
 *                 (the literal 16-bit form; far less accurate than SPLIT).
 * The 16-bit scale is fp16_scale, or (0) chosen at init as the power of two
 * that puts the largest stored magnitude (the non-equilibrium part after the
 * first step for SPLIT, the shifted equilibrium for SHIFTED) at about 1/256
 * of the half range.  Values that would exceed the half range are
 * saturated and make later reductions return LBM_CDE_EOVERFLOW. */
enum { LBM_CDE_FP64 = 0, LBM_CDE_FP32_SHIFTED = 1, LBM_CDE_FP16_SPLIT = 2, LBM_CDE_FP16_SHIFTED = 3 };

/* Boundary of one axis (both faces).  Walls sit halfway between the first
 * (last) node and its missing neighbour:
 *   PERIODIC     wrap-around.
 *   BOUNCE_BACK  a population whose source lies beyond the wall is the one
 *                that left the same node with the opposite velocity.
 *   SPECULAR     a mirror: only the velocity component normal to the wall is
 *                reversed, the population moves on along the wall; the
 *                halfway analog of the zero-flux plate rule f2 = f4,
 *                f5 = f8, f6 = f7 of Sec. 3.2.
 *   NODE_MIRROR  the paper's plate rule of Sec. 3.2 (f2 = f4, f5 = f8, f6 = f7
 *                on a bottom wall): the first and last nodes lie on the walls
 *                and each population arriving from outside equals its mirror
 *                image arriving at the same node.  D2Q9 only, on one axis with
 *                every other axis periodic, at least 2 nodes across.  Not a
 *                permutation, so no adjoint is built.  With D_xy = 0 and u
 *                mirror-symmetric about each plate (e.g. parallel to it) the
 *                run equals the even reflection of a periodic domain and
 *                conserves sum phi with the plate rows weighted 1/2. */
enum { LBM_CDE_PERIODIC = 0, LBM_CDE_BOUNCE_BACK = 1, LBM_CDE_SPECULAR = 2, LBM_CDE_NODE_MIRROR = 3 };

/* Collision model (Sec. 3): MRT_A is the paper's modified model (S of
 * Eq. 31, m_eq of Eq. 37) and the default; MRT_B1/B2/B3 are the unmodified
 * anisotropic model (S of Eq. 24) with the equilibria of Eq. (38), (39) and
 * (37).  The B models are D2Q9 only, FP64/FP32 storage, no adjoint. */
enum { LBM_CDE_MRT_A = 0, LBM_CDE_MRT_B1 = 1, LBM_CDE_MRT_B2 = 2, LBM_CDE_MRT_B3 = 3 };

/* Velocity field u(x):
 *   CONST      u_const[0..dim-1].
 *   SEPARABLE  u_c(x,y,z) = amp_c * X_c[x] * Y_c[y] * Z_c[z] per component c,
 *              from host tables (see u_tables).
 *   FIELD      per node, device FP64 array [dim][nz][ny][nx], copied (FP64)
 *              into the workspace at init (EUNSTABLE if |u| >= 1/sqrt(3)
 *              anywhere); lbm_cde_set_velocity() points the steps at a
 *              caller array whenever the flow changes in time.  The steps
 *              read the FP64 field (16 B per node in 2D, 24 B in 3D). */
enum { LBM_CDE_U_CONST = 0, LBM_CDE_U_SEPARABLE = 1, LBM_CDE_U_FIELD = 2 };

/* Rates s4, s6 (, s8) of the heat-flux moments, which the modified S
 * couples into the flux rows (Eq. 31, A.5); D does not depend on them.
 *   LAMBDA_MIN  all equal to the smallest eigenvalue of A (default; equals
 *               1/tau for isotropic D).
 *   PAPER       s4 = s_xx, s6 = s_yy (, s8 = s_zz) as in Sec. 3.1.
 *   EXPLICIT    heat_rates[]. */
enum { LBM_CDE_HEAT_LAMBDA_MIN = 0, LBM_CDE_HEAT_PAPER = 1, LBM_CDE_HEAT_EXPLICIT = 2 };

/* Reductions (all FP64).  Sums over nodes weight the nodes of an on-node
 * plate (NODE_MIRROR) by 1/2, the quadrature that the plate rule conserves;
 * every other node has weight 1. */
enum {
  LBM_CDE_RED_MASS = 0,      /* out[0] = sum_x phi(x)                                   */
  LBM_CDE_RED_XMOMENTS = 1,  /* out[0..2] = S0, S1, S2 of phibar(x) = sum over y, z of
                                phi, S_k = sum_x d^k phibar(x), d the minimum image of
                                x - x_ref in [-nx/2, nx/2) (Eq. 46-47)                  */
  LBM_CDE_RED_NONFINITE = 2  /* out[0] = number of stored values that are NaN or Inf    */
};

/* ---- run description ----------------------------------------------------- */
typedef struct lbm_cde_run_desc {
  int32_t lattice;          /* LBM_CDE_D2Q9 | LBM_CDE_D3Q15                           */
  int32_t precision;        /* LBM_CDE_FP64 | LBM_CDE_FP32_SHIFTED | LBM_CDE_FP16_SPLIT */
  int64_t nx, ny, nz;       /* nodes per axis, >= 1; nz must be 1 for D2Q9            */
  int32_t bc[3];            /* boundary kind per axis x, y, z                          */
  double D[6];              /* constant D: xx, yy, zz, xy, xz, yz (2D uses xx, yy, xy) */
  const double* D_field;    /* NULL, or device FP64 per-node D, components as D[]
                               (2D: xx, yy, xy; 3D: all six), layout [comp][nz][ny][nx] */
  int32_t u_kind;           /* LBM_CDE_U_*                                              */
  double u_const[3];
  const double* u_tables;   /* SEPARABLE: host, for c = 0..dim-1 in turn:
                               amp_c, X_c[nx], Y_c[ny], Z_c[nz]                         */
  const double* u_field;    /* FIELD: device FP64 [dim][nz][ny][nx]                     */
  int32_t heat_rule;        /* LBM_CDE_HEAT_*                                           */
  double heat_rates[3];     /* EXPLICIT: s4, s6, s8                                     */
  double rates[15];         /* diagonal rates by moment index; 0 = default.  D2Q9 reads
                               s1, s2 (default 1.1), s7, s8 (1.2); D3Q15 reads s1, s2
                               (1.1), s9..s14 (1.2).  s0 never matters (m0 = m0eq).     */
  double phi_ref;           /* background level of shifted / split storage              */
  double fp16_scale;        /* FP16_SPLIT: power-of-two scale of f_neq; 0 = automatic   */
  double xref0, xref_drift; /* sampled x-moments use x_ref(t) = xref0 + xref_drift * t  */
  int64_t max_steps;        /* per-run step budget (< 0: unlimited); a run that has
                               used it is left unchanged by further steps               */
  int32_t model;            /* LBM_CDE_MRT_A (0, default) | _MRT_B1 | _MRT_B2 | _MRT_B3    */
  int32_t skip_stability_check; /* 0 (default): a run with constant D and constant u whose
                               linearised step has a spectral radius above 1 is rejected
                               with EUNSTABLE (see lbm_cde_spectral_radius); 1: accept it
                               (e.g. to repeat a published set-up whose slow growth of
                               short waves stays below round-off over the run)          */
} lbm_cde_run_desc;

typedef struct lbm_cde* lbm_cde_handle;

/* Bytes of device workspace needed for nruns runs.  Returns the errors of
 * lbm_cde_init's checks of the descriptions that need no GPU (EINVAL,
 * ENOTSPD, EUNSTABLE, EUNSUPPORTED). */
int lbm_cde_workspace_bytes(const lbm_cde_run_desc* runs, int32_t nruns, size_t* bytes);

/* Von Neumann stability of the run described by d, which must have a
 * constant D and a constant u (EUNSUPPORTED otherwise): *rho receives an
 * upper bound (tight to about 1e-6) of the spectral radius of the linearised
 * step G(k) = diag(exp(-i k.e_j)) C over a 48^2 (D2Q9) or 10^3 (D3Q15) grid
 * of wave vectors k, C = I - M^-1 S (M - m_eq 1^T) the collision of
 * Eq. (10)-(14) with the run's S and equilibrium.  Fourier modes grow where
 * rho > 1; lbm_cde_init rejects runs with rho > 1 + 1e-5 unless
 * skip_stability_check is set.  Host only; no GPU is used. */
int lbm_cde_spectral_radius(const lbm_cde_run_desc* d, double* rho);

/* Set up nruns independent runs in the caller's workspace (device memory of
 * ws_bytes bytes, 256-byte aligned) and initialise every population to the
 * equilibrium of phi0 and u (collision leaves an equilibrium unchanged, so
 * this is the post-collision state at t = 0).  phi0 is a host array of nruns
 * device pointers, each to nx*ny*nz FP64 values (x fastest).  D and the
 * rates are mapped to S as in Eq. (31)/(A.5), A = (D/kappa + I/2)^-1.
 * Errors: EINVAL, ENOTSPD, EUNSTABLE, ENOSPC, EUNSUPPORTED, EHIP.  On error
 * *out is NULL. */
int lbm_cde_init(const lbm_cde_run_desc* runs, int32_t nruns, const double* const* phi0,
                 void* workspace, size_t ws_bytes, void* hip_stream, lbm_cde_handle* out);

/* Advance every run n >= 0 time steps (each stops at its max_steps).  Long
 * advances are replayed from a captured HIP graph.  EINVAL for n < 0. */
int lbm_cde_step(lbm_cde_handle h, int64_t n);

/* Steps taken so far by run `run`. */
int lbm_cde_steps_done(lbm_cde_handle h, int32_t run, int64_t* steps);

/* phi(x) = sum_i f_i(x) (Eq. 8) of run `run`, as FP64 into the device buffer
 * phi_out of nx*ny*nz values, whatever the storage precision. */
int lbm_cde_moments(lbm_cde_handle h, int32_t run, double* phi_out);

/* FP64 reduction `kind` (LBM_CDE_RED_*) of run `run` into host memory out
 * (3 doubles).  x_ref is used by XMOMENTS only.  Waits for the stream.
 * Returns ENONFINITE (with out filled) when MASS or XMOMENTS met NaN/Inf, and
 * EOVERFLOW (with out filled) when 16-bit storage of the run has saturated. */
int lbm_cde_reduce(lbm_cde_handle h, int32_t run, int32_t kind, double x_ref, double* out);

/* For callers that cannot allocate memory or wait for the GPU (code under
 * HIP graph capture, tight serving loops): the reduction of lbm_cde_reduce,
 * enqueued on the handle's stream without waiting and without allocating.
 * out is a device buffer of 4 doubles that receives S0, S1, S2 (S1 = S2 = 0
 * unless kind is XMOMENTS; S0 = sum phi) and the number of non-finite stored
 * values, for every kind; nothing is reported through the return status
 * about the state (no ENONFINITE, no EOVERFLOW).  The partial sums live in a
 * static device array of the library, one per GPU, held until the process
 * ends (1 MiB: room for runs of up to 536,870,912 nodes; larger runs return
 * EINVAL).  Every call on one GPU uses the same array: calls whose work can
 * overlap on that GPU (other streams, other host threads) race and must be
 * ordered by the caller.  Errors: EINVAL. */
int lbm_cde_reduce_noalloc(lbm_cde_handle h, int32_t run, int32_t kind, double x_ref, double* out);

/* Advance n steps and, after every `every` steps, append the XMOMENTS
 * (S0, S1, S2) of each run, taken about x_ref(t) of that run, to the device
 * history buffer hist (FP64, [capacity][nruns][3]).  Sampling continues the
 * history where the previous call stopped; EINVAL if it would overflow
 * capacity.  n must be a multiple of every. */
int lbm_cde_run_sampled(lbm_cde_handle h, int64_t n, int64_t every, double* hist, int64_t capacity);

/* Number of history rows written so far by lbm_cde_run_sampled(). */
int lbm_cde_samples_written(lbm_cde_handle h, int64_t* rows);

/* The relaxation matrix S of run `run` (constant D only), row-major Q x Q,
 * into host memory S_out (Q*Q doubles); Q = 9 or 15.  Eq. (31) / (A.5) for
 * MRT_A, Eq. (24) for the MRT_B models. */
int lbm_cde_relaxation_matrix(lbm_cde_handle h, int32_t run, double* S_out);

/* Make the device FP64 array u [dim][nz][ny][nx] the velocity field of run
 * `run` (initialised with u_kind FIELD; Eq. 1 with u = u(x, t)).  The steps
 * read u itself, no copy is made: the caller keeps u valid and unchanged
 * until every step enqueued before the next lbm_cde_set_velocity of this run
 * (or lbm_cde_destroy) has run.  Each step relaxes the populations it
 * arrives at with the field current when the step is enqueued: the field set
 * before the call that takes a run from step n-1 to step n is u(x, t_n).
 * Enqueued on the handle's stream (no wait); captured graphs need no
 * rebuild.  A step that meets |u| >= 1/sqrt(3) at a node marks the run, and
 * the next lbm_cde_reduce of the run returns EUNSTABLE.  EINVAL if the run
 * has no velocity field or an argument is NULL. */
int lbm_cde_set_velocity(lbm_cde_handle h, int32_t run, const double* u);

/* Launch variants.  A variant is seven integers: block x, block y, rows per
 * thread, streaming stores (0/1), block order (0: hardware order, 1: each
 * XCD takes a contiguous range of tiles, 2: tile rows interleaved over the 8
 * XCDs with all x-tiles of a row on one XCD), for a batched handle
 * (several D2Q9 runs in one FP64 or FP32 precision, stepped by one persistent
 * launch over a flat list of block-x-wide row tiles) the number of blocks
 * of that launch (0: one block per tile; otherwise each block walks every
 * grid-th tile), and the number of steps one launch takes.  More than one
 * step per launch is built for D2Q9 FP64/FP32 MRT-A or MRT-B3 runs periodic
 * in x, and periodic or bounded by walls in y, whose periodic axes span the
 * tile (block x by block y times rows per thread nodes) plus that many steps
 * minus one nodes on each side (nx and ny below 2^24, a population plane
 * below 4 GiB): the launch keeps the
 * intermediate steps of a tile and its halo in LDS (Eq. 5: a population
 * moves one node per step), so the state crosses HBM once per launch; the
 * steps left over when a call's count is not a multiple go one per launch.
 * A run that can take several steps per launch starts with 4 (64 x 24
 * tiles in FP32 where the grid allows them, else 64 x 16; 64 x 8 in FP64),
 * any other with one.  A batched handle has
 * one variant for all its runs; the run index only has to be valid.  Results
 * are bitwise the same for every variant. */

/* Autotuner: time `trials` launches of every compiled variant (those listed
 * by lbm_cde_variant_at) and keep, per run, the one that takes a 32-step
 * block (the captured-graph length) in the least time, the steps a
 * multi-step variant leaves over going to the fastest one-step variant
 * (kept for them), or once for a batched handle the fastest.  Each timed launch reads the current state and overwrites
 * only the other population buffer, so the simulation state is unchanged.
 * If the environment variable LBM_CDE_TUNE_CACHE names a file, results are
 * looked up there (keyed by GPU architecture, lattice, precision, grid and
 * boundaries, and for a batch by every run's grid, boundaries and budget)
 * and new ones appended.  Waits for the stream.  EINVAL for trials < 1. */
int lbm_cde_tune(lbm_cde_handle h, int32_t trials);

/* The launch variant of run `run` into out[0..6] (layout above; out[5] is
 * the launch's actual number of blocks on a batched handle, else 0).  The
 * environment variables LBM_CDE_TILE = "BXxBYxNY[xSTEPS]", LBM_CDE_TILE3,
 * LBM_CDE_NT, LBM_CDE_XCD, LBM_CDE_TILE16 = "BXxBY[xNT[xORDER]]" and
 * LBM_CDE_BATCH = "BX[xNT[xGRID]]", read by lbm_cde_init(), fix the initial
 * variant of D2Q9 FP64/FP32, D3Q15, FP16_SPLIT runs and batches. */
int lbm_cde_get_variant(lbm_cde_handle h, int32_t run, int32_t* out);

/* Number of compiled launch variants of run `run` (the tuner's candidates). */
int lbm_cde_variant_count(lbm_cde_handle h, int32_t run, int32_t* count);

/* Candidate `index` (0 <= index < count) of run `run` into out[0..6].
 * EINVAL for an index out of range. */
int lbm_cde_variant_at(lbm_cde_handle h, int32_t run, int32_t index, int32_t* out);

/* Make v[0..6] the launch variant of run `run` (of the whole batch on a
 * batched handle).  Captured graphs are rebuilt on the next step.  EINVAL
 * if the variant is not compiled for the run (a block count must be 0 for a
 * run stepped alone, >= 0 for a batch; the row-interleaved order needs a
 * multiple of 8 tile rows).  Waits for the stream on a batched handle. */
int lbm_cde_set_variant(lbm_cde_handle h, int32_t run, const int32_t* v);

/* ---- state access (checkpoints) ------------------------------------------ */

/* Bytes of one population state of run `run` (Q planes in storage precision,
 * planes laid out as in the workspace). */
int lbm_cde_state_bytes(lbm_cde_handle h, int32_t run, size_t* bytes);

/* Copy the current state of run `run` to the device buffer dst
 * (lbm_cde_state_bytes bytes).  Async on the stream. */
int lbm_cde_get_state(lbm_cde_handle h, int32_t run, void* dst);

/* Overwrite the state of run `run` with src and set its step count to
 * `steps` (a restart from a checkpoint).  EUNSUPPORTED on batched handles
 * (several D2Q9 runs of one precision), whose runs share one step clock. */
int lbm_cde_set_state(lbm_cde_handle h, int32_t run, const void* src, int64_t steps);

/* ---- discrete adjoint (D2Q9, FP64 or FP32 storage) ------------------------
 * The step is linear in the populations, p_{t+1} = C(D) Pi p_t with Pi the
 * streaming permutation (Eq. 5 with the wall rules) and C the collision of
 * Eq. (10)-(14) with the modified S of Eq. (31).  For a loss L of the phi
 * snapshots the adjoint recursion is lambda_t = Pi^T C^T lambda_{t+1} +
 * dL/dp_t and dL/dD = sum_t lambda_{t+1}^T (dC/dD) Pi p_t; the library keeps
 * mu_t = C^T lambda_{t+1} between reverse steps.  D enters S through
 * A = (D/kappa + I/2)^-1 (Eq. 36).  The heat-flux rates must be EXPLICIT
 * (fixed); otherwise EUNSUPPORTED.  All buffers are device memory. */

/* Bytes of the scratch `seg` of lbm_cde_adjoint_segment for nsteps steps:
 * two states (the recomputation's ping-pong pair), the two values
 * v = (n3 + s4 n4 / 2, n5 + s6 n6 / 2) per node and step that the reverse
 * steps need from the forward pass (storage precision), and an FP32 gradient
 * partial of three values per node. */
int lbm_cde_adjoint_scratch_bytes(lbm_cde_handle h, int32_t run, int32_t nsteps, size_t* bytes);

/* Reverse sweep over one checkpoint segment of nsteps = K >= 1 steps,
 * t0 .. t0+K.  ckpt: the state p_t0 (lbm_cde_get_state layout).  seg:
 * scratch of lbm_cde_adjoint_scratch_bytes(h, run, K) bytes; the segment is
 * recomputed forward from ckpt into it (bitwise the run's own steps).  inj:
 * NULL, or a host array of K device pointers, inj[k] = dL/dphi at step
 * t0+k+1 (FP64 per node, x fastest) or NULL.  mu: in mu_{t0+K} (all zero for
 * the last segment), out mu_{t0}; mu_tmp: scratch of the same size (both
 * state-sized, storage precision).  grad: FP64 [3][ny][nx], components xx,
 * yy, xy of dL/dD at every node (for a constant D their sum over nodes),
 * accumulated (+=).  With FP32 storage the contributions of the segment's
 * steps are summed in FP32 (each is an FP32 product) and added to grad once;
 * that sum adds a relative error of at most about K * 6e-8 of the sum of
 * their magnitudes.  The run's own state is not touched. */
int lbm_cde_adjoint_segment(lbm_cde_handle h, int32_t run, const void* ckpt, int32_t nsteps, void* seg,
                            const double* const* inj, void* mu, void* mu_tmp, double* grad);

/* dL/dphi0 (FP64 per node) from mu_0 and dL/dphi at t = 0 (inj0, may be
 * NULL), through the equilibrium initialisation f(0) = f_eq(phi0, u). */
int lbm_cde_adjoint_phi0(lbm_cde_handle h, int32_t run, const void* mu0, const double* inj0, double* dphi0);

/* Release the handle (host memory only; the workspace stays the caller's). */
int lbm_cde_destroy(lbm_cde_handle h);

/* Text of the last error of h (NULL: of the last failed init on this thread). */
const char* lbm_cde_last_error(lbm_cde_handle h);

#ifdef __cplusplus
}
#endif
#endif /* LBM_CDE_H */
