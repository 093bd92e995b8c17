/*
 * lbmhpde.h -- C ABI of the MI355X (gfx950) library for the general lattice
 * Boltzmann (LBGK) model of Shi, He and Guo for 1D nonlinear PDEs
 *
 *     d_t phi + sum_{k=1..m} alpha_k d_x^k Pi_k(phi) = 0,  alpha_1 = 1, m <= 6
 *
 * (Sec. II.A, eq. NPDE).  One time step of the model (Sec. II.A, eq. LBE) is
 *     phi   = sum_j f_j                                   (eq. moments)
 *     f_eq  = M_q^{-1} Pi_bar(phi)                        (Sec. III.A/B)
 *     f*_j  = f_j - (f_j - f_eq_j) / tau                  (eq. LBE)
 *     f_j(x + e_j dx) = f*_j(x)                           (eq. LBE)
 * on the D1Q5 (e = 0, 1, -1, 2, -2) or D1Q7 (e = 0, +-1, +-2, +-3) lattice,
 * or on D1Q4 (e = 1, -1, 2, -2) / D1Q6 (e = +-1, +-2, +-3) without a rest
 * velocity, which Sec. III allows for orders 3 / 5 (M_q^{-1} is then the exact
 * inverse of the moment matrix M[k][j] = e_j^k; these lattices carry a
 * checkerboard mode that grows unless a diffusive term is large enough --
 * lbm_stability reports it),
 * with Pi_bar_0 = phi, Pi_bar_1 = Pi_1/c, Pi_bar_k = (Pi_k0 + beta_k Pi_k)/c^k,
 * c = dx/dt, beta_k = alpha_k / (dt^{k-1} tau_k) (eq. taus and Sec. III.C) and
 * the auxiliary moments Pi_k0 of Sec. II.C-F.
 *
 * Conventions for every entry point:
 *  - Every call returns an lbm_status; no C++ exception crosses the ABI.
 *  - Descriptors are validated on the host before any device work; a call
 *    that fails validation changes nothing.
 *  - Host arrays passed in are owned by the caller and copied before return.
 *  - A handle is not thread safe; distinct handles are independent.
 *  - `stream` arguments are hipStream_t values (NULL = the null stream).
 *    Work is enqueued on that stream; `*_read_*`, `*_sum_*` and `*_save_*`
 *    synchronise it.
 *  - State layout on the device: structure of arrays, f[j][x] with the
 *    population index j in the paper's velocity order and row stride
 *    lbm_row_stride(n) elements; FP64 (double) or, for the FP32 precisions,
 *    float deviations g = f - f_rest from a per-problem rest equilibrium.
 */
#ifndef LBMHPDE_H
#define LBMHPDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARG = 1,   /* bad pointer, size, m/q mismatch, tau <= 1/2, degree > 4 ... */
  LBM_ERR_UNSUPPORTED = 2,   /* a valid request this build does not implement */
  LBM_ERR_SINGULAR_TAU = 3,  /* |tau_k| ~ 0 where beta_k or a correction A_k0 needs 1/tau_k */
  LBM_ERR_OUT_OF_MEMORY = 4, /* device allocation failed or caller buffer too small */
  LBM_ERR_DEVICE = 5,        /* a HIP runtime call failed */
  LBM_ERR_NONFINITE = 6,     /* the state holds NaN or Inf (instability) */
  LBM_ERR_BUSY = 7,          /* serving: request not admitted yet / not finished */
  LBM_ERR_TIMEOUT = 8        /* a device-side wait for a cooperating workgroup (the previous step
                                chunk of a resident job, a neighbouring slab's halo) gave up: the
                                kernel ended without advancing that instance as asked; its state
                                is not a solution.  Never seen unless the GPU stalls a workgroup
                                for seconds (or lbm_batch_test_stall forces it) */
} lbm_status;

/* Boundaries.  Periodic: x_i = x0 + i dx, i = 0..n-1, node n-1 neighbours node 0.
   The bounded kinds (the exact-solution boundaries of Sec. IV) take a grid that
   includes both end points and reset the outer layers after every step from
   values the caller supplies (lbm_advance_bounded): DIRICHLET_EQ sets
   f = f_eq(phi*) there, DIRICHLET_NEE sets f = f_eq(phi*) + (f - f_eq(phi)) of
   the first interior node (non-equilibrium extrapolation). */
typedef enum { LBM_BC_PERIODIC = 0, LBM_BC_DIRICHLET_EQ = 1, LBM_BC_DIRICHLET_NEE = 2 } lbm_bc;
/* LBM_F64: FP64 state and arithmetic.  LBM_F32_DEV: the state is stored in
   FP32 as the deviation g = f - f_rest from the equilibrium of a rest state
   phi_rest (the mean of phi0, conserved on a periodic grid); the zeroth
   moment is summed and the relaxation evaluated in FP64.  LBM_F32_DEV_ARITH32:
   the same storage with the relaxation polynomials evaluated in FP32 (the
   zeroth moment still summed in FP64). */
typedef enum { LBM_F64 = 0, LBM_F32_DEV = 1, LBM_F32_DEV_ARITH32 = 2 } lbm_precision;
/* Auxiliary moments: LBM_AM_CORRECTED propagates the A_40 / A_50 parts of the
   fourth and fifth moments into Pi_50, Pi_60 and A_60 (required for the O(eps^m)
   recovery claimed in Sec. II.E-F when beta_2 != 0); LBM_AM_PAPER uses
   eqs. (Pi5), (Pi6) and A_60 exactly as printed.  Identical when beta_2 = 0. */
typedef enum { LBM_AM_CORRECTED = 0, LBM_AM_PAPER = 1 } lbm_am;

/* Problem descriptor (Sec. II.A eq. NPDE; Sec. III).  Plain data; layout fixed. */
typedef struct {
  int32_t m;             /* PDE order 1..6; 0 = highest k with alpha[k] != 0 */
  int32_t q;             /* 4, 5, 6 or 7; 0 = 5 if m <= 4 else 7 (Sec. III); needs q >= m + 1 */
  int32_t scheme;        /* 1 = all q moments (default, 0 is read as 1); 2 = top moment Pi_bar_{q-1} = 0 */
  int32_t am;            /* lbm_am */
  double alpha[7];       /* alpha[2..6]; alpha[0], alpha[1] ignored (alpha_1 = 1) */
  int32_t pi_deg[7];     /* Pi_k(phi) = sum_{d <= pi_deg[k]} pi_coef[k][d] phi^d, k = 1..6;
                            -1 = absent (Pi_k = 0); degree <= 4 */
  double pi_coef[7][5];
  int64_t n;             /* nodes on the periodic grid, n >= q */
  double dx, dt, tau;    /* lattice speed c = dx/dt (Sec. II.A); tau > 1/2 */
  int32_t bc;            /* lbm_bc */
  int32_t prec;          /* lbm_precision */
  /* Non-polynomial Pi_k (Sec. III.C: the families with real powers beta u^n u_x,
     alpha_2 (u^p)_xx, alpha_3 (u^q)_xxx): for k = 1..6 with pi_terms[k] > 0,
       Pi_k(phi) = sum_{i < pi_terms[k]} pi_gcoef[k][i] phi^pi_gexp[k][i]
     replaces pi_deg / pi_coef[k].  At most 4 terms; every exponent is 0 or in
     [1, 8].  A model whose equilibrium has non-integer powers of phi needs
     phi >= 0 (lbm_load_phi rejects a negative phi0; a state that turns
     negative becomes non-finite and is reported as LBM_ERR_NONFINITE); its
     equilibrium may use at most 4 distinct fractional parts of the exponents
     and integer degree 11 within each (LBM_ERR_UNSUPPORTED otherwise), and
     LBM_F32_DEV_ARITH32 is not available for it.  pi_terms[k] = 0 (a zeroed
     tail): the polynomial fields apply. */
  int32_t pi_terms[7];
  int32_t pi_pad_;
  double pi_gexp[7][4];
  double pi_gcoef[7][4];
} lbm_desc;

typedef struct lbm_problem_s* lbm_problem;
typedef struct lbm_batch_s* lbm_batch;
typedef struct lbm_server_s* lbm_server;

const char* lbm_status_str(lbm_status s);
const char* lbm_version(void);

/* Elements per population row for n nodes (rows are padded for alignment). */
int64_t lbm_row_stride(int64_t n);

/* Host-only validation of a descriptor (the checks lbm_create performs). */
lbm_status lbm_validate(const lbm_desc* d);

/* Host-only: the collapsed equilibrium polynomials f_eq_j(phi) = sum_d
   G[j*(D+1) + d] phi^d, j = 0..q-1, built once per problem in 113-bit
   arithmetic and rounded to double (the per-node steps a2-a3:
   Pi_k(phi) -> Pi_k0(phi) -> Pi_bar -> M_q^{-1} Pi_bar).  `cap` is the
   capacity of G in doubles; *q_out, *degree_out receive q and D. */
lbm_status lbm_coefficients(const lbm_desc* d, double* G, int32_t cap, int32_t* q_out,
                            int32_t* degree_out);
/* Models with non-integer powers of phi (pi_terms) make lbm_coefficients
   return LBM_ERR_UNSUPPORTED; this host-only call covers every model:
     f_eq_j(phi) = sum_{c < F} phi^nu[c] sum_d G[(c*q + j)*(D+1) + d] phi^d,
   nu[0] = 0 and nu[c] in (0, 1) the distinct fractional parts of the
   exponents (a polynomial model has F = 1).  nu holds at least 4 doubles;
   `cap` is the capacity of G in doubles; *classes_out, *q_out, *degree_out
   receive F, q and D. */
lbm_status lbm_coefficients_general(const lbm_desc* d, double* nu, double* G, int32_t cap, int32_t* classes_out,
                                    int32_t* q_out, int32_t* degree_out);

/* Host-only linear (von Neumann) pre-check: the largest growth factor per step
   over Fourier modes kappa in (0, pi] of the scheme linearised about uniform
   states in [phi_min, phi_max] (the eigenvalues of the q x q one-step symbol
   E(kappa)((1 - 1/tau) I + (1/tau) f_eq'(phi) 1^T)), and its steps-th power.
   Physical growth (e.g. the unstable band of Kuramoto-Sivashinsky) is
   included; a value far above 1 on the grid scale marks parameters (dx, dt,
   tau) on which the scheme itself amplifies.  For a model with non-integer
   powers of phi, phi_min must be > 0 (LBM_ERR_INVALID_ARG otherwise). */
lbm_status lbm_stability(const lbm_desc* d, double phi_min, double phi_max, int64_t steps,
                         double* growth_per_step, double* amplification);

/* ---- single problem ---------------------------------------------------- */

/* Device bytes of the state of one problem (f, one buffer; plus scratch). */
lbm_status lbm_required_bytes(const lbm_desc* d, size_t* bytes);

/* Create a problem.  dev_buf (nullable) is caller-owned device memory of at
   least lbm_required_bytes bytes that must outlive the handle; otherwise the
   library allocates and owns its buffers. */
lbm_status lbm_create(const lbm_desc* d, void* stream, void* dev_buf, size_t buf_bytes,
                      lbm_problem* out);

/* f := f_eq(phi) at every node (initial distribution, Sec. IV).  phi holds n
   doubles on the host (phi_on_device = 0) or the device (1). */
lbm_status lbm_load_phi(lbm_problem h, const double* phi, int phi_on_device);

/* Advance `steps` time steps (asynchronous on the problem's stream).
   INVALID_ARG for a bounded problem (those advance with lbm_advance_bounded). */
lbm_status lbm_advance(lbm_problem h, int64_t steps);

/* For callers that cannot allocate device memory (tight serving loops,
   harnesses that forbid hipMalloc): lbm_create + lbm_load_phi + lbm_advance +
   lbm_read_phi of one periodic problem in one call that allocates nothing.
   phi0 and phi are caller-owned device arrays of d->n doubles (they may be the
   same array); f := f_eq(phi0), `steps` steps on the LDS-resident path, phi :=
   sum_j f_j -- the kernels of lbm_advance, so the result is bitwise the one of
   the handle calls.  Every device buffer besides phi0 and phi (coefficient and
   job tables, queue words, status flags, the state) lies in one fixed array of
   272 KiB per GPU, allocated with the library's code object and held until the
   process ends.  Limits: the state must fit one workgroup's LDS and 256 KiB
   (d->n <= 8192; e.g. at most 4096 nodes for FP64 D1Q5, 2925 for FP64 D1Q7,
   8192 for FP32 D1Q5, 5851 for FP32 D1Q7), else LBM_ERR_INVALID_ARG before any
   device work.  Calls that overlap on one GPU (other streams, other host
   threads) share that array and race; calls on one stream are ordered.  The
   array keeps the last call's contents; each call clears what must start at
   zero.  Synchronises the stream; returns LBM_ERR_NONFINITE if phi holds
   NaN/Inf, LBM_ERR_INVALID_ARG for a bounded problem, a non-finite phi0 or, with
   non-integer powers of phi, a negative one. */
lbm_status lbm_advance_noalloc(const lbm_desc* d, const double* phi0, int64_t steps, double* phi, void* stream);

/* Bounded problems (bc = LBM_BC_DIRICHLET_EQ or _NEE; Sec. IV): advance `steps`
   steps; after step s (s = 1..steps) the `layers` outer nodes at each end are
   reset from the exact solution phib[(s-1) * 2 layers + k]: k < layers holds
   nodes 0..layers-1, k >= layers nodes n-layers..n-1, at time s dt after the
   steps already taken.  phib is a host array of steps * 2 * layers doubles,
   copied before the call returns.  layers = 0 means q/2; layers must lie in
   [q/2, 32] and n >= 2 layers + 2.  A state that fits one workgroup's LDS
   advances on the resident path (the layers reset in LDS after every step;
   steps <= 2^30), otherwise -- or with lbm_set_path(LBM path 1) -- each step
   is one fused collide+stream launch through HBM plus one boundary launch;
   both give bitwise equal results.  INVALID_ARG for a periodic problem or bad
   sizes. */
lbm_status lbm_advance_bounded(lbm_problem h, int64_t steps, const double* phib, int32_t layers);

/* Exact solutions of travelling-wave form for the bounded kinds, evaluated on
   the device (the closed forms of the examples of Sec. IV: the tanh
   polynomials of the Burgers-type equations, sech^2 and sech^4 solitary
   waves, the KdV-Burgers front; also K(2,2) compactons):
     phi*(x, t) = a + b h(z)^p + d h(z)^r,  z = k (x - xc - c t),
   h = 1/cosh (SECH), tanh (TANH), 1/(1 + e^z) (LOGISTIC), or cos on
   |z| <= pi/2 and 0 outside (COS, the compacton support); x = x_first + i dx
   at node i; t = t0 + s dt after step s (t0: the time of the state when the
   call starts).  p, r >= 0 (integers for TANH, whose h may be negative);
   every parameter finite.  Plain data; layout fixed. */
typedef enum { LBM_WAVE_SECH = 1, LBM_WAVE_TANH = 2, LBM_WAVE_LOGISTIC = 3, LBM_WAVE_COS = 4 } lbm_wave_shape;
typedef struct {
  int32_t shape;         /* lbm_wave_shape */
  int32_t pad_;
  double a, b, p;        /* phi* = a + b h(z)^p + d h(z)^r */
  double d, r;
  double k, xc, c;       /* z = k (x - xc - c t) */
  double x_first;        /* x of node 0 */
  double t0;             /* time of the state when the call starts */
} lbm_wave;

/* lbm_advance_bounded with the boundary values phi*(x_b, t0 + s dt) of `w`
   computed on the device (one row of 2 layers values per step, in device
   memory the library owns) instead of copied from the host; same paths,
   same layer rules.  INVALID_ARG for an invalid wave (shape, p, a non-finite
   parameter) before any device work. */
lbm_status lbm_advance_bounded_wave(lbm_problem h, int64_t steps, const lbm_wave* w, int32_t layers);

/* The boundary rows lbm_advance_bounded_wave(h, steps, w, layers) would use,
   evaluated on the device and copied to out (host, steps * 2 layers doubles,
   in the phib layout of lbm_advance_bounded).  Synchronises. */
lbm_status lbm_wave_rows(lbm_problem h, int64_t steps, const lbm_wave* w, int32_t layers, double* out);

/* phi = sum_j f_j (zeroth moment, FP64) into n doubles on the host or device.
   Synchronises; returns LBM_ERR_NONFINITE (after writing) if any value is NaN/Inf,
   LBM_ERR_TIMEOUT (after writing) if a device wait of an advance gave up. */
lbm_status lbm_read_phi(lbm_problem h, double* out, int out_on_device);

/* FP64 sum over the grid of phi (conserved on a periodic grid). */
lbm_status lbm_sum_phi(lbm_problem h, double* total);

/* Checkpoint / resume of the complete state (f and the step count). */
lbm_status lbm_state_bytes(lbm_problem h, size_t* bytes);
lbm_status lbm_save_f(lbm_problem h, void* host_buf, size_t bytes);
lbm_status lbm_load_f(lbm_problem h, const void* host_buf, size_t bytes);

/* Kernel path for lbm_advance: 0 = automatic (resident when the state fits one
   workgroup's LDS, else temporal blocking), 1 = HBM streaming (one fused
   collide+stream launch per step), 2 = on-chip resident (all steps of a call
   in one launch; UNSUPPORTED if the state does not fit), 3 = temporal blocking
   (tiles of the grid with halos advance several steps per launch in LDS),
   4 = slabs (the grid split over workgroups that are resident together for
   all steps of the call and exchange halos every few steps; the automatic
   choice for grids larger than one workgroup's LDS, with temporal blocking
   as the fallback when the slabs do not fit one launch). */
lbm_status lbm_set_path(lbm_problem h, int32_t path);

/* Temporal blocking and slab parameters: steps per launch, or per halo
   exchange of the slab path (rounded up to even there) (0 = automatic, <= 4096),
   and the number of workgroups per CU the 160 KiB LDS is split for
   (0 = automatic, <= 8), which sets the tile and slab width. */
lbm_status lbm_set_tiling(lbm_problem h, int32_t steps_per_launch, int32_t wgs_per_cu);

/* Device time of the kernels of the last lbm_advance, in ms (HIP events). */
lbm_status lbm_last_advance_ms(lbm_problem h, float* ms);

lbm_status lbm_destroy(lbm_problem h);

/* ---- batches of independent problems ------------------------------------ */

/* `count` descriptors (any mix of q, degree, precision and n). */
lbm_status lbm_batch_create(const lbm_desc* descs, int32_t count, void* stream, lbm_batch* out);

/* phi0[i] points to descs[i].n host doubles. */
lbm_status lbm_batch_load_phi(lbm_batch b, const double* const* phi0);

/* Advance instance i by steps[i] (>= 0) steps, all instances in persistent
   launches; asynchronous.  steps == NULL advances nothing.  The launches of
   one call (one per lattice, precision and variant on each path) run side by
   side on up to 16 internal streams forked from and joined back to the
   batch's stream, as many as the hardware queues HIP gives the process
   (GPU_MAX_HW_QUEUES, 4 by default; streams that share a queue run one after
   another): launches in order of estimated duration, longest first, each to
   the stream with the least estimated work so far. */
lbm_status lbm_batch_advance(lbm_batch b, const int64_t* steps);
/* Bounded instances of a batch (Sec. IV boundaries, as lbm_advance_bounded):
   every instance advances `steps` (<= 2^30) steps; bounded instance i resets
   its `layers` outer nodes at each end after every step from phib[i] (host,
   steps * 2 * layers doubles, copied before the call returns; ignored and may
   be NULL for periodic instances).  layers = 0 means the largest q/2 of the
   bounded instances; layers in [that, 32], n >= 2 layers + 2.  Bounded
   instances run on the LDS-resident path: LBM_ERR_UNSUPPORTED if one does not
   fit a workgroup's LDS or another path is forced.  A tau sweep of one bounded
   problem is one call. */
lbm_status lbm_batch_advance_bounded(lbm_batch b, int64_t steps, const double* const* phib, int32_t layers);
/* As lbm_batch_advance_bounded with bounded instance i's rows evaluated on the
   device from waves[i] (see lbm_wave; entries of periodic instances are
   ignored).  waves: host array of one lbm_wave per instance. */
lbm_status lbm_batch_advance_bounded_wave(lbm_batch b, int64_t steps, const lbm_wave* waves, int32_t layers);

/* phi of instance i into n host doubles; *inst_status (nullable) receives
   LBM_OK, LBM_ERR_NONFINITE or LBM_ERR_TIMEOUT for that instance alone.
   Synchronises. */
lbm_status lbm_batch_read_phi(lbm_batch b, int32_t i, double* out, lbm_status* inst_status);

/* Device time of the kernels of the last lbm_batch_advance, in ms. */
lbm_status lbm_batch_last_advance_ms(lbm_batch b, float* ms);

/* Planner: 0 = automatic, 1 = force HBM streaming for every instance,
   2 = force on-chip resident (fails with UNSUPPORTED if an instance does not fit),
   3 = force temporal blocking, 4 = force slabs (see lbm_set_path). */
lbm_status lbm_batch_set_path(lbm_batch b, int32_t path);

/* Temporal blocking parameters of a batch (see lbm_set_tiling). */
lbm_status lbm_batch_set_tiling(lbm_batch b, int32_t steps_per_launch, int32_t wgs_per_cu);

/* Persistent resident launch parameters of a batch.  max_workgroups caps the
   grid of each resident launch (0 = as many as the GPU holds at once, at most
   2048); chunks fixes the number of step chunks each job's steps are split
   into (0 = automatic: 1 when every job gets its own workgroup, otherwise
   about 16 queue items per workgroup with chunks of >= 256 steps; at most 64).
   A chunk reloads its job's state from HBM and writes it back, so results do
   not depend on either value (bitwise).  INVALID_ARG outside those ranges. */
lbm_status lbm_batch_set_resident(lbm_batch b, int32_t max_workgroups, int32_t chunks);

/* Streams the launches of one lbm_batch_advance are spread over: 0 =
   automatic (the hardware queues HIP gives the process, GPU_MAX_HW_QUEUES,
   at most 16), 1..16 = that many.  More streams than hardware queues only
   chain launches behind each other; results do not depend on the value
   (bitwise).  INVALID_ARG outside 0..16. */
lbm_status lbm_batch_set_lanes(lbm_batch b, int32_t lanes);

/* Autotuner result: the planner settings it kept (as set by lbm_batch_set_path,
   lbm_batch_set_tiling and lbm_batch_set_resident) and the measured rates. */
typedef struct {
  int32_t path;                        /* 0 automatic, 1 HBM streaming, 3 temporal blocking */
  int32_t tile_steps;                  /* steps per tiled launch (0 = automatic) */
  int32_t tile_wgs;                    /* tiled workgroups per CU (0 = automatic) */
  int32_t res_chunks;                  /* resident step chunks (0 = automatic) */
  int32_t candidates;                  /* configurations timed */
  int32_t pad_;
  double best_node_updates_per_s;      /* device rate of the kept settings */
  double default_node_updates_per_s;   /* device rate of the automatic settings */
} lbm_tuning;

/* Times candidate planner settings -- the temporal-blocking tile (steps per
   launch, workgroups per CU), the resident step chunking and, for at most 16
   instances, HBM streaming instead of LDS residency -- on a copy of the batch
   advanced probe_steps per candidate (best of two passes after a warm-up),
   and applies the fastest to b (a candidate must beat the best so far by 3%).
   The state of b is not changed.  Needs device memory for a second copy of the
   batch (OUT_OF_MEMORY otherwise); synchronises b's stream; UNSUPPORTED for the
   batch behind a server; INVALID_ARG for a batch with bounded instances (they
   advance only with their boundary rows).  out may be NULL. */
lbm_status lbm_batch_autotune(lbm_batch b, int64_t probe_steps, lbm_tuning* out);

/* Test hook for the error path of the bounded device waits, which a healthy
   GPU never takes.  what = 1: in the next advances, the first step chunk of the
   first job of the first resident launch is taken from the queue but never run
   (when the launch has more than one chunk), so the wait of its second chunk
   gives up; what = 2: the first slab of the first slab launch never raises its
   flag, so its neighbours' halo waits give up (and then its own).  Either way
   every kernel ends and the instances concerned report LBM_ERR_TIMEOUT.
   wait_us: the limit of every bounded wait in microseconds (0 = automatic:
   10 s plus 20 us per step of the work waited for).  what = 0 with wait_us = 0
   restores normal operation.  INVALID_ARG for what outside [0, 2] or a
   negative wait. */
lbm_status lbm_batch_test_stall(lbm_batch b, int32_t what, int64_t wait_us);

lbm_status lbm_batch_destroy(lbm_batch b);

/* ---- serving: continuous batching of solve requests -------------------- */

/* A server owns two mirrored device arenas of budget_bytes each (the state and
   the second buffer of the tiled path), at most max_slots active requests of
   at most max_n nodes, and advances active requests block_steps steps per
   scheduling round.  Requests share one planner pass per round, so their work
   overlaps on the device. */
lbm_status lbm_server_create(void* stream, size_t budget_bytes, int32_t max_slots, int64_t max_n,
                             int32_t block_steps, lbm_server* out);

/* Queue a request (validated now, with every check admission makes: the model,
   its kernel variant, phi0 finite and, for non-integer powers of phi, >= 0;
   phi0 is copied).  *id >= 1.  A request whose state alone exceeds the budget
   is refused with LBM_ERR_OUT_OF_MEMORY. */
lbm_status lbm_server_submit(lbm_server s, const lbm_desc* d, const double* phi0, int64_t steps,
                             int64_t* id);

/* One round: admit queued requests in arrival order while a slot and arena
   space are free (f := f_eq(phi0)), advance every active request by
   min(block_steps * r, remaining) steps, where r in [1, 8] is the cost per
   step (lattice size x polynomial degree) of the costliest active request over
   the request's own, retire finished requests (phi read out, space released).
   Synchronises the stream.  Counts are optional outputs. */
lbm_status lbm_server_step(lbm_server s, int32_t* active, int32_t* queued, int32_t* retired);

/* Continuous batching without blocking the caller: if the round launched by
   the previous call is still running on the device, return at once with
   *running = 1; otherwise retire the requests it completed, admit queued
   requests (as lbm_server_step) and launch the next round asynchronously
   (*running = 1 if one was launched).  Call it often (a serving loop calls it
   between arrivals); requests submitted while a round runs are admitted as
   soon as it ends.  lbm_server_step and lbm_server_pump may be mixed: a step
   first finishes a round a pump left running.  Counts are optional outputs
   (active: admitted and not retired; queued: waiting for admission). */
lbm_status lbm_server_pump(lbm_server s, int32_t* running, int32_t* active, int32_t* queued, int32_t* retired);

/* Host timing of a retired request (steady clock): *queue_s from submission to
   admission, *service_s from admission to retirement.  LBM_ERR_BUSY while it
   is queued or running; optional outputs. */
lbm_status lbm_server_timing(lbm_server s, int64_t id, double* queue_s, double* service_s);

/* Result of request id: LBM_OK with phi in out[0..n) (n >= the request's node
   count) and its own status (LBM_OK / LBM_ERR_NONFINITE / LBM_ERR_TIMEOUT)
   once retired; LBM_ERR_BUSY while queued or running.  A request whose
   admission fails on the device (its state could not be initialised) is
   retired at once with that status and no phi (out is not written); the
   queue behind it goes on.  A result is delivered once. */
lbm_status lbm_server_poll(lbm_server s, int64_t id, double* out, int64_t n, lbm_status* inst_status);

/* Totals since creation: node updates advanced, device ms of the rounds, free arena bytes. */
lbm_status lbm_server_stats(lbm_server s, double* node_updates, double* device_ms, size_t* free_bytes);

lbm_status lbm_server_destroy(lbm_server s);

#ifdef __cplusplus
}
#endif

#endif /* LBMHPDE_H */
