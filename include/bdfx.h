/*
 * bdfx.h -- C ABI of the MI355X batched stiff-kinetics BDF integrator.
 *
 * Problem (arXiv 2405.01713, Balos et al.): operator splitting (Sec. 3.1,
 * Eq. (7)) leaves one independent ODE system per grid cell,
 *     y' = R(y; k_c) + F_c,   y(t0) = y0_c,   t in [t0, t_out],
 * with R mass-action chemistry and F a constant forcing.  Every cell is
 * integrated by a variable-order (1..5), variable-step BDF method (Sec. 2,
 * Eq. (1)) with its own step and order control: local error in the WRMS norm
 * of Sec. 2, Eq. (3) with tolerances rtol and atol_i; modified Newton with the
 * stopping test of Sec. 2, Eq. (4); Newton matrix I - gamma J from the analytic
 * Jacobian, factored by dense LU with partial pivoting (Table 1, approaches
 * 2A/2B; Sec. 4.1.4).  Options: the Jacobian by difference quotients
 * (approaches 3A/3B), or an inexact Newton iteration with matrix-free GMRES
 * (approaches 1A/1B; Sec. 2, Eqs. (5) and (6)).
 *
 * Conventions
 *  - All d_* arguments are device pointers owned by the caller.  The library
 *    borrows them from bdfx_bind() until the next bind or bdfx_destroy().  The
 *    library owns only the context and the mechanism tables; it allocates no
 *    device memory after bdfx_bind() (the paper's memory-pool lesson,
 *    Sec. 4.3.1), so bdfx_integrate() and bdfx_perturb() can be captured in a
 *    HIP graph.
 *  - State layout is cell-major ("CY" ordering of Sec. 4.1.2):
 *    y[cell * ldy + species], FP64.
 *  - Every function returns BDFX_OK (0) or a negative call status; the text of
 *    the last error is available from bdfx_last_error().  Failures of single
 *    cells never fail a call: they are reported per cell in d_status.
 *  - A context is bound to one device and one HIP stream and is not
 *    thread-safe.  Work is enqueued on the context's stream; only
 *    bdfx_stats_summary() and bdfx_bind() synchronise it.
 */
#ifndef BDFX_H
#define BDFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BDFX_MAX_SPECIES 64
#define BDFX_MAX_ORDER 5
#define BDFX_SLOTS 3
#define BDFX_MAX_MECH 8
#define BDFX_GMRES_MAXL 10 /* largest Krylov dimension of bdfx_options.gmres_maxl */
#define BDFX_MAX_LOCKSTEP 16 /* largest lock-step batch of bdfx_options.lockstep */

/* call status */
#define BDFX_OK 0
#define BDFX_EINVAL (-1)    /* invalid argument */
#define BDFX_EWORKSPACE (-2) /* workspace smaller than bdfx_plan() asked for */
#define BDFX_EHIP (-3)      /* HIP runtime error */
#define BDFX_EORDER (-4)    /* functions called in the wrong order */
#define BDFX_EUNSUPPORTED (-5)

/* per-cell status (CVODE-like) */
#define BDFX_CELL_SUCCESS 0
#define BDFX_CELL_TOO_MUCH_WORK (-1)  /* max_steps reached before t_out */
#define BDFX_CELL_ERR_FAILURE (-3)    /* repeated error-test failures or step too small */
#define BDFX_CELL_CONV_FAILURE (-4)   /* repeated Newton convergence failures */
#define BDFX_CELL_SETUP_FAILURE (-6)  /* singular Newton matrix twice in one step */
#define BDFX_CELL_NONFINITE (-9)      /* non-finite y0, T or right-hand side */
#define BDFX_CELL_RECORD_FULL (-10)   /* adjoint step record capacity exceeded */

typedef struct bdfx_ctx_s *bdfx_ctx;
typedef struct bdfx_mech_s *bdfx_mech;

/* Mass-action mechanism, host arrays, copied by bdfx_mech_create().
 * Reaction r: sum_l y[reac[r][l]]  <=>  sum_l y[prod[r][l]] with up to three
 * slots per side (-1 = empty, a repeated species is a stoichiometric
 * coefficient), net rate q_r = k_f prod y_reac - k_r prod y_prod and
 * f_i = F_i + sum_r nu_ir q_r.  Rate constants are Arrhenius,
 * k_f = exp(lnA_r - EaR_r / T_c) * kscale_c[r], k_r = k_f exp(-lnK_r).
 *
 * Non-isothermal cells (cv and u0 given; the Arrhenius terms of Sec. 3.1
 * with the temperature evolving, as in the zero-dimensional constant-energy
 * reactor of Sec. 4.1.3): the
 * temperature is state entry n_species of every cell of this mechanism
 * (y[cell][n_species], so the state has n_species + 1 entries and ldy, atol
 * and the workspace count it), T_c is not used, the rate constants are
 * re-evaluated from the state's temperature at every right-hand side, and
 * dT/dt = F_T - sum_i u_i(T) f_i / sum_i cv_i y_i with u_i(T) = u0_i + cv_i T
 * (adiabatic, constant volume).  Step recording (bdfx_adjoint) is not
 * available for such mechanisms. */
typedef struct {
  int32_t n_species;   /* S, 1..BDFX_MAX_SPECIES */
  int32_t n_reactions; /* R >= 1 */
  const int32_t *reac; /* [R][3] */
  const int32_t *prod; /* [R][3] */
  const double *lnA;   /* [R] */
  const double *EaR;   /* [R] activation temperature (K), or NULL (all zero) */
  const double *lnK;   /* [R] ln equilibrium constant, or NULL (irreversible) */
  const double *cv;    /* [S] heat capacities (> 0), or NULL (isothermal) */
  const double *u0;    /* [S] species energies at T = 0, with cv (NULL iff cv is) */
} bdfx_mech_desc;

/* Scheduler for bdfx_options.scheduler */
#define BDFX_SCHED_STATIC 0 /* one lane group per cell, grid covers every cell */
#define BDFX_SCHED_QUEUE 1  /* persistent waves pop cells from an atomic work queue */
#define BDFX_SCHED_FUSED 2  /* as BDFX_SCHED_QUEUE, and a batch of two mechanisms runs in
                               one launch: each block holds waves for both, the larger
                               mechanism's cells start first and the smaller one's run
                               beside them and in the tail (the load balancing of uneven
                               cells, Sec. 2 and Sec. 4.1.1).  Applies to isothermal
                               A + B <=> C mechanisms on the direct solver with the analytic
                               Jacobian whose padded sizes have a compiled pair (53 with 9);
                               otherwise the bins are launched one after the other.  One
                               cell per wave.  bdfx_autotune() also times the one launch
                               against the per-mechanism launches on its samples and keeps
                               the faster (bdfx_tuning.fused).  Results equal the
                               BDFX_SCHED_QUEUE ones bit for bit. */

typedef struct {
  double rtol;           /* relative tolerance of Eq. (3), > 0 */
  const double *atol;    /* host [atol_len] absolute tolerances, copied */
  int32_t atol_len;      /* 1 (all species) or >= S_max (per species index) */
  int32_t max_order;     /* 1..5 (0 = 5) */
  int32_t max_steps;     /* per cell per integrate call (0 = 5000) */
  int32_t lu_precision;  /* 64 (default) or 32: Newton-matrix factor/solve in FP32 */
  int32_t scheduler;     /* BDFX_SCHED_* */
  int32_t record_steps;  /* > 0: record up to this many accepted steps per cell
                            for bdfx_adjoint(); 0: no recording */
  int32_t waves_per_block; /* 0 = library choice / autotuned value */
  int32_t blocks_per_cu;   /* persistent grid: resident blocks per CU (0 = auto) */
  int32_t queue_chunk;     /* cells per work-queue pop (0 = 1) */
  int32_t waves_per_simd;  /* register budget of the integrator kernel: 0 = compiler's
                              choice, 3, 4 or 5 = code built for that many resident waves
                              per SIMD (at most 168 / 128 / 96 VGPRs, spilling if needed;
                              the one-launch pair of BDFX_SCHED_FUSED has no 5-wave code
                              and then runs as two launches) */
  int32_t cells_per_wave;  /* 0 or 1; 2 = each half-wave integrates its own cell
                              (mechanisms of at most 32 species) */
  int32_t jacobian;        /* BDFX_JAC_ANALYTIC (0) or BDFX_JAC_DQ (1): Newton matrix from
                              forward difference quotients, one right-hand side per state
                              entry (Table 1, approaches 3A/3B) */
  int32_t gmres_maxl;      /* 0: modified Newton with the direct solve (above).
                              1..BDFX_GMRES_MAXL: inexact Newton (Table 1, approaches 1A/1B):
                              each Newton system (I - gamma J(y_m)) x = b at the current
                              iterate is solved by GMRES with at most this many Krylov
                              vectors, on the system scaled by the error weights (Sec. 2,
                              Eq. (5), S1 = S2 = diag(w), no preconditioner), with
                              J v = (f(y_m + sigma v) - f(y_m)) / sigma, sigma = 1/||v||_wrms,
                              and the stopping test of Eq. (6), c_l = 0.05, on the
                              residual norm from the Givens rotations.  No matrix is formed:
                              jacobian must be BDFX_JAC_ANALYTIC, lu_precision and
                              cells_per_wave = 2 do not apply, record_steps must be 0.  A
                              solve that misses its tolerance after the first Newton
                              iteration (or does not reduce the residual at all) is a
                              convergence failure. */
  int32_t lockstep;        /* 0: every cell has its own step size and order (default).
                              1..BDFX_MAX_LOCKSTEP: the paper's lock-step batches (Sec. 2):
                              each mechanism's cells, in bin order, are cut into consecutive
                              batches of this many cells; the cells of a batch share one
                              step size and order, and every WRMS norm of Eqs. (3)-(4) runs
                              over the batch vector (N = cells x state entries).  The batch
                              succeeds or fails as a whole; each of its cells reports the
                              batch's status and counters.  Direct solver with the analytic
                              Jacobian, isothermal mechanisms, no step recording; one wave
                              per cell, so the batch's LDS (cells x the per-wave area) must
                              fit 64 KiB, else bdfx_bind() fails with BDFX_EUNSUPPORTED.
                              The launch shape is fixed: one block of this many waves per
                              batch; bdfx_autotune() times nothing and reports it, and
                              bdfx_set_tuning() does not change it. */
  int32_t max_err_test_fails; /* error-test failures within one step that fail the cell with
                                 BDFX_CELL_ERR_FAILURE (0 = 7); the cell keeps its last
                                 accepted state and time (the accept/reject logic of Sec. 2) */
  int32_t max_conv_fails;     /* Newton convergence failures within one step that fail the cell
                                 with BDFX_CELL_CONV_FAILURE (0 = 10) */
  int32_t checkpoint_every;   /* with record_steps > 0: 0 stores every accepted step for
                                 bdfx_adjoint() (record_steps x (S_max + 2) doubles per cell).
                                 K > 0 stores instead the integrator's whole state at every
                                 K-th accepted step (ceil(record_steps / K) checkpoints of
                                 20 + 8 S doubles per cell, S the largest mechanism size
                                 padded to a compiled size), and bdfx_adjoint() reruns
                                 each K-step segment from its checkpoint with the same step
                                 code before sweeping it backwards: the gradient equals the
                                 full record's bit for bit, for about one more forward run of
                                 work.  Needs lu_precision 64 and the analytic Jacobian;
                                 cells run one per wave; bdfx_get_record_layout() does not
                                 apply (BDFX_EUNSUPPORTED). */
} bdfx_options;

#define BDFX_JAC_ANALYTIC 0
#define BDFX_JAC_DQ 1

/* Per-cell statistics written by bdfx_integrate() (56 bytes, [N]). */
typedef struct {
  int32_t status;  /* BDFX_CELL_* */
  int32_t nst;     /* accepted steps */
  int32_t nfe;     /* right-hand-side evaluations */
  int32_t nni;     /* Newton iterations */
  int32_t nsetups; /* Jacobian evaluations + LU factorisations */
  int32_t netf;    /* error-test failures */
  int32_t ncfn;    /* Newton convergence failures */
  int32_t q_last;  /* order at the end */
  int32_t nli;     /* GMRES iterations (each one right-hand side, counted in nfe too) */
  int32_t ncfl;    /* GMRES solves that did not reach their tolerance */
  double h_last;   /* step size at the end */
  double t_reached;/* t_out on success, else time of the last accepted step */
} bdfx_cell_stats;

/* Batch summary from bdfx_stats_summary(). */
typedef struct {
  int64_t n_cells;
  int64_t n_success;
  int64_t n_failed;
  int64_t nst, nfe, nni, nsetups, netf, ncfn; /* totals over cells */
  int64_t max_nst;
  int64_t status_count[11]; /* count of cells with status == -k, k = 0..10 */
  int64_t nli, ncfl;        /* totals over cells */
} bdfx_summary;

/* Create a context on HIP device `device` enqueueing on `hip_stream`
 * (hipStream_t, NULL = default stream).  *out receives the handle. */
int bdfx_create(bdfx_ctx *out, int device, void *hip_stream);
/* Change the stream later work is enqueued on. */
int bdfx_set_stream(bdfx_ctx ctx, void *hip_stream);
/* Release the context and everything it owns (not the bound buffers). */
int bdfx_destroy(bdfx_ctx ctx);
/* Text of the last error of ctx (or of the last failed create when ctx is
 * NULL).  The pointer stays valid until the next call on the context. */
const char *bdfx_last_error(bdfx_ctx ctx);

/* Upload a mechanism (derives the RHS gather lists and the analytic-Jacobian
 * term lists from the stoichiometry).  Synchronous. */
int bdfx_mech_create(bdfx_ctx ctx, const bdfx_mech_desc *desc, bdfx_mech *out);
int bdfx_mech_destroy(bdfx_mech mech);
/* Replace the mechanism's ln pre-exponential factors lnA_r (the parameters
 * of the Arrhenius terms of Sec. 3.1 that bdfx_adjoint() differentiates) by
 * d_lnA, a device array [R] of FP64 owned by the caller: one device-to-device
 * copy enqueued on the context's stream (no allocation, no synchronisation),
 * so that a bound context can integrate again with new parameters.  Later
 * bdfx_integrate() calls on the stream use the new values.  Errors:
 * BDFX_EINVAL for NULL arguments, BDFX_EHIP if the copy cannot be
 * enqueued. */
int bdfx_mech_set_lnA(bdfx_mech mech, const double *d_lnA);

/* Fix the batch shape and options; *workspace_bytes receives the device
 * workspace size bdfx_bind() needs (queue counters, cell bins, adjoint
 * records).  mechs[m] is the mechanism of cells with cell_mech == m.
 * Planning and binding separate all allocation from the integration, so that
 * the device memory comes from the caller's pool once and later calls
 * allocate nothing (the memory-pool lesson of Sec. 4.3.1).  Host-only.
 * Errors: BDFX_EINVAL for n_cells < 1, n_mech outside 1..BDFX_MAX_MECH,
 * NULL mechanisms or option values outside their documented ranges;
 * BDFX_EUNSUPPORTED for option combinations the kernels do not provide. */
int bdfx_plan(bdfx_ctx ctx, int64_t n_cells, int32_t n_mech, const bdfx_mech *mechs,
              const bdfx_options *opts, size_t *workspace_bytes);

/* Bind caller-owned device buffers:
 *   d_workspace [workspace_bytes]   scratch owned by the caller, >= plan size
 *   d_y         [N][ldy] in/out     initial state on entry, final state after
 *                                   bdfx_integrate() (updated in place);
 *                                   ldy >= S_max, entries beyond a cell's S are
 *                                   never read or written
 *   d_cell_mech [N] or NULL         mechanism index of every cell (NULL: all 0)
 *   d_T         [N] or NULL         temperature (NULL: zero activation terms)
 *   d_kscale    [N][ldk] or NULL    multiplicative per-reaction rate scale
 *   d_forcing   [N][ldy] or NULL    constant forcing F
 *   d_status    [N] out             per-cell BDFX_CELL_* status
 *   d_stats     [N] out or NULL     per-cell statistics
 * Reads d_cell_mech once (synchronously) to build the per-mechanism cell
 * bins in the workspace.  The state stays where the application keeps it, in
 * its cell-major ("CY", Sec. 4.1.2) array; no copy is made (Sec. 4.3.1 on
 * device-resident data).  Errors: BDFX_EORDER before bdfx_plan();
 * BDFX_EWORKSPACE if workspace_bytes is below the planned size; BDFX_EINVAL
 * for NULL d_y / d_status / d_workspace, ldy below the largest state length,
 * or a cell_mech entry outside 0..n_mech-1. */
int bdfx_bind(bdfx_ctx ctx, void *d_workspace, size_t workspace_bytes, double *d_y, int32_t ldy,
              const int32_t *d_cell_mech, const double *d_T, const double *d_kscale,
              int32_t ldk, const double *d_forcing, int32_t *d_status,
              bdfx_cell_stats *d_stats);

/* Integrate every bound cell from t0 to t_out (t_out > t0): one outer
 * (splitting) step of Sec. 3.1, Eq. (7), for every cell's ODE system
 * y' = R(y) + F by the BDF method of Sec. 2, Eq. (1), each cell with its own
 * step size and order.  d_y holds y(t_out) afterwards (or the last accepted
 * state of a failed cell, whose d_status entry is negative).  Enqueue only
 * (no allocation, no synchronisation; capturable in a HIP graph).  Errors:
 * BDFX_EINVAL unless t_out > t0 (both finite); BDFX_EORDER before
 * bdfx_bind(); BDFX_EHIP if a launch fails. */
int bdfx_integrate(bdfx_ctx ctx, double t0, double t_out);

/* Outer-step perturbation between splitting steps: for every cell and
 * species, y_i <- max(0, y_i (1 + amplitude u)), u uniform in [-1, 1) from
 * SplitMix64 (Steele, Lea & Flood 2014) keyed by (seed, outer_step, cell,
 * species), then the cell is rescaled so that sum_i w_i y_i keeps its value
 * (w = d_weights of the cell's mechanism, see bdfx_mech_set_weights()).
 * Enqueue only. */
int bdfx_perturb(bdfx_ctx ctx, uint64_t seed, int64_t outer_step, double amplitude);

/* Typical-value absolute tolerances (Sec. 4.1.3, Eq. (9)).  For every
 * mechanism m and species i < S_m, the typical value ytyp[m][i] is
 * 0.5 * (min + max) of y[c][i] over the bound cells c of mechanism m (their
 * current states), and atol[m][i] = eta * ytyp[m][i], or eta where ytyp is
 * not positive (a species absent everywhere; the paper's default typical
 * value 1).  A NaN state entry makes ytyp NaN and atol eta.  Every later
 * bdfx_integrate() uses these per-mechanism tolerances in place of the
 * options' atol; calling again (e.g. every K outer steps) recomputes them
 * from the current states; eta = 0 returns to the options' atol.  The choice
 * of tolerance array is fixed into graphs captured meanwhile.
 * d_typical: NULL, or device memory [n_mech][S_max] (S_max = largest species
 * count of the plan) that receives ytyp (0 beyond S_m and for a mechanism
 * without cells).  Enqueue only (two kernels, no allocation, capturable).
 * Errors: BDFX_EINVAL for eta < 0 or not finite; BDFX_EORDER before bind. */
int bdfx_typical_atol(bdfx_ctx ctx, double eta, double *d_typical);
/* bdfx_typical_atol() for callers that cannot allocate device memory or bind
 * a workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the typical-value tolerances of n_cells cells of
 * one mechanism, with no context.
 *   d_y       [n_cells][ldy] FP64 in   states (entries 0..n_species-1 read)
 *   d_atol    [n_species] FP64 out     eta * ytyp_i, or eta where ytyp_i is
 *                                      not positive (as bdfx_typical_atol())
 *   d_typical [n_species] FP64 out     ytyp_i = 0.5 (min + max), or NULL
 * Work is enqueued on hip_stream (hipStream_t, NULL = default stream) of HIP
 * device `device`; the caller's current device is restored before return.
 * Scratch: the per-block extremes live in a fixed 256 KiB device array of the
 * library (room for 64 species), one copy per device, held until the process
 * ends; the first call on a device looks up its address, no call allocates.
 * Calls that overlap on one device (any streams) share that array and race:
 * serialise them.  For the same states, the results equal bit for bit those
 * of bdfx_typical_atol() on a context whose cells all belong to one mechanism.
 * Errors (text from bdfx_last_error(NULL)): BDFX_EINVAL for NULL d_y or d_atol,
 * n_cells < 1, n_species outside 1..BDFX_MAX_SPECIES (the scratch's limit),
 * ldy < n_species, eta not finite or not > 0, or a bad device; BDFX_EHIP if
 * the device cannot be selected or a launch fails. */
int bdfx_typical_atol_static(int device, void *hip_stream, const double *d_y, int64_t n_cells,
                             int32_t ldy, int32_t n_species, double eta, double *d_atol,
                             double *d_typical);
/* Species weights w [S] (host) used by bdfx_perturb(); default all ones. */
int bdfx_mech_set_weights(bdfx_mech mech, const double *weights);

/* Sum the per-cell statistics of the last integrate; synchronises the
 * context's stream.  Requires d_stats bound.  The right-hand-side counts are
 * the per-cell work estimates an application can feed back into its load
 * balancing (Sec. 4.1.1).  Errors: BDFX_EORDER before bdfx_bind() or without
 * d_stats; BDFX_EHIP if the copy fails. */
int bdfx_stats_summary(bdfx_ctx ctx, bdfx_summary *out);

/* Discrete adjoint of the last bdfx_integrate() (which must have been run
 * with record_steps > 0, single outer step, no bdfx_perturb() since):
 *   d_ybar    [N][ldy]  dL/dy(t_out)
 *   d_y0bar   [N][ldy]  out: dL/dy(t0)
 *   d_lnA_bar [n_mech][R_max] out: dL/dlnA_r summed over the cells of each
 *                       mechanism (may be NULL)
 * The gradient is that of the discrete map with the recorded step sizes and
 * orders held fixed and each corrector solved exactly (Jacobians re-evaluated
 * at the recorded states).  With checkpoint_every = K > 0 the sweep runs in
 * passes over the segments from the last: each pass reruns one K-step segment
 * of every cell from its checkpoint into the workspace ((K + 6) x (S_max + 2)
 * doubles per cell), which gives the same steps bit for bit, and then sweeps
 * it; ceil(record_steps / K) passes of two launches each.  The bound inputs
 * (T, rate scales, forcing) must be unchanged since the integrate.  Enqueue
 * only. */
int bdfx_adjoint(bdfx_ctx ctx, const double *d_ybar, double *d_y0bar, double *d_lnA_bar);

/* Where bdfx_integrate() with record_steps > 0 leaves the step record in the
 * bound workspace (byte offsets from d_workspace), for callers that inspect or
 * checkpoint it.  For cell c (its index in d_y):
 *   steps [N][cap][stride] FP64: accepted step n (0-based) of cell c, whose
 *         mechanism has S state entries, holds the accepted state y_n in
 *         entries 0..S-1, the step size h_n in entry S and
 *         q_n + 256 * rebuilt_n in entry S+1, where q_n is the order the step
 *         was taken with and rebuilt_n = 1 if the Nordsieck array was rebuilt
 *         at order 1 (repeated error-test failures, Sec. 2) before it;
 *   count [N] int32: accepted steps recorded;
 *   hpad  [N] FP64: the initial step size, with which the step-size history
 *         before the first step is padded;
 *   y0    [N][stride] FP64: the state at t0.
 * The record describes the frozen discrete map that bdfx_adjoint()
 * differentiates (the step sequence of the run with each corrector solved
 * exactly).  Host-only.  Errors: BDFX_EORDER before bdfx_bind() or without
 * recording; BDFX_EUNSUPPORTED with checkpoint_every > 0 (no per-step record). */
typedef struct {
  int32_t cap;    /* recorded steps per cell (bdfx_options.record_steps) */
  int32_t stride; /* doubles per recorded step (largest state length + 2) */
  size_t off_steps, off_count, off_hpad, off_y0;
} bdfx_record_layout;
int bdfx_get_record_layout(bdfx_ctx ctx, bdfx_record_layout *out);

/* Launch shape of the integrator for the cells of one mechanism. */
typedef struct {
  int32_t mech;            /* mechanism index (as in d_cell_mech) */
  int32_t waves_per_simd;  /* 0, 3, 4 or 5, as bdfx_options.waves_per_simd */
  int32_t waves_per_block; /* 1..16 */
  int32_t queue_chunk;     /* cells per work-queue pop, >= 1 */
  int64_t sample_cells;    /* bdfx_autotune(): cells timed */
  float ms;                /* bdfx_autotune(): time of the fastest shape on the sample */
  int32_t cells_per_wave;  /* 1, or 2 for mechanisms of at most 32 species */
  int32_t tables;          /* out: where the reaction tables of this launch live, chosen by
                              occupancy: 1 all in LDS; 0 slot words read from global memory;
                              2 slot words and the cell's rate constants in global memory
                              (a per-wave workspace slot; work-queue scheduler, one cell per
                              wave, 32 species or more).  Ignored by bdfx_set_tuning(). */
  int32_t fused;           /* out: 1 if the mechanisms' cells run in one launch
                              (BDFX_SCHED_FUSED with an eligible pair), with the larger
                              mechanism's register budget and table placement.  Ignored by
                              bdfx_set_tuning(). */
} bdfx_tuning;

/* Autotuner: for every mechanism, times each candidate launch shape
 * (cells_per_wave in {1, 2} (2 only up to 32 species) x waves_per_simd in
 * {0, 3, 4, 5} x waves_per_block in {1, 2, 4} x queue_chunk in {1, 4} for the
 * queue scheduler) integrating the first min(sample_cells,
 * 16384) cells of that mechanism over [t0, t_out] with HIP events, and keeps
 * the fastest; sample_cells <= 0 means 16384.  The sampled states are saved
 * in the workspace and restored after every trial; their d_status / d_stats
 * entries are overwritten.  out: [n_mech] results in launch order (larger
 * mechanisms first), or NULL.  Synchronises the stream.  The choice holds
 * until the next bdfx_bind(). */
int bdfx_autotune(bdfx_ctx ctx, double t0, double t_out, int64_t sample_cells, bdfx_tuning *out);
/* Apply launch shapes chosen earlier (for example cached results of
 * bdfx_autotune()); entries name their mechanism; the rest are ignored. */
int bdfx_set_tuning(bdfx_ctx ctx, const bdfx_tuning *tunings, int32_t n);
/* The launch shape in effect for every mechanism (after bdfx_bind(),
 * bdfx_autotune() or bdfx_set_tuning()), in launch order: out[k] for
 * k < min(n, n_mech); sample_cells and ms are 0 unless the shape came from
 * bdfx_autotune() in this binding.  Host-only. */
int bdfx_get_tuning(bdfx_ctx ctx, bdfx_tuning *out, int32_t n);

/* Library version string. */
const char *bdfx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BDFX_H */
