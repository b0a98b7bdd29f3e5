/*
 * turboadmm.h -- C ABI of the MI355X (gfx950) ADMM multi-agent trajectory solver.
 *
 * Method: the ADMM decomposition of the centralized multi-agent QP of
 * Sec. III-A, Eq. (1).  Every iteration solves one local QP per agent
 * (Sec. IV-A, Eq. 3: linear dynamics, quadratic tracking and effort cost,
 * augmented-Lagrangian penalty toward the consensus positions, input box),
 * then performs the consensus update (Eq. 4) and the dual update (Eq. 5) for
 * every pair of agents and time step, then evaluates the primal and dual
 * residuals (stopping rule of Sec. V-A).  Each local QP is solved by a
 * Riccati backward sweep (Eq. 7), a forward rollout (Eq. 8) and costates
 * (Eq. 9) inside a primal active-set loop on the input bounds; the Riccati
 * factors are cached across ADMM iterations while the active set is unchanged
 * (the factorization hotstart of Sec. IV-C) and iteration 1 starts from the
 * unconstrained Riccati solution (the warm start of Sec. IV-B).
 *
 * Conventions shared by every entry point:
 *  - Pointers marked DEVICE are device (HBM) addresses on the context's
 *    device; pointers marked HOST are ordinary host memory.  The library never
 *    frees caller memory and never keeps a caller pointer beyond the call,
 *    except that tadmm_polish() and tadmm_adjoint() read the workspace (and
 *    the batch inputs) of the matching tadmm_solve().
 *  - All device work is ordered on the stream given to tadmm_create().
 *    tadmm_solve(), tadmm_polish() and tadmm_adjoint() return after the work
 *    has completed (they synchronize the stream once at the end).
 *  - A context is not thread-safe; use one context per host thread.
 *  - Return codes report argument and runtime errors only.  Per-scenario
 *    outcomes (converged, iteration cap, ...) are data in tadmm_out::status.
 *  - Floating point is FP32 on the device (the derivative: see eqp_fp64).
 *
 * Problem layout (homogeneous agents; C selects the first dp = nu entries of
 * the state as the position):
 *   x_{t+1} = A x_t + B u_t,  t = 0..T-1,  x_0 given
 *   cost  sum_{t=0}^{T-1} (x_t - r_t)' Q (x_t - r_t) + u_t' R u_t
 *         + (x_T - r_T)' (qT_scale Q) (x_T - r_T)          (Eq. 1, no 1/2)
 *   u_lo <= u_t <= u_hi componentwise
 *   for every pair i < j and t = 1..T:  n_ij,t' (C x_i,t - C x_j,t) >= d_min,
 *   the half-plane linearisation of ||p_i - p_j|| >= d_min (Sec. III-A).
 */
#ifndef TURBOADMM_H
#define TURBOADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TADMM_OK = 0,
  TADMM_ERR_INVALID_ARG = 1,     /* a parameter outside its documented range        */
  TADMM_ERR_SHAPE = 2,           /* inconsistent sizes / offsets                     */
  TADMM_ERR_NONFINITE = 3,       /* NaN/Inf (or a non-positive weight) in the inputs */
  TADMM_ERR_INFEASIBLE_START = 4,/* two agents start closer than d_min               */
  TADMM_ERR_HIP = 5,             /* a HIP runtime call failed                        */
  TADMM_ERR_WORKSPACE = 6,       /* workspace missing or too small                   */
  TADMM_ERR_STATE = 7            /* call out of order (polish/adjoint without solve) */
} tadmm_status;

/* Per-scenario outcome, written to tadmm_out::status. */
typedef enum {
  TADMM_SCEN_CONVERGED = 0,      /* primal and dual residual tests passed            */
  TADMM_SCEN_MAX_ITER = 1,       /* max_iter iterations without passing the test     */
  TADMM_SCEN_ACTIVE_SET_CAP = 2, /* a local QP hit max_as_iter passes (solve stopped) */
  TADMM_SCEN_NONFINITE = 3       /* a residual became NaN/Inf (solve stopped)        */
} tadmm_scen_status;

/* Which half-planes the consensus step projects onto. */
typedef enum {
  /* Linearised about the latest primal iterate: n = (C x_i - C x_j)/||.||
   * from the x just computed, with a fallback to the reference geometry when
   * the two positions coincide (< 1e-6). */
  TADMM_NORMAL_PER_ITER = 0,
  /* Fixed for the whole solve: tadmm_batch::normals, or the reference
   * normals when that pointer is NULL. */
  TADMM_NORMAL_FROZEN = 1
} tadmm_normal_mode;

typedef enum {
  /* Scenarios one after another; every ADMM iteration is three kernel
   * launches plus a device-to-host copy and a stream synchronisation. */
  TADMM_MODE_PLAIN = 0,
  /* All scenarios in one persistent kernel: workgroups take scenarios from an
   * atomic queue (largest first) and iterate ADMM on the device until each
   * scenario's own stopping test passes; launched through a cached hipGraph. */
  TADMM_MODE_BATCHED = 1,
  /* Scenarios one after another, every phase spread over many workgroups:
   * the x-update one lane per agent, the consensus step one lane per
   * agent-stage (each block staging the positions of its stages in LDS), the
   * test one wavefront; iterations run in cached hipGraphs of 8 with the
   * iteration number and scenario index in device memory, launched until the
   * scenario stops (one 4-byte read-back per launch).  For a few large
   * scenarios (a single scenario of 128 agents), where one workgroup per
   * scenario would leave most compute units idle.  Results are bitwise those
   * of the other modes. */
  TADMM_MODE_WIDE = 2
} tadmm_mode;

/* Problem constants and solver options (host struct, passed by pointer and
 * copied by tadmm_create). */
typedef struct {
  int32_t nx, nu;            /* (4,2): 2-D double integrator; (6,3): 3-D. dp = nu */
  float A[36];               /* row-major nx*nx (first nx*nx entries used)        */
  float B[18];               /* row-major nx*nu                                    */
  float u_lo[3], u_hi[3];    /* input box, u_lo[c] < u_hi[c]                       */
  float qT_scale;            /* terminal weight Q_T = qT_scale * Q, > 0            */
  float d_min;               /* minimum separation, >= 0                           */
  float rho;                 /* ADMM penalty, > 0                                  */
  float eps_abs, eps_rel;    /* stopping tolerances, >= 0                          */
  float mu_tol;              /* a bound multiplier below -mu_tol is released, >= 0 */
  int32_t max_iter;          /* >= 1                                               */
  int32_t max_as_iter;       /* active-set passes per local QP; <= 0: 10*T*nu      */
  int32_t normal_mode;       /* tadmm_normal_mode                                  */
  int32_t cache_factors;     /* 1: keep Riccati factors while the active set is
                                unchanged (default); 0: refactor on every pass     */
  int32_t riccati_warmstart; /* 1: iteration 1 starts from the unconstrained
                                Riccati solution, clipped (default); 0: u = 0      */
  int32_t hotstart;          /* 1: iterations >= 2 start from the previous (x,u,W)
                                (default); 0: every iteration starts afresh        */
  int32_t check_inputs;      /* 1: reject non-finite inputs / close starts with an
                                error code (default); 0: skip the checks, a bad
                                scenario ends with status NONFINITE                 */
  int32_t block_threads;     /* batched mode workgroup size: 64, 128, 192 or 256;
                                0: use the context's tuned value                   */
  int32_t refine;            /* 1: one step of mixed-precision iterative refinement
                                of every local QP solution (reduced gradient in
                                FP64, correction with the FP32 factors) (default);
                                0: plain FP32 solve                                */
  float refine_band;         /* with refine = 1: refine in every iteration (0), or
                                only once the primal and dual residuals of the
                                last stopping test are both within refine_band
                                times their tolerances (> 0; 10 is the binding's
                                default: before that the FP32 rounding of the
                                local QPs is far below what the iteration
                                resolves)                                           */
  int32_t eqp_fp64;          /* real type of the Riccati sweeps of tadmm_polish /
                                tadmm_adjoint: 1 FP64 (recommended), 0 FP32;
                                their multipliers and reductions are FP64 either
                                way                                                 */
  int32_t adaptive_rho;      /* 1: per-scenario penalty by residual balancing
                                (Boyd et al. 2011, Sec. 3.4.1; the paper names
                                adaptive penalties as future work, Sec. VI):
                                every rho_every iterations, rho <- rho_tau rho if
                                r > rho_mu s, rho <- rho / rho_tau if s > rho_mu r
                                (lambda unscaled, unchanged); a change refactors
                                every stage.  0: rho fixed (default)              */
  float rho_mu, rho_tau;     /* with adaptive_rho: rho_mu >= 1, rho_tau > 1      */
  int32_t rho_every;         /* with adaptive_rho: >= 1                           */
  int32_t state_box;         /* 1: box s_lo <= x_t,k <= s_hi on the non-position
                                states (k = nu..nx-1, the velocities of the
                                double integrator; t = 1..T), the state sets of
                                Eq. 1, by a further ADMM split: a copy y of those
                                states held in the box, its dual, penalty = the
                                initial rho.  Not with tadmm_polish/adjoint.     */
  float s_lo[3], s_hi[3];    /* with state_box: s_lo < s_hi (+-inf: unbounded)   */
  float alpha;               /* over-relaxation (Boyd et al. 2011, Sec. 3.4.3;
                                the paper names ADMM variants as future work,
                                Sec. VI): the consensus and dual updates use
                                alpha C x^(k+1) + (1 - alpha) z^k, 0 < alpha
                                < 2.  1 (or 0, for zero-initialized structs):
                                plain ADMM.  Otherwise the workspace holds 2 nu
                                floats more per ordered pair copy and step (the
                                copies' z).  The derivative of a relaxed solve is
                                that of its converged point, as without.         */
  float p_lo[3], p_hi[3];    /* with state_box: a box p_lo <= x_t,c <= p_hi on the
                                positions (c < nu, t = 1..T), by the same split;
                                p_lo < p_hi (+-inf: unbounded).  Each group
                                (positions, other states) is split only where
                                one of its bounds is finite.                     */
  int32_t momentum;          /* 1: momentum ADMM, the fast ADMM with restart of
                                Goldstein et al. (2014, Alg. 8) on the consensus
                                block: each iteration takes extrapolated copies
                                and duals, restarting when the combined residual
                                fails to fall by the factor mom_eta.  Not with
                                adaptive_rho, alpha != 1,
                                state_box or tadmm_sqp (the derivative of the
                                solve is that of its converged point, as
                                without).  The workspace holds 6 nu floats more per
                                ordered pair copy and step.  0: off (default)    */
  float mom_eta;             /* with momentum: 0 < mom_eta < 1 (0.999)            */
} tadmm_params;

/* A ragged batch of S independent scenarios.  Scenario s has N_s agents and
 * horizon T_s.  Orderings (row-major, scenarios back to back):
 *   x0      DEVICE float [sum_s N_s][nx]            (s, agent)
 *   xref    DEVICE float [sum_s N_s (T_s+1)][nx]    (s, agent, t = 0..T_s)
 *   q_diag  DEVICE float [S][nx]   diagonal of Q, > 0
 *   r_diag  DEVICE float [S][nu]   diagonal of R, > 0
 *   normals DEVICE float [sum_s P_s T_s][nu] or NULL; FROZEN mode only;
 *           (s, pair i<j in lexicographic order, t = 1..T_s), unit vectors.
 * Heterogeneous agents (each optional, NULL: the scenario's or the params'
 * value for every agent; not supported by tadmm_polish / tadmm_adjoint,
 * whose gradients are per scenario):
 *   agent_q   DEVICE float [sum_s N_s][nx]  each agent's diagonal of Q, > 0
 *   agent_r   DEVICE float [sum_s N_s][nu]  each agent's diagonal of R, > 0
 *   agent_lo, agent_hi  DEVICE float [sum_s N_s][nu]  each agent's input
 *             box (both or neither), finite, lo < hi
 *   agent_A, agent_B  DEVICE float [sum_s N_s][nx*nx], [sum_s N_s][nx*nu]
 *             each agent's dynamics x_{t+1} = A x_t + B u_t, row-major
 *             (both or neither), finite; the solve then takes the
 *             one-lane-per-agent path for every agent
 * P_s = N_s (N_s - 1) / 2. */
typedef struct {
  int32_t n_scen;
  const int32_t *n_agents;   /* HOST [S], N_s >= 1 */
  const int32_t *horizon;    /* HOST [S], T_s >= 1 */
  const float *x0;
  const float *xref;
  const float *q_diag;
  const float *r_diag;
  const float *normals;
  const float *agent_q, *agent_r, *agent_lo, *agent_hi;
  const float *agent_A, *agent_B;
} tadmm_batch;

/* Outputs, caller-allocated DEVICE buffers (any may be NULL except status
 * and iters). */
typedef struct {
  float *x;                  /* [sum N_s (T_s+1)][nx]   (s, agent, t)           */
  float *u;                  /* [sum N_s T_s][nu]       (s, agent, t)           */
  int8_t *w;                 /* [sum N_s T_s][nu]  0 free, 1 at lower, 2 upper  */
  uint8_t *pair_active;      /* [sum P_s T_s]  1 if the half-plane was violated
                                at the last consensus update (s, pair, t=1..T)  */
  int32_t *status;           /* [S] tadmm_scen_status                           */
  int32_t *iters;            /* [S] ADMM iterations performed                   */
  float *r_norm, *s_norm;    /* [S] final primal / dual residual norms          */
  float *eps_pri, *eps_dual; /* [S] final tolerances of the stopping test       */
  int64_t *counters;         /* [S][8]: active-set passes, refactored
                                agent-stages, affine agent-stage passes, pair-
                                step updates; batched mode also the time spent
                                in the x-update, pair and test phases (ticks of
                                the 100 MHz device clock, one workgroup), 0.
                                Diagnostics only: batched mode tallies each
                                lane's share of the first three over a whole
                                scenario in 32 bits, so they wrap once one
                                lane's share passes 2^32 (max_iter x T x
                                passes per iteration beyond about 4e9)        */
  float *hist;               /* [S][max_iter][2] or NULL: for every iteration k
                                = 1..iters the primal and dual residual norms
                                ||r||, ||s|| of its stopping test (Sec. V-A) at
                                [s][k-1][0..1]; entries beyond the scenario's
                                last iteration are left untouched.  With
                                tadmm_sqp: the last round of each scenario      */
} tadmm_out;

typedef struct tadmm_ctx tadmm_ctx;

/* Bytes of device workspace needed by tadmm_solve() for this batch shape
 * (HOST n_agents / horizon as in tadmm_batch).  The workspace holds the
 * factor cache, trajectories, working sets and the pair duals; it must stay
 * untouched between a solve and its adjoint. */
tadmm_status tadmm_workspace_size(const tadmm_params *params, int32_t n_scen, const int32_t *n_agents,
                                  const int32_t *horizon, size_t *bytes);

/* Create a context on the current HIP device.  `stream` is a hipStream_t
 * (NULL = the default stream).  Validates params (TADMM_ERR_INVALID_ARG). */
tadmm_status tadmm_create(tadmm_ctx **ctx, const tadmm_params *params, void *stream);

/* Solve every scenario of the batch (Eqs. 3-5 iterated to the stopping test
 * of Sec. V-A).  `workspace` is a DEVICE buffer of at least
 * tadmm_workspace_size() bytes, 256-byte aligned.  mode: tadmm_mode. */
tadmm_status tadmm_solve(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                         size_t workspace_bytes, int32_t mode);

/* tadmm_solve() for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, in TADMM_MODE_PLAIN or TADMM_MODE_BATCHED, with the
 * workspace taken from a static device array of the library instead of the
 * caller.  The array holds 64 MiB (TADMM_NOALLOC_WORKSPACE_BYTES) per device,
 * from the library's load until the process ends; a batch whose
 * tadmm_workspace_size() exceeds it returns TADMM_ERR_WORKSPACE.  The call
 * makes no device or pinned-host allocation: the batched mode launches its
 * kernels directly on the context's stream (no graph), the scenario tables
 * are copied from ordinary host memory, and every region the solve reads is
 * initialized by the solve itself.  Every call on a device shares that
 * device's array, so calls that overlap in time on one device (two host
 * threads, or two streams) race and corrupt each other's results; serialize
 * them.  tadmm_polish() / tadmm_adjoint() do not follow this call
 * (TADMM_ERR_STATE): they need the caller-owned workspace of tadmm_solve().
 * Errors: as tadmm_solve(); TADMM_ERR_INVALID_ARG for TADMM_MODE_WIDE. */
#define TADMM_NOALLOC_WORKSPACE_BYTES (64u << 20)
tadmm_status tadmm_solve_noalloc(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, int32_t mode);

/* The derivative of a converged solve (an extension: the paper defines the
 * solve, not its derivative).  The solution of the last tadmm_solve() on this
 * context is read as the solution of the centralized QP (Sec. III-A, Eq. 1)
 * with its final active sets held as equalities: the inputs of the working
 * sets (tadmm_out::w) at their bounds, and the half-planes of the last
 * consensus step (Eq. 4) that were violated (tadmm_out::pair_active) as
 * n'(C x_i,t - C x_j,t) = d_min, with the normals of that step frozen
 * (PER_ITER: from the final positions; FROZEN: the given or reference ones).
 *
 * tadmm_polish solves that equality QP: per agent a fixed-input LQR (Riccati
 * factors of the local QP of Eq. 3 without the consensus penalty, Eq. 7),
 * coupled only through the held half-planes, whose multipliers solve the
 * Schur system D H^-1 D' nu = d - D w(0) by MINRES (warm start: the duals of
 * the last consensus step; when the held rows cannot all hold, which a solve
 * stopped at max_iter can leave, MINRES stops at a least-squares solution,
 * once ||S r|| <= 1e-4 ||S|| ||r|| (3e-4 with eqp_fp64 = 0), or after 4000
 * iterations).  It overwrites out->x and out->u
 * (required, DEVICE, layouts of tadmm_out) with the polished solution and
 * keeps it in the workspace.  Call it once per solve; TADMM_ERR_STATE without
 * a preceding successful tadmm_solve with the same batch (pointers and
 * shapes) and workspace, or when already called for that solve.
 *
 * tadmm_adjoint then back-propagates a loss L(x, u) through the polished
 * solution by the implicit function theorem on the KKT system of the same
 * equality QP: the adjoint system is an equality QP of the same structure
 * (homogeneous rows, linear term -dL/dw), solved the same way with the same
 * factors, and the parameter gradients are -wbar' dF/dtheta, accumulated in
 * FP64.  Upstream gradients at the polished solution (DEVICE, layouts of
 * tadmm_out::x / u; dL_du may be NULL):
 *   dL_dx [sum N_s (T_s+1)][nx],  dL_du [sum N_s T_s][nu]
 * Outputs (DEVICE, any may be NULL):
 *   dL_dx0    [sum N_s][nx]          dL_dxref [sum N_s (T_s+1)][nx]
 *   dL_dlogq  [S][nx]  (w.r.t. log of q_diag)   dL_dlogr [S][nu]
 * TADMM_ERR_STATE without a preceding tadmm_polish of the same solve.
 *
 * stats (both; DEVICE float [S][4] or NULL): number of held half-planes,
 * MINRES iterations, final relative MINRES residual, and the largest
 * |n'(C x_i - C x_j) - d| over the held rows after the final solve (d = d_min
 * for the polish, 0 for the adjoint).  Both calls synchronize the stream. */
tadmm_status tadmm_polish(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                          size_t workspace_bytes, float *stats);
tadmm_status tadmm_adjoint(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                           size_t workspace_bytes, const float *dL_dx, const float *dL_du, float *dL_dx0,
                           float *dL_dxref, float *dL_dlogq, float *dL_dlogr, float *stats);

/* SQP outer loop around the solve: the separation constraints of Eq. 1,
 * convexified as half-planes with frozen normals (Sec. III-A), re-linearized
 * about each round's solution.
 *   Round 0 solves with the batch's normals (batch->normals; NULL: those of
 *   the reference trajectories), whatever params->normal_mode says; every
 *   later round takes the normals of the previous round's positions,
 *   n = (p_i - p_j)/|p_i - p_j| (the reference normal where two positions
 *   coincide), and continues from the previous round's iterate, duals,
 *   working sets and Riccati factors (a warm start) instead of the
 *   references.  Each round runs the ADMM in `mode` (tadmm_mode) to its
 *   stopping test or max_iter.
 *   A scenario leaves the loop, as under the stopping rule of Sec. V-A, after
 *   a round (other than the first) whose objective of Eq. 1,
 *     sum_i sum_{t<T} ||x_t - r_t||_Q^2 + ||u_t||_R^2 + ||x_T - r_T||_{Q_T}^2,
 *   differs from the previous round's by at most rtol times its magnitude,
 *   and whose positions keep every pair at least d_min - sep_tol apart at
 *   every step t = 1..T; otherwise after max_rounds (>= 1).  rtol, sep_tol:
 *   finite, >= 0 (the paper's rule: rtol = 1e-4; sep_tol absorbs the ADMM
 *   tolerance, e.g. 1e-2).
 *   out receives the last round's solution of every scenario (as
 *   tadmm_solve; out->counters sum over the rounds).  stats (DEVICE, [S][4]
 *   floats, may be NULL): rounds solved, 1 if the stopping rule was met, the
 *   last round's objective, its smallest distance between two agents.
 *   Errors: as tadmm_solve, and TADMM_ERR_INVALID_ARG for a bad max_rounds,
 *   rtol, sep_tol or mode.  The workspace's normals region holds the last
 *   round's normals afterwards; tadmm_polish()/tadmm_adjoint() then return
 *   TADMM_ERR_STATE (the derivative is defined for tadmm_solve() results).
 *   tadmm_last_kernel_ms() gives the summed time of the rounds' solves. */
tadmm_status tadmm_sqp(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                       size_t workspace_bytes, int32_t mode, int32_t max_rounds, float rtol, float sep_tol,
                       float *stats);

/* Measure candidate workgroup sizes of the batched kernel on this batch and
 * keep the fastest in the context (used when params.block_threads == 0).
 * Writes the chosen size to *best_threads (HOST, may be NULL). */
tadmm_status tadmm_autotune(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                            size_t workspace_bytes, int32_t *best_threads);

/* Duration in milliseconds of the last batched solve, plain solve, polish or
 * adjoint on this context (HIP events recorded around its launches on the
 * context's stream), or -1 if none. */
float tadmm_last_kernel_ms(const tadmm_ctx *ctx);

tadmm_status tadmm_destroy(tadmm_ctx *ctx);
const char *tadmm_status_string(tadmm_status s);
/* Message of the last error on this context ("" if none); owned by ctx. */
const char *tadmm_last_error(const tadmm_ctx *ctx);
/* Library version string. */
const char *tadmm_version(void);

#ifdef __cplusplus
}
#endif
#endif
