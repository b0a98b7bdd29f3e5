/*
 * FP64 reference ("oracle") for the ADMM multi-agent trajectory solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load or call this code.  It shares no
 * source, header, table or helper with the HIP library; its only common
 * ground with it is the seeded input generator.
 *
 * What it computes (every step in plain, unblocked form, in double precision):
 *   - the per-agent local QP of Sec. IV-A, Eq. (3), with stage costs over
 *     t = 0..T-1, the terminal weight at T, and the consensus penalty on the
 *     coupled steps t = 1..T; solved exactly by a primal active-set method on
 *     the input bounds whose equality subproblems are dense KKT systems
 *     factorised by LU with partial pivoting;
 *   - the consensus update Eq. (4) read as the joint Euclidean projection of
 *     the two agents' copies onto the linearised separation half-plane, and the
 *     dual update Eq. (5), both on plain (uncollapsed) z and lambda for every
 *     ordered pair;
 *   - Boyd-style primal/dual residuals and the stopping test (Sec. V-A).
 *
 * Parity unpinned: with normals re-linearized every iteration, which side two
 * agents pass on is path-dependent, and so are runs stopped at max_iter and
 * degenerate ties of the active set.  No closed form or brute force fixes
 * those results; they are held only by lockstep agreement of the first
 * iterations and by the oracle's own sensitivity to perturbed starts.
 */
#ifndef TADMM_ORACLE_H
#define TADMM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_CONVERGED = 0, ORC_MAX_ITER = 1, ORC_ACTIVE_SET_CAP = 2, ORC_NONFINITE = 3 };
enum { ORC_NORMAL_PER_ITER = 0, ORC_NORMAL_FROZEN = 1 };
enum { ORC_START_PREV = 0, ORC_START_WARM = 1, ORC_START_COLD = 2 };

typedef struct {
  int nx, nu, dp;            /* dp = nu; positions are the first dp state entries */
  double A[36], B[18];       /* row-major nx*nx and nx*nu */
  double u_lo[3], u_hi[3];   /* per-component input box */
  double qT_scale;           /* Q_T = qT_scale * Q */
  double d_min, rho, eps_abs, eps_rel;
  double mu_tol;             /* a bound multiplier below -mu_tol is dropped */
  int max_iter;
  int max_as_iter;           /* <= 0 selects 10*T*nu */
  int normal_mode;           /* ORC_NORMAL_* */
  int warm_start;            /* 1: unconstrained solve, clip, roll out; 0: u = 0, W empty */
  int hotstart;              /* 1: later ADMM iterations start from the previous (w, W) */
  int lu_reuse;              /* 1: keep the KKT factors while W is unchanged */
  int fixed_iters;           /* > 0: run exactly this many iterations (stop test ignored) */
  /* Adaptive penalty by residual balancing (Boyd et al. 2011, Sec. 3.4.1):
   * every rho_every iterations, rho <- rho_tau rho if r > rho_mu s,
   * rho <- rho / rho_tau if s > rho_mu r (lambda unscaled, unchanged). */
  int adaptive_rho;
  double rho_mu, rho_tau;
  int rho_every;
  /* State box (x_t, t >= 1) by a further ADMM split: a copy y of the boxed
   * states held in the box, its dual mu, penalty sigma = the initial rho.
   * Two groups, each split only where one of its bounds is finite: the
   * non-position states (components dp..nx-1) in [s_lo, s_hi], the
   * positions in [p_lo, p_hi]; +-inf: unbounded. */
  int state_box;
  double s_lo[3], s_hi[3];
  double p_lo[3], p_hi[3];
  /* Over-relaxation (Boyd et al. 2011, Sec. 3.4.3): the z- and dual updates
   * use alpha C x^(k+1) + (1 - alpha) z^k; 1 is plain ADMM, (0, 2) valid. */
  double alpha;
  /* Momentum: fast ADMM with restart (Goldstein et al. 2014, Alg. 8) on the
   * consensus block: the next iteration takes extrapolated copies and duals,
   * restarting when the combined residual fails to fall by mom_eta.  Not
   * combined with adaptive_rho, alpha != 1 or the state box. */
  int momentum;
  double mom_eta;
} orc_params;

typedef struct {
  int N, T;
  const double *x0;          /* [N][nx] */
  const double *xref;        /* [N][T+1][nx] */
  const double *q_diag;      /* [nx] */
  const double *r_diag;      /* [nu] */
  const double *normals;     /* FROZEN: [P][T][dp] (pair i<j lexicographic, t=1..T) or NULL */
  /* heterogeneous agents (each NULL: the scenario's / the params' value) */
  const double *agent_q;     /* [N][nx] diagonal of Q per agent */
  const double *agent_r;     /* [N][nu] diagonal of R per agent */
  const double *agent_lo, *agent_hi;   /* [N][nu] input box per agent */
  const double *agent_A, *agent_B;     /* [N][nx*nx], [N][nx*nu] dynamics per agent (row-major) */
} orc_scenario;

typedef struct {
  double *x;                 /* [N][T+1][nx] */
  double *u;                 /* [N][T][nu] */
  signed char *w;            /* [N][T][nu]: 0 free, 1 at lower bound, 2 at upper bound */
  double *mu;                /* [N][T][nu]: bound multipliers of the last local solve (0 if free) */
  unsigned char *pair_active;/* [P][T]: half-plane violated at the last consensus update */
  double *z;                 /* optional [N][N][T][dp]: z_ij at t = 1..T */
  double *lam;               /* optional [N][N][T][dp]: lambda_ij at t = 1..T */
  double *hist;              /* optional [max_iter][4]: r, s, eps_pri, eps_dual */
  int status, iters;
  double r_norm, s_norm, eps_pri, eps_dual;
  long as_passes;            /* equality-QP solves over the whole run */
  long lu_factorizations;
  double *rho_hist;          /* optional [max_iter]: the rho of iteration k */
} orc_result;

/* One agent's local QP (Eq. 3) with the consensus data folded into
 * ysum[t] = sum_j (rho z_ij,t - lambda_ij,t), t = 1..T (row 0 ignored).
 * x [T+1][nx], u [T][nu], w [T][nu] are in/out; with start = ORC_START_PREV
 * they must hold a feasible point and its working set.  mu [T][nu] receives
 * the bound multipliers.  Returns 0, or 1 if the active-set cap was hit. */
int orc_agent_qp(const orc_params *prm, int T, int n_nbr, const double *x0, const double *xref,
                 const double *q_diag, const double *r_diag, const double *ysum,
                 double *x, double *u, signed char *w, double *mu, int start,
                 long *passes, long *facts);

/* One scenario: ADMM until the stopping test passes or max_iter. */
int orc_admm(const orc_params *prm, const orc_scenario *sc, orc_result *res, int threads);

/* S independent scenarios, OpenMP over scenarios (dynamic schedule). */
int orc_admm_batch(const orc_params *prm, int S, const orc_scenario *scs, orc_result *res, int threads);

int orc_max_threads(void);

/* Normals of every pair (i < j) and step t = 1..T linearized about the
 * positions of x [N][T+1][nx]: (p_i - p_j)/|p_i - p_j|, or the reference
 * normal when |p_i - p_j| < 1e-6.  normals [P][T][dp], P = N(N-1)/2 in
 * lexicographic pair order (the layout of orc_scenario.normals). */
int orc_relinearize(const orc_params *prm, const orc_scenario *sc, const double *x, double *normals);

#ifdef __cplusplus
}
#endif
#endif
