/*
 * FP64 reference ("oracle") for the ADMM multi-agent trajectory solver.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, by the package smoke check
 * and by the benchmark's CPU-baseline leg, never by the product path.  Plain,
 * slow and unblocked on purpose; see tadmm_oracle.h for the scope.
 *
 * Notation (paper Sec. III-IV): agent i has state x_t in R^nx, input u_t in
 * R^nu, positions C x_t = first dp entries of x_t.  The local QP of Eq. (3)
 * is written over w = (u_0..u_{T-1}, x_1..x_T) as
 *     min 1/2 w'Hw + c'w   s.t.  x_{t+1} = A x_t + B u_t,  x_0 given,
 *                                u_lo <= u_t <= u_hi,
 * with H = blockdiag(2R,...,2R, 2Q + rho n_nbr C'C, ..., 2 Q_T + rho n_nbr C'C)
 * (stage costs as in Eq. (1), no 1/2, tracking over t = 0..T-1 and the
 * terminal weight at T; penalty (rho/2)||C x_t - z_ij,t + lambda_ij,t/rho||^2
 * for each of the n_nbr partners on the coupled steps t = 1..T).
 */
#include "tadmm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (Golub & Van Loan, Alg. 3.4.1), row-major. */
/* ------------------------------------------------------------------------ */

static int lu_factor(double *a, int n, int *piv) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(a[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      double v = fabs(a[(size_t)r * n + k]);
      if (v > best) { best = v; p = r; }
    }
    piv[k] = p;
    if (best == 0.0) return 1;
    if (p != k) {
      for (int c = 0; c < n; ++c) {
        double t = a[(size_t)k * n + c];
        a[(size_t)k * n + c] = a[(size_t)p * n + c];
        a[(size_t)p * n + c] = t;
      }
    }
    const double inv = 1.0 / a[(size_t)k * n + k];
    for (int r = k + 1; r < n; ++r) {
      const double f = a[(size_t)r * n + k] * inv;
      a[(size_t)r * n + k] = f;
      if (f != 0.0)
        for (int c = k + 1; c < n; ++c) a[(size_t)r * n + c] -= f * a[(size_t)k * n + c];
    }
  }
  return 0;
}

static void lu_solve(const double *a, int n, const int *piv, double *b) {
  for (int k = 0; k < n; ++k) {
    const int p = piv[k];
    if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
  }
  for (int r = 1; r < n; ++r) {
    double s = b[r];
    for (int c = 0; c < r; ++c) s -= a[(size_t)r * n + c] * b[c];
    b[r] = s;
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int c = r + 1; c < n; ++c) s -= a[(size_t)r * n + c] * b[c];
    b[r] = s / a[(size_t)r * n + r];
  }
}

/* ------------------------------------------------------------------------ */
/* One agent's local QP (Eq. 3 / compact Eq. 6)                              */
/* ------------------------------------------------------------------------ */

typedef struct {
  const orc_params *prm;
  int T, n_nbr, nx, nu, dp, nv, nd;
  const double *x0;
  const double *qd;  /* diagonal of Q */
  const double *lo, *hi;  /* input box of this agent */
  const double *A, *B;    /* dynamics of this agent, row-major nx*nx and nx*nu */
  double *Hd;      /* [nv] diagonal of H                       */
  double *cv;      /* [nv] linear term                          */
  /* KKT factor cache, valid for the working set stored in wkey */
  double *K;
  int *piv;
  signed char *wkey;
  int nk_cached;
  int cache_valid;
} qp_ws;

static int iu(const qp_ws *q, int t, int c) { return t * q->nu + c; }
static int ix(const qp_ws *q, int t, int r) { return q->T * q->nu + (t - 1) * q->nx + r; } /* t >= 1 */

/* The state box covers two groups of states, each only where one of its
 * bounds is finite: the positions (state r < dp; p_lo, p_hi) and the other
 * states (r >= dp; s_lo, s_hi). */
static int state_boxed(const orc_params *prm, int r) {
  if (!prm->state_box) return 0;
  const double *lo = r < prm->dp ? prm->p_lo : prm->s_lo, *hi = r < prm->dp ? prm->p_hi : prm->s_hi;
  for (int c = 0; c < prm->dp; ++c)
    if (isfinite(lo[c]) || isfinite(hi[c])) return 1;
  return 0;
}
static double state_lo(const orc_params *prm, int r) { return r < prm->dp ? prm->p_lo[r] : prm->s_lo[r - prm->dp]; }
static double state_hi(const orc_params *prm, int r) { return r < prm->dp ? prm->p_hi[r] : prm->s_hi[r - prm->dp]; }

/* Equality-constrained QP for working set W: dynamics plus u_tc fixed at its
 * bound for every (t,c) in W.  KKT system
 *     [H  E'] [w]   [-c]
 *     [E  0 ] [y] = [ e]
 * sol receives (w, y_dyn, y_fix); returns 0 on success. */
static int eqp_solve(qp_ws *q, const signed char *W, double *sol, long *facts) {
  const orc_params *prm = q->prm;
  const int T = q->T, nx = q->nx, nu = q->nu, nv = q->nv, nd = q->nd;
  int na = 0;
  for (int k = 0; k < T * nu; ++k) na += (W[k] != 0);
  const int nk = nv + nd + na;

  int reuse = prm->lu_reuse && q->cache_valid && q->nk_cached == nk &&
              memcmp(q->wkey, W, (size_t)T * nu) == 0;
  if (!reuse) {
    double *K = q->K;
    memset(K, 0, sizeof(double) * (size_t)nk * nk);
    for (int k = 0; k < nv; ++k) K[(size_t)k * nk + k] = q->Hd[k];
    for (int t = 0; t < T; ++t) {
      for (int r = 0; r < nx; ++r) {
        const int R = nv + t * nx + r;
        /* x_{t+1,r} - sum_c A_rc x_{t,c} - sum_c B_rc u_{t,c} = (t == 0 ? (A x0)_r : 0) */
        const int cx1 = ix(q, t + 1, r);
        K[(size_t)R * nk + cx1] = 1.0;
        K[(size_t)cx1 * nk + R] = 1.0;
        if (t >= 1) {
          for (int c = 0; c < nx; ++c) {
            const double a = q->A[r * nx + c];
            if (a == 0.0) continue;
            const int col = ix(q, t, c);
            K[(size_t)R * nk + col] = -a;
            K[(size_t)col * nk + R] = -a;
          }
        }
        for (int c = 0; c < nu; ++c) {
          const double b = q->B[r * nu + c];
          if (b == 0.0) continue;
          const int col = iu(q, t, c);
          K[(size_t)R * nk + col] = -b;
          K[(size_t)col * nk + R] = -b;
        }
      }
    }
    int a = 0;
    for (int k = 0; k < T * nu; ++k) {
      if (!W[k]) continue;
      const int R = nv + nd + a;
      K[(size_t)R * nk + k] = 1.0;   /* u block is at columns 0..T*nu-1 in flat (t,c) order */
      K[(size_t)k * nk + R] = 1.0;
      ++a;
    }
    if (lu_factor(K, nk, q->piv)) { q->cache_valid = 0; return 1; }
    memcpy(q->wkey, W, (size_t)T * nu);
    q->nk_cached = nk;
    q->cache_valid = 1;
    if (facts) ++*facts;
  }
  for (int k = 0; k < nv; ++k) sol[k] = -q->cv[k];
  for (int t = 0; t < T; ++t)
    for (int r = 0; r < nx; ++r) {
      double e = 0.0;
      if (t == 0)
        for (int c = 0; c < nx; ++c) e += q->A[r * nx + c] * q->x0[c];
      sol[nv + t * nx + r] = e;
    }
  int a = 0;
  for (int k = 0; k < T * nu; ++k) {
    if (!W[k]) continue;
    const int c = k % nu;
    sol[nv + nd + a] = (W[k] == 1) ? q->lo[c] : q->hi[c];
    ++a;
  }
  lu_solve(q->K, nk, q->piv, sol);
  return 0;
}

static void rollout(const qp_ws *q, double *x, const double *u) {
  const int nx = q->nx, nu = q->nu;
  for (int r = 0; r < nx; ++r) x[r] = q->x0[r];
  for (int t = 0; t < q->T; ++t) {
    for (int r = 0; r < nx; ++r) {
      double v = 0.0;
      for (int c = 0; c < nx; ++c) v += q->A[r * nx + c] * x[t * nx + c];
      for (int c = 0; c < nu; ++c) v += q->B[r * nu + c] * u[t * nu + c];
      x[(t + 1) * nx + r] = v;
    }
  }
}

static int qp_ws_init(qp_ws *q, const orc_params *prm, int T, int n_nbr, const double *x0,
                      const double *xref, const double *qd, const double *rd, const double *ysum) {
  memset(q, 0, sizeof(*q));
  q->prm = prm; q->T = T; q->n_nbr = n_nbr; q->nx = prm->nx; q->nu = prm->nu; q->dp = prm->dp;
  q->nv = T * (q->nu + q->nx);
  q->nd = T * q->nx;
  q->x0 = x0;
  q->qd = qd;
  q->lo = prm->u_lo;
  q->hi = prm->u_hi;
  q->A = prm->A;
  q->B = prm->B;
  const int nkmax = q->nv + q->nd + T * q->nu;
  q->Hd = (double *)malloc(sizeof(double) * q->nv);
  q->cv = (double *)malloc(sizeof(double) * q->nv);
  q->K = (double *)malloc(sizeof(double) * (size_t)nkmax * nkmax);
  q->piv = (int *)malloc(sizeof(int) * nkmax);
  q->wkey = (signed char *)malloc((size_t)T * q->nu);
  if (!q->Hd || !q->cv || !q->K || !q->piv || !q->wkey) return 1;
  for (int t = 0; t < T; ++t)
    for (int c = 0; c < q->nu; ++c) {
      q->Hd[iu(q, t, c)] = 2.0 * rd[c];
      q->cv[iu(q, t, c)] = 0.0;
    }
  for (int t = 1; t <= T; ++t)
    for (int r = 0; r < q->nx; ++r) {
      const double wq = (t == T ? prm->qT_scale : 1.0) * qd[r];
      const int k = ix(q, t, r);
      q->Hd[k] = 2.0 * wq + (r < q->dp ? prm->rho * (double)n_nbr : 0.0) + (state_boxed(prm, r) ? prm->rho : 0.0);
      q->cv[k] = -2.0 * wq * xref[t * q->nx + r] - (r < q->dp && ysum ? ysum[t * q->dp + r] : 0.0);
    }
  return 0;
}

/* ysum [T+1][dp]: sum_j (rho z - lambda) on the positions; vsum [T+1][nx]
 * (or NULL): sigma y - mu on the boxed states (0 elsewhere). */
static void qp_ws_set_linear(qp_ws *q, const double *xref, const double *qd, const double *ysum,
                             const double *vsum) {
  const int dp = q->dp;
  for (int t = 1; t <= q->T; ++t)
    for (int r = 0; r < q->nx; ++r) {
      const double wq = (t == q->T ? q->prm->qT_scale : 1.0) * qd[r];
      double v = -2.0 * wq * xref[t * q->nx + r];
      if (r < dp && ysum) v -= ysum[t * dp + r];
      if (vsum) v -= vsum[t * q->nx + r];
      q->cv[ix(q, t, r)] = v;
    }
}

/* A new penalty rho: the position entries of H change, so the cached KKT
 * factors no longer hold. */
static void qp_ws_set_rho(qp_ws *q, double rho) {
  for (int t = 1; t <= q->T; ++t)
    for (int r = 0; r < q->dp; ++r) {
      const double wq = (t == q->T ? q->prm->qT_scale : 1.0) * q->qd[r];
      q->Hd[ix(q, t, r)] = 2.0 * wq + rho * (double)q->n_nbr + (state_boxed(q->prm, r) ? q->prm->rho : 0.0);
    }
  q->cache_valid = 0;
}

static void qp_ws_free(qp_ws *q) {
  free(q->Hd); free(q->cv); free(q->K); free(q->piv); free(q->wkey);
  memset(q, 0, sizeof(*q));
}

/* Primal active-set method on the input bounds (Nocedal & Wright, Alg. 16.3),
 * with the zero-length step after a full step folded into the same pass: when
 * the equality-QP solution is feasible it is accepted and the multipliers of
 * the working set are examined right away.  Ties: lowest flat index t*nu+c. */
static int active_set(qp_ws *q, double *x, double *u, signed char *W, double *mu, int start,
                      long *passes, long *facts) {
  const orc_params *prm = q->prm;
  const int T = q->T, nx = q->nx, nu = q->nu, nv = q->nv, nd = q->nd;
  const int cap = prm->max_as_iter > 0 ? prm->max_as_iter : 10 * T * nu;
  double *sol = (double *)malloc(sizeof(double) * (nv + nd + T * nu));
  if (!sol) return -1;

  if (start == ORC_START_WARM || start == ORC_START_COLD) {
    if (start == ORC_START_WARM) {
      /* Unconstrained affine-LQ solution (the auxiliary QP of Sec. IV-B). */
      memset(W, 0, (size_t)T * nu);
      if (eqp_solve(q, W, sol, facts)) { free(sol); return -1; }
      if (passes) ++*passes;
      for (int k = 0; k < T * nu; ++k) u[k] = sol[k];
    } else {
      for (int k = 0; k < T * nu; ++k) u[k] = 0.0;
    }
    /* Clip to the box, take the clipped components as the working set and
     * roll the dynamics out so that the start point is feasible. */
    for (int k = 0; k < T * nu; ++k) {
      const int c = k % nu;
      W[k] = 0;
      if (u[k] < q->lo[c]) { u[k] = q->lo[c]; W[k] = 1; }
      else if (u[k] > q->hi[c]) { u[k] = q->hi[c]; W[k] = 2; }
    }
    rollout(q, x, u);
  }

  int rc = 1;
  for (int it = 0; it < cap; ++it) {
    if (eqp_solve(q, W, sol, facts)) { rc = -1; break; }
    if (passes) ++*passes;
    /* ratio test over the free components moving past a bound */
    double alpha = 1.0;
    int blk = -1, side = 0;
    for (int k = 0; k < T * nu; ++k) {
      if (W[k]) continue;
      const int c = k % nu;
      const double ue = sol[k], uc = u[k];
      if (ue < q->lo[c]) {
        const double r = (q->lo[c] - uc) / (ue - uc);
        if (r < alpha) { alpha = r; blk = k; side = 1; }
      } else if (ue > q->hi[c]) {
        const double r = (q->hi[c] - uc) / (ue - uc);
        if (r < alpha) { alpha = r; blk = k; side = 2; }
      }
    }
    if (blk >= 0) {
      if (alpha < 0.0) alpha = 0.0;
      for (int k = 0; k < T * nu; ++k) u[k] += alpha * (sol[k] - u[k]);
      for (int t = 1; t <= T; ++t)
        for (int r = 0; r < nx; ++r) x[t * nx + r] += alpha * (sol[ix(q, t, r)] - x[t * nx + r]);
      u[blk] = (side == 1) ? q->lo[blk % nu] : q->hi[blk % nu];
      W[blk] = (signed char)side;
      continue;
    }
    /* full step: accept the equality-QP solution */
    for (int k = 0; k < T * nu; ++k) u[k] = sol[k];
    for (int t = 1; t <= T; ++t)
      for (int r = 0; r < nx; ++r) x[t * nx + r] = sol[ix(q, t, r)];
    for (int r = 0; r < nx; ++r) x[r] = q->x0[r];
    /* multipliers of the fixed inputs: stationarity H w + c + E' y = 0 gives
     * y_fix = -dJ/du along the dynamics; lower bound mu = -y, upper mu = +y */
    double mu_min = 0.0;
    int drop = -1, a = 0;
    for (int k = 0; k < T * nu; ++k) {
      double m = 0.0;
      if (W[k]) {
        const double y = sol[nv + nd + a];
        ++a;
        m = (W[k] == 1) ? -y : y;
        if (m < mu_min) { mu_min = m; drop = k; }
      }
      if (mu) mu[k] = m;
    }
    if (drop >= 0 && mu_min < -prm->mu_tol) {
      W[drop] = 0;
      continue;
    }
    rc = 0;
    break;
  }
  free(sol);
  return rc;
}

int orc_agent_qp(const orc_params *prm, int T, int n_nbr, const double *x0, const double *xref,
                 const double *q_diag, const double *r_diag, const double *ysum,
                 double *x, double *u, signed char *w, double *mu, int start,
                 long *passes, long *facts) {
  qp_ws q;
  if (qp_ws_init(&q, prm, T, n_nbr, x0, xref, q_diag, r_diag, ysum)) { qp_ws_free(&q); return -1; }
  const int rc = active_set(&q, x, u, w, mu, start, passes, facts);
  qp_ws_free(&q);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Consensus normals (linearisation of ||p_i - p_j|| >= d_min, Sec. III-A)    */
/* ------------------------------------------------------------------------ */

static void reference_normal(const orc_params *prm, const orc_scenario *sc, int i, int j, int t, double *n) {
  const int nx = prm->nx, dp = prm->dp;
  const double *ri = sc->xref + ((size_t)i * (sc->T + 1) + t) * nx;
  const double *rj = sc->xref + ((size_t)j * (sc->T + 1) + t) * nx;
  double d[3] = {0, 0, 0}, nn = 0.0;
  for (int k = 0; k < dp; ++k) { d[k] = ri[k] - rj[k]; nn += d[k] * d[k]; }
  nn = sqrt(nn);
  if (nn >= 1e-6) { for (int k = 0; k < dp; ++k) n[k] = d[k] / nn; return; }
  double v[3] = {0, 0, 0}, nv = 0.0;
  for (int k = 0; k < dp; ++k) { v[k] = ri[dp + k] - rj[dp + k]; nv += v[k] * v[k]; }
  nv = sqrt(nv);
  if (nv >= 1e-6) {
    double c[3] = {0, 0, 0};
    if (dp == 2) { c[0] = -v[1]; c[1] = v[0]; }
    else {
      int kmin = 0;
      for (int k = 1; k < 3; ++k) if (fabs(v[k]) < fabs(v[kmin])) kmin = k;
      double e[3] = {0, 0, 0};
      e[kmin] = 1.0;
      c[0] = v[1] * e[2] - v[2] * e[1];
      c[1] = v[2] * e[0] - v[0] * e[2];
      c[2] = v[0] * e[1] - v[1] * e[0];
    }
    double cn = 0.0;
    for (int k = 0; k < dp; ++k) cn += c[k] * c[k];
    cn = sqrt(cn);
    if (cn > 0.0) { for (int k = 0; k < dp; ++k) n[k] = c[k] / cn; return; }
  }
  for (int k = 0; k < dp; ++k) n[k] = (k == 0) ? 1.0 : 0.0;
}

/* ------------------------------------------------------------------------ */
/* ADMM on one scenario                                                      */
/* ------------------------------------------------------------------------ */

static int all_finite(const double *a, size_t n) {
  for (size_t k = 0; k < n; ++k) if (!isfinite(a[k])) return 0;
  return 1;
}

/* Weights of agent i: its own (heterogeneous agents) or the scenario's. */
static const double *agent_q(const orc_scenario *sc, int nx, int i) {
  return sc->agent_q ? sc->agent_q + (size_t)i * nx : sc->q_diag;
}
static const double *agent_r(const orc_scenario *sc, int nu, int i) {
  return sc->agent_r ? sc->agent_r + (size_t)i * nu : sc->r_diag;
}

int orc_admm(const orc_params *prm, const orc_scenario *sc, orc_result *res, int threads) {
  const int N = sc->N, T = sc->T, nx = prm->nx, nu = prm->nu, dp = prm->dp;
  const int P = N * (N - 1) / 2;
  double rho = prm->rho;
  const size_t zsz = (size_t)N * N * T * dp;
  if (threads < 1) threads = 1;

  double *z = (double *)calloc(zsz, sizeof(double));
  double *lam = (double *)calloc(zsz, sizeof(double));
  double *zsum_old = (double *)calloc((size_t)N * T * dp, sizeof(double));
  double *ysum = (double *)calloc((size_t)N * (T + 1) * dp, sizeof(double));
  /* state box split: yb in the box, its dual mb, vsum = sigma yb - mb, per
   * agent, step and state ([N][T+1][nx]; entries of unboxed states stay 0) */
  const int box = state_boxed(prm, 0) || state_boxed(prm, dp);
  const int relax = prm->alpha != 1.0;
  const double sigma = prm->rho;
  double *yb = (double *)calloc((size_t)N * (T + 1) * nx, sizeof(double));
  double *mb = (double *)calloc((size_t)N * (T + 1) * nx, sizeof(double));
  double *vsum = (double *)calloc((size_t)N * (T + 1) * nx, sizeof(double));
  /* momentum (fast ADMM with restart, Goldstein et al. 2014, Alg. 8): the
   * extrapolated copies zh and duals lh that the next iteration uses, and
   * the previous iterates zp, lp; plain ADMM otherwise, and not combined
   * with the other variants */
  const int mom = prm->momentum;
  if (mom && (box || relax || prm->adaptive_rho)) return -1;
  double *zh = (double *)calloc(zsz, sizeof(double));
  double *lh = (double *)calloc(zsz, sizeof(double));
  double *zp = (double *)calloc(zsz, sizeof(double));
  double *lp = (double *)calloc(zsz, sizeof(double));
  double mom_a = 1.0, mom_c = INFINITY;
  qp_ws *qs = (qp_ws *)calloc((size_t)N, sizeof(qp_ws));
  if (!z || !lam || !zsum_old || !ysum || !qs || !yb || !mb || !vsum || !zh || !lh || !zp || !lp) {
    free(z); free(lam); free(zsum_old); free(ysum); free(qs); free(yb); free(mb); free(vsum);
    free(zh); free(lh); free(zp); free(lp);
    return -1;
  }
#define ZI(i, j, t) (((size_t)(i) * N + (j)) * T + ((t) - 1)) * dp
  const int maxit = prm->fixed_iters > 0 ? prm->fixed_iters : prm->max_iter;

  /* z^(0)_ij,t = C r_i,t ; lambda^(0) = 0 */
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      if (i == j) continue;
      for (int t = 1; t <= T; ++t)
        for (int k = 0; k < dp; ++k)
          z[ZI(i, j, t) + k] = sc->xref[((size_t)i * (T + 1) + t) * nx + k];
    }
  /* momentum: zh^(1) = z^(0), lh^(1) = lambda^(0) = 0, alpha_1 = 1, c_0 = inf */
  if (mom) { memcpy(zh, z, zsz * sizeof(double)); memcpy(zp, z, zsz * sizeof(double)); }
  /* y^(0): the references' boxed states, clipped; mu^(0) = 0 */
  if (box)
    for (int i = 0; i < N; ++i)
      for (int t = 1; t <= T; ++t)
        for (int r = 0; r < nx; ++r) {
          if (!state_boxed(prm, r)) continue;
          const size_t o = ((size_t)i * (T + 1) + t) * nx + r;
          yb[o] = fmin(fmax(sc->xref[o], state_lo(prm, r)), state_hi(prm, r));
        }
  int setup_fail = 0;
  for (int i = 0; i < N; ++i) {
    setup_fail |= qp_ws_init(&qs[i], prm, T, N - 1, sc->x0 + (size_t)i * nx,
                             sc->xref + (size_t)i * (T + 1) * nx, agent_q(sc, nx, i), agent_r(sc, nu, i), NULL);
    if (sc->agent_lo) qs[i].lo = sc->agent_lo + (size_t)i * nu;
    if (sc->agent_hi) qs[i].hi = sc->agent_hi + (size_t)i * nu;
    if (sc->agent_A) qs[i].A = sc->agent_A + (size_t)i * nx * nx;
    if (sc->agent_B) qs[i].B = sc->agent_B + (size_t)i * nx * nu;
  }
  res->status = ORC_MAX_ITER;
  res->iters = 0;
  res->as_passes = 0;
  res->lu_factorizations = 0;
  res->r_norm = res->s_norm = res->eps_pri = res->eps_dual = 0.0;
  memset(res->pair_active, 0, (size_t)P * T);
  if (setup_fail) goto done_fail;

  for (int k = 1; k <= maxit; ++k) {
    /* ---- x-update: each agent's local QP (Eq. 3), independent ---- */
    for (int i = 0; i < N; ++i) {
      double *ys = ysum + (size_t)i * (T + 1) * dp;
      for (int t = 1; t <= T; ++t)
        for (int c = 0; c < dp; ++c) {
          double s = 0.0;
          for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            s += mom ? rho * zh[ZI(i, j, t) + c] - lh[ZI(i, j, t) + c] : rho * z[ZI(i, j, t) + c] - lam[ZI(i, j, t) + c];
          }
          ys[t * dp + c] = s;
        }
    }
    int cap_hit = 0, fail = 0;
    long passes = 0, facts = 0;
#pragma omp parallel for schedule(dynamic) num_threads(threads) reduction(| : cap_hit, fail) reduction(+ : passes, facts)
    for (int i = 0; i < N; ++i) {
      qp_ws *q = &qs[i];
      if (box)
        for (int e = 0; e < (T + 1) * nx; ++e) {
          const size_t o = (size_t)i * (T + 1) * nx + e;
          vsum[o] = sigma * yb[o] - mb[o];
        }
      qp_ws_set_linear(q, sc->xref + (size_t)i * (T + 1) * nx, agent_q(sc, nx, i), ysum + (size_t)i * (T + 1) * dp,
                       box ? vsum + (size_t)i * (T + 1) * nx : NULL);
      int start = ORC_START_PREV;
      if (k == 1 || !prm->hotstart) start = prm->warm_start ? ORC_START_WARM : ORC_START_COLD;
      const int rc = active_set(q, res->x + (size_t)i * (T + 1) * nx, res->u + (size_t)i * T * nu,
                                res->w + (size_t)i * T * nu, res->mu + (size_t)i * T * nu, start,
                                &passes, &facts);
      if (rc == 1) cap_hit = 1;
      if (rc < 0) fail = 1;
    }
    res->as_passes += passes;
    res->lu_factorizations += facts;
    res->iters = k;
    if (fail) goto done_fail;
    if (cap_hit) { res->status = ORC_ACTIVE_SET_CAP; break; }

    /* previous consensus sums, for the dual residual */
    for (int i = 0; i < N; ++i)
      for (int t = 1; t <= T; ++t)
        for (int c = 0; c < dp; ++c) {
          double s = 0.0;
          for (int j = 0; j < N; ++j) if (j != i) s += mom ? zh[ZI(i, j, t) + c] : z[ZI(i, j, t) + c];
          zsum_old[((size_t)i * T + (t - 1)) * dp + c] = s;
        }
    /* momentum: the consensus and dual updates start from the extrapolated
     * duals; keep the previous iterates for the next extrapolation */
    if (mom) {
      memcpy(zp, z, zsz * sizeof(double));
      memcpy(lp, lam, zsz * sizeof(double));
      memcpy(lam, lh, zsz * sizeof(double));
    }

    /* ---- z-update (Eq. 4) and dual update (Eq. 5) for every pair and step ---- */
    int p = 0;
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j, ++p)
        for (int t = 1; t <= T; ++t) {
          const double *pi = res->x + ((size_t)i * (T + 1) + t) * nx;
          const double *pj = res->x + ((size_t)j * (T + 1) + t) * nx;
          double n[3] = {0, 0, 0};
          if (prm->normal_mode == ORC_NORMAL_FROZEN) {
            if (sc->normals) for (int c = 0; c < dp; ++c) n[c] = sc->normals[((size_t)p * T + (t - 1)) * dp + c];
            else reference_normal(prm, sc, i, j, t, n);
          } else {
            double dd = 0.0;
            for (int c = 0; c < dp; ++c) dd += (pi[c] - pj[c]) * (pi[c] - pj[c]);
            dd = sqrt(dd);
            if (dd >= 1e-6) for (int c = 0; c < dp; ++c) n[c] = (pi[c] - pj[c]) / dd;
            else reference_normal(prm, sc, i, j, t, n);
          }
          /* over-relaxation (Boyd et al. 2011, Sec. 3.4.3): the z- and dual
           * updates take xh = alpha C x^(k+1) + (1 - alpha) z^k in place of
           * C x^(k+1); alpha = 1 is plain ADMM */
          double xi[3], xj[3];
          for (int c = 0; c < dp; ++c) {
            xi[c] = relax ? prm->alpha * pi[c] + (1.0 - prm->alpha) * z[ZI(i, j, t) + c] : pi[c];
            xj[c] = relax ? prm->alpha * pj[c] + (1.0 - prm->alpha) * z[ZI(j, i, t) + c] : pj[c];
          }
          /* the two agents' copies shifted by their scaled duals */
          double a[3], b[3];
          for (int c = 0; c < dp; ++c) {
            a[c] = xi[c] + lam[ZI(i, j, t) + c] / rho;
            b[c] = xj[c] + lam[ZI(j, i, t) + c] / rho;
          }
          /* Euclidean projection of (a, b) onto {n'(a - b) >= d_min}: the
           * half-space normal in R^{2dp} is (n, -n) with squared norm 2 */
          double g = 0.0;
          for (int c = 0; c < dp; ++c) g += n[c] * (a[c] - b[c]);
          const double v = prm->d_min - g;
          if (v > 0.0) {
            for (int c = 0; c < dp; ++c) { a[c] += 0.5 * v * n[c]; b[c] -= 0.5 * v * n[c]; }
          }
          res->pair_active[(size_t)p * T + (t - 1)] = (unsigned char)(v > 0.0);
          for (int c = 0; c < dp; ++c) {
            z[ZI(i, j, t) + c] = a[c];
            z[ZI(j, i, t) + c] = b[c];
            lam[ZI(i, j, t) + c] += rho * (xi[c] - a[c]);
            lam[ZI(j, i, t) + c] += rho * (xj[c] - b[c]);
          }
        }

    /* ---- residuals and stopping test (Boyd et al. 2011, Sec. 3.3.1) ---- */
    double r2 = 0.0, s2 = 0.0, ax2 = 0.0, z2 = 0.0, aty2 = 0.0;
    /* the state box block: y = clip(x + mu / sigma), mu += sigma (x - y) */
    if (box)
      for (int i = 0; i < N; ++i)
        for (int t = 1; t <= T; ++t)
          for (int r = 0; r < nx; ++r) {
            if (!state_boxed(prm, r)) continue;
            const size_t o = ((size_t)i * (T + 1) + t) * nx + r;
            const double xv = res->x[o];
            const double yn = fmin(fmax(xv + mb[o] / sigma, state_lo(prm, r)), state_hi(prm, r));
            const double ds = sigma * (yn - yb[o]);
            mb[o] += sigma * (xv - yn);
            yb[o] = yn;
            r2 += (xv - yn) * (xv - yn);
            s2 += ds * ds;
            ax2 += xv * xv;
            z2 += yn * yn;
            aty2 += mb[o] * mb[o];
          }
    for (int i = 0; i < N; ++i)
      for (int t = 1; t <= T; ++t) {
        const double *pi = res->x + ((size_t)i * (T + 1) + t) * nx;
        double zs[3] = {0, 0, 0}, ls[3] = {0, 0, 0};
        for (int j = 0; j < N; ++j) {
          if (j == i) continue;
          for (int c = 0; c < dp; ++c) {
            const double zc = z[ZI(i, j, t) + c];
            r2 += (pi[c] - zc) * (pi[c] - zc);
            z2 += zc * zc;
            ax2 += pi[c] * pi[c];
            zs[c] += zc;
            ls[c] += lam[ZI(i, j, t) + c];
          }
        }
        for (int c = 0; c < dp; ++c) {
          const double ds = rho * (zs[c] - zsum_old[((size_t)i * T + (t - 1)) * dp + c]);
          s2 += ds * ds;
          aty2 += ls[c] * ls[c];
        }
      }
    const double rn = sqrt(r2), sn = sqrt(s2);
    /* rows and coupled states of the box block */
    const double nbox = (double)N * T * dp * (state_boxed(prm, 0) + state_boxed(prm, dp));
    const double eps_pri = sqrt((double)2 * P * T * dp + nbox) * prm->eps_abs + prm->eps_rel * fmax(sqrt(ax2), sqrt(z2));
    const double eps_dual = sqrt((double)N * T * dp + nbox) * prm->eps_abs + prm->eps_rel * sqrt(aty2);
    res->r_norm = rn; res->s_norm = sn; res->eps_pri = eps_pri; res->eps_dual = eps_dual;
    if (res->hist) {
      res->hist[(k - 1) * 4 + 0] = rn; res->hist[(k - 1) * 4 + 1] = sn;
      res->hist[(k - 1) * 4 + 2] = eps_pri; res->hist[(k - 1) * 4 + 3] = eps_dual;
    }
    if (res->rho_hist) res->rho_hist[k - 1] = rho;
    if (!isfinite(rn) || !isfinite(sn) || !all_finite(res->x, (size_t)N * (T + 1) * nx)) {
      res->status = ORC_NONFINITE;
      break;
    }
    const int conv = (rn <= eps_pri) && (sn <= eps_dual);
    if (prm->fixed_iters > 0) {
      if (k == maxit) res->status = conv ? ORC_CONVERGED : ORC_MAX_ITER;
    } else if (conv) {
      res->status = ORC_CONVERGED;
      break;
    }
    /* momentum: the combined residual decides between extrapolation and restart */
    if (mom && k < maxit) {
      double ck = 0.0;
      for (size_t o = 0; o < zsz; ++o) {
        const double dl = lam[o] - lh[o], dz = z[o] - zh[o];
        ck += dl * dl / rho + rho * dz * dz;
      }
      if (ck < prm->mom_eta * mom_c) {
        const double an = 0.5 * (1.0 + sqrt(1.0 + 4.0 * mom_a * mom_a));
        const double beta = (mom_a - 1.0) / an;
        for (size_t o = 0; o < zsz; ++o) {
          zh[o] = z[o] + beta * (z[o] - zp[o]);
          lh[o] = lam[o] + beta * (lam[o] - lp[o]);
        }
        mom_a = an;
        mom_c = ck;
      } else {
        memcpy(zh, zp, zsz * sizeof(double));
        memcpy(lh, lp, zsz * sizeof(double));
        mom_a = 1.0;
        mom_c = mom_c / prm->mom_eta;
      }
    }
    /* residual balancing: the next iteration's penalty (none after the last) */
    if (prm->adaptive_rho && k < maxit && k % prm->rho_every == 0) {
      double nr = rho;
      if (rn > prm->rho_mu * sn) nr = rho * prm->rho_tau;
      else if (sn > prm->rho_mu * rn) nr = rho / prm->rho_tau;
      if (nr != rho) {
        rho = nr;
        for (int i = 0; i < N; ++i) qp_ws_set_rho(&qs[i], rho);
      }
    }
  }

  if (res->z || res->lam)
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j)
        for (int t = 1; t <= T; ++t)
          for (int c = 0; c < dp; ++c) {
            const size_t o = ZI(i, j, t) + c;
            if (res->z) res->z[o] = (i == j) ? 0.0 : z[o];
            if (res->lam) res->lam[o] = (i == j) ? 0.0 : lam[o];
          }
  for (int i = 0; i < N; ++i) qp_ws_free(&qs[i]);
  free(z); free(lam); free(zsum_old); free(ysum); free(qs); free(yb); free(mb); free(vsum);
  free(zh); free(lh); free(zp); free(lp);
  return 0;

done_fail:
  for (int i = 0; i < N; ++i) qp_ws_free(&qs[i]);
  free(z); free(lam); free(zsum_old); free(ysum); free(qs); free(yb); free(mb); free(vsum);
  free(zh); free(lh); free(zp); free(lp);
  return -1;
#undef ZI
}

int orc_admm_batch(const orc_params *prm, int S, const orc_scenario *scs, orc_result *res, int threads) {
  int fail = 0;
  if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic) num_threads(threads) reduction(| : fail)
  for (int s = 0; s < S; ++s) fail |= (orc_admm(prm, &scs[s], &res[s], 1) != 0);
  return fail ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* SQP re-linearization (the outer loop around the ADMM, Sec. V-A)           */
/* ------------------------------------------------------------------------ */
/* The half-plane of pair (i < j) at step t, linearized about positions x:
 * n = (p_i - p_j) / |p_i - p_j|, or the reference normal when the two
 * positions are closer than 1e-6 (the convexification of Sec. III-A taken
 * about the current trajectories instead of the references). */
int orc_relinearize(const orc_params *prm, const orc_scenario *sc, const double *x, double *normals) {
  const int N = sc->N, T = sc->T, nx = prm->nx, dp = prm->dp;
  int p = 0;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j, ++p)
      for (int t = 1; t <= T; ++t) {
        const double *pi = x + ((size_t)i * (T + 1) + t) * nx;
        const double *pj = x + ((size_t)j * (T + 1) + t) * nx;
        double *n = normals + ((size_t)p * T + (t - 1)) * dp;
        double d[3] = {0, 0, 0}, nn = 0.0;
        for (int k = 0; k < dp; ++k) { d[k] = pi[k] - pj[k]; nn += d[k] * d[k]; }
        nn = sqrt(nn);
        if (nn >= 1e-6) for (int k = 0; k < dp; ++k) n[k] = d[k] / nn;
        else reference_normal(prm, sc, i, j, t, n);
      }
  return 0;
}
