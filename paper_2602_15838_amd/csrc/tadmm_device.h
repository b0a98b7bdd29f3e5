// Device-side building blocks of the ADMM hot path (gfx950, FP32, wave64).
//
// Work decomposition
//   * local QP (x-update, Sec. IV-A Eq. 3): one lane per agent.  The stage
//     loop is serial in t (Eqs. 7-8 are recurrences); the 4x4 / 6x6 stage
//     blocks live in VGPRs, the per-stage factors and trajectories live in
//     the scenario's workspace region, structure-of-arrays with the agent
//     index fastest, so that the lanes of a wave read consecutive words.
//   * consensus + dual update (Eqs. 4-5): one lane per agent-stage (i, t)
//     looping over the partners j.  Each lane owns its ordered copies
//     lambda_ij,t; the pair arithmetic is evaluated in canonical (i<j) order on
//     both sides so that lambda_ji = -lambda_ij holds bitwise and no atomics or
//     cross-lane reductions are needed; the per-agent sums the next x-update
//     needs fall out of the same loop.
//   * residuals: per agent-stage partial sums in the workspace, reduced by one
//     wavefront in a fixed order (deterministic, independent of the launch
//     shape, identical for the plain and the batched path).
// No MFMA: the blocks are far below the size of a matrix-core tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tadmm {

enum { SCEN_CONVERGED = 0, SCEN_MAX_ITER = 1, SCEN_CAP = 2, SCEN_NONFINITE = 3 };
enum { NORMAL_PER_ITER = 0, NORMAL_FROZEN = 1 };

// Problem constants by value in the kernel arguments.
struct Prob {
  float A[36], B[18];
  float dt, h;                   // double integrator: A = [[I, dt I], [0, I]], B = [[h I], [dt I]]
  float ulo[3], uhi[3];
  float qT, dmin, rho, eps_abs, eps_rel, mu_tol;
  float refine_band;             // refine when both residuals are within this factor of their tolerances (0: always)
  int max_iter, max_as, normal_mode, cache, warm, hot, refine;
  int cont;                      // continue from the workspace's state (a later SQP round)
  int adapt, rho_every;          // residual balancing of the per-scenario penalty
  float rho_mu, rho_tau;
  int sbox;                      // box on the non-position states (ADMM split, penalty sigma)
  float sigma, slo[3], shi[3];
  int pbox;                      // box on the positions (the same split)
  float plo[3], phi[3];
  int relax;                     // over-relaxation with factor alpha (alpha != 1)
  float alpha;
  int mom;                       // momentum (fast ADMM with restart), restart factor mom_eta
  float mom_eta;
  // the shared dynamics, in the form the dynamics products read
  __host__ __device__ __forceinline__ float a(int k) const { return A[k]; }
  __host__ __device__ __forceinline__ float b(int k) const { return B[k]; }
};

// Per-scenario table columns (int64).
enum { TB_F = 0, TB_B, TB_L, TB_A, TB_XO, TB_UO, TB_PO, TB_D, TB_NCOL };
// Per-scenario int32 state columns.
// ST_COLD: a continuing SQP round restarts the duals (the previous round did
// not converge); written by the round's bookkeeping, read by the setup.
enum { ST_STATUS = 0, ST_ITERS, ST_CAP, ST_DONE, ST_NEAR, ST_COLD, ST_NCOL = 8 };
// Per-scenario float state columns.
enum { SN_R = 0, SN_S, SN_EPRI, SN_EDUAL, SN_NCOL = 4 };
// Per-scenario counters (int64): work units, and in the batched kernel the
// time spent in each phase (ticks of the 100 MHz device real-time clock).
enum { CT_PASSES = 0, CT_REFACTOR, CT_AFFINE, CT_PAIRS, CT_T_X, CT_T_PAIR, CT_T_TEST, CT_RESERVED, CT_NCOL = 8 };
// the first CT_NXU columns are the x-update's own (passes, refactored and
// affine stages), counted per lane
constexpr int CT_NXU = 3;

struct WS {
  const int *N, *T;                  // [S]
  const long long *tab;              // [S][TB_NCOL]
  const int *order;                  // [S] launch order (largest first)
  int *queue;                        // [1] next item of the persistent queue
  float *fr;                         // float regions
  double *dr;                        // FP64 refinement scratch [NX][N(T+1)] per scenario
  int8_t *wr;                        // working-set regions  [NU][N(T+1)] per scenario
  int *adirty;                       // [agents][nu] highest stale factor stage of each local QP (-1: none)
  float *gam;                        // [T][N][N] per scenario: gamma of ordered copy (i, j) at [t][j][i]
                                     // (> 0 exactly where the half-plane was violated)
  int *sst;                          // [S][ST_NCOL]
  float *snorm;                      // [S][SN_NCOL]
  unsigned long long *cnt;           // [S][CT_NCOL]
  int *skip;                         // [S] SQP: scenario converged, not solved again
  float *rhos;                       // [S][2] penalty of the next / of the last iteration
  // over-relaxation only: per scenario 2 NU planes shaped like gam, the
  // copies' z: D = z_ij - z_ji (NU planes), then e = z_ij - C x_i (NU planes)
  float *orx;
  // momentum only: per scenario 6 NU planes shaped like gam (the copies'
  // extrapolated dual and copy, z_k, z_(k-1), lambda_k, lambda_(k-1)), and
  // per scenario [a_k, c_(k-1), beta, restart]
  float *mom;
  float *momst;
  // optional output: [S][max_iter][2] residual norms of every stopping test
  float *hist;
  float *tpart;                      // many-workgroup mode: block sums of the stopping test [blocks][5][64]
  // inputs (caller layouts)
  const float *x0, *xref, *qd, *rd, *normals;
  const float *aq, *ar, *alo, *ahi;  // heterogeneous agents (each NULL: the shared value)
  const float *aA, *aB;              // per-agent dynamics [agents][NX*NX], [agents][NX*NU] (NULL: shared)
};

// Layout of a scenario's float region: structure of arrays of 4-float groups
// over the agent-stages g = t * N + i (t = 0..T, agent index fastest).  Every
// field is padded to a multiple of 4 floats; group q = field / 4 is an array
// [GS][4] of 16-byte vectors, so the lanes of a wave (consecutive agents)
// read a group as one contiguous run and a pass over the stages fetches only
// the groups it uses.  The working set is [g][4] bytes, the FP64 refinement
// scratch [g][NX] doubles.
__host__ __device__ constexpr int pad4(int n) { return (n + 3) & ~3; }

// index of element `field` of agent-stage g in a region of GS agent-stages
__device__ __forceinline__ unsigned fidx(unsigned GS, unsigned g, int field) {
  return (unsigned)(field >> 2) * (GS * 4u) + g * 4u + (unsigned)(field & 3);
}

// the same element as (uniform group base) + (per-lane offset g * 4): the
// group base can stay in scalar registers and every group shares one offset
__device__ __forceinline__ float &fref(float *R, unsigned GS, unsigned g, int field) {
  float *grp = R + (size_t)((unsigned)(field >> 2) * (GS * 4u));
  return grp[g * 4u + (unsigned)(field & 3)];
}

template <int NX, int NU>
struct Fld {
  static constexpr int DP = NU;
  static constexpr int NS = NU * (NU + 1) / 2;  // packed symmetric NU x NU
  static constexpr int NP = NX * (NX + 1) / 2;  // packed symmetric NX x NX
  // cached Riccati factor of stage t for the current working set (read by the sweep)
  static constexpr int K = 0;                   // feedback gain K_t              [NU*NX]
  static constexpr int SV = K + pad4(NU * NX);  // S'^-1 (zero on fixed rows)     [NS]
  static constexpr int KC = SV + pad4(NS);      // feedforward constant           [NU]
  static constexpr int CC = KC + pad4(NU);      // value-gradient constant c_t    [NX]
  // linear term of the local QP at stage t:
  //   q_t = -2 Q_t r_t - C' sum_j (rho z_ij,t - lambda_ij,t);
  // its velocity part (constant) is here, its position part in QZ
  static constexpr int Q = CC + pad4(NX);       //                                [NX]
  static constexpr int PV = Q + pad4(NX);       // affine value term p_t          [NX]
  static constexpr int KV = PV + pad4(NX);      // affine feedforward k_t         [NU]
  static constexpr int U = KV + pad4(NU);       // current iterate u_t            [NU]
  static constexpr int X = U + pad4(NU);        // current iterate x_t            [NX]
  static constexpr int UE = X + pad4(NX);       // equality-QP solution u_t       [NU]
  // (the previous positions C x^k are a dense array after the inputs)
  // written together by every consensus step: the position part of q,
  //   GQP - rho n_nbr C x^k_t - sum_j (lambda_ij^(k-1) - 2 lambda_ij^k)
  // (from the small dual part: no long sums of position-sized terms in
  // FP32), then ZD = sum_j z_ij - n_nbr C x^k                      [2 DP]
  static constexpr int QZ = UE + pad4(NU);
  static constexpr int GQP = QZ + pad4(2 * DP);  // -2 Q_t r_t, positions          [DP]
  // state box on the non-position states: the copy y and its dual mu
  // [2 DP], and the constant velocity tracking term -2 Q_t r_t     [DP]
  static constexpr int YM = GQP + pad4(DP);
  static constexpr int GQV = YM + pad4(2 * DP);
  static constexpr int YP = GQV + pad4(DP);     // position box: copy y and dual mu [2 DP]
  static constexpr int PU = YP + pad4(2 * DP);  // value Hessian P_t (upper)      [NP]
  static constexpr int RED = PU + pad4(NP);     // residual partial sums          [5]
  static constexpr int NF = RED + pad4(5);
};

template <int N>
__host__ __device__ constexpr int sym_idx(int r, int c) {  // r <= c
  return r * N - r * (r - 1) / 2 + (c - r);
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct Scen {
  int s, N, T, GS;
  long long fo, bo, lo, ao, xo, uo, po, dof;
};

// Scenario descriptors are wave-uniform; readfirstlane tells the compiler so
// (the table is read with vector loads because the kernels also write global
// memory), which keeps the region bases in scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni64(long long v) {
  const unsigned lo = (unsigned)uni((int)(unsigned)(v & 0xffffffffll));
  const unsigned hi = (unsigned)uni((int)(unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ Scen load_scen(const WS &ws, int s) {
  Scen sc;
  sc.s = uni(s);
  sc.N = uni(ws.N[sc.s]);
  sc.T = uni(ws.T[sc.s]);
  sc.GS = sc.N * (sc.T + 1);
  const long long *tb = ws.tab + (long long)sc.s * TB_NCOL;
  sc.fo = uni64(tb[TB_F]); sc.bo = uni64(tb[TB_B]); sc.lo = uni64(tb[TB_L]); sc.ao = uni64(tb[TB_A]);
  sc.xo = uni64(tb[TB_XO]); sc.uo = uni64(tb[TB_UO]); sc.po = uni64(tb[TB_PO]);
  sc.dof = uni64(tb[TB_D]);
  return sc;
}

// ---------------------------------------------------------------------------
// Dynamics x_{t+1} = A x_t + B u_t: products with A, A', B, B'.  The general
// form reads A and B through pb.a() / pb.b() (the kernel arguments, or an
// agent's own matrices); the double-integrator form
// (A = [[I, dt I], [0, I]], B = [[dt^2/2 I], [dt I]], positions first) uses
// only dt and h = dt^2/2 and is selected by the host when A and B have it.
// ---------------------------------------------------------------------------
template <int NX, int NU, bool DI>
struct Dyn;

template <int NX, int NU>
struct Dyn<NX, NU, false> {
  template <class M, class R>
  __device__ static __forceinline__ void ax(const M &pb, const R *x, R *y) {
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      R v = R(0);
#pragma unroll
      for (int c = 0; c < NX; ++c) v = fma((R)pb.a(r * NX + c), x[c], v);
      y[r] = v;
    }
  }
  template <class M, class R>
  __device__ static __forceinline__ void atx(const M &pb, const R *x, R *y) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      R v = R(0);
#pragma unroll
      for (int r = 0; r < NX; ++r) v = fma((R)pb.a(r * NX + c), x[r], v);
      y[c] = v;
    }
  }
  template <class M, class R>
  __device__ static __forceinline__ void add_bu(const M &pb, const R *u, R *y) {
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      R v = y[r];
#pragma unroll
      for (int a = 0; a < NU; ++a) v = fma((R)pb.b(r * NU + a), u[a], v);
      y[r] = v;
    }
  }
  template <class M, class R>
  __device__ static __forceinline__ void btx(const M &pb, const R *x, R *y) {
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      R v = R(0);
#pragma unroll
      for (int r = 0; r < NX; ++r) v = fma((R)pb.b(r * NU + a), x[r], v);
      y[a] = v;
    }
  }
};

template <int NX, int NU>
struct Dyn<NX, NU, true> {
  template <class M, class R>
  __device__ static __forceinline__ void ax(const M &pb, const R *x, R *y) {
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      y[c] = fma((R)pb.dt, x[NU + c], x[c]);
      y[NU + c] = x[NU + c];
    }
  }
  template <class M, class R>
  __device__ static __forceinline__ void atx(const M &pb, const R *x, R *y) {
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      y[c] = x[c];
      y[NU + c] = fma((R)pb.dt, x[c], x[NU + c]);
    }
  }
  template <class M, class R>
  __device__ static __forceinline__ void add_bu(const M &pb, const R *u, R *y) {
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      y[c] = fma((R)pb.h, u[c], y[c]);
      y[NU + c] = fma((R)pb.dt, u[c], y[NU + c]);
    }
  }
  template <class M, class R>
  __device__ static __forceinline__ void btx(const M &pb, const R *x, R *y) {
#pragma unroll
    for (int a = 0; a < NU; ++a) y[a] = fma((R)pb.dt, x[NU + a], (R)pb.h * x[a]);
  }
};

// Stage weights (cost Eq. 1 without 1/2, penalty (rho/2)||.||^2 per partner):
// H_x,t = 2 Q_t + rho n_nbr C'C with Q_T = qT Q, plus sigma on the non-position
// states with the state box; H_u = 2 R.
template <int NX, int NU>
__device__ __forceinline__ void stage_hx(const Prob &pb, const float *qd, int t, int T, int n_nbr, float rho,
                                         float hx[NX]) {
  const float w = (t == T) ? pb.qT : 1.0f;
#pragma unroll
  for (int r = 0; r < NX; ++r)
    hx[r] = 2.0f * w * qd[r] + (r < NU ? rho * (float)n_nbr + (pb.pbox ? pb.sigma : 0.0f)
                                       : (pb.sbox ? pb.sigma : 0.0f));
}

// ---------------------------------------------------------------------------
// Riccati factor of one stage for a working set (Eq. 7 with inputs fixed),
// in the real type R (FP32 for the ADMM iterations; the equality-QP solves of
// the adjoint also instantiate it in FP64)
// ---------------------------------------------------------------------------
// Given P_{t+1}, the free/fixed pattern of u_t and the bound values ubar
// (lo[a] or hi[a] on a fixed input):
//   S = H_u + B'P B,  M = B'P A,  S' = S on the free block, identity elsewhere,
//   Sv = S'^-1 with the fixed rows/columns zeroed (the inverse of S_ff),
//   K = -Sv M (zero rows on fixed inputs),
//   kc = -Sv (S ubar) on free rows, ubar on fixed rows,
//   c = K' (S ubar)_f + M' ubar,
//   P_t = H_x + A'P A + M'K (symmetric; only for t >= 1).
// With these, the affine terms of the sweep are
//   k_t = kc - Sv B'p_{t+1},   p_t = q_t + c + A'p_{t+1} + K' B'p_{t+1},
// since A + B K is the closed loop and -Sv B' the gain of k_t on p_{t+1}.
template <int NX, int NU, bool DI, class R, class DM>
__device__ __forceinline__ void factor_stage(const DM &pb, const R hx[NX], const R hu[NU], const R Pn[NX][NX],
                                             const int8_t wt[NU], const float *lo, const float *hi, bool want_P,
                                             R Pt[NX][NX], R K[NU][NX], R Sv[NU][NU], R kc[NU], R cc[NX]) {
  using D = Dyn<NX, NU, DI>;
  R PB[NX][NU];  // row r of P B is B' (row r of P), P symmetric
#pragma unroll
  for (int r = 0; r < NX; ++r) D::btx(pb, Pn[r], PB[r]);
  R S[NU][NU];
#pragma unroll
  for (int b = 0; b < NU; ++b) {
    R col[NX], sb[NU];
#pragma unroll
    for (int r = 0; r < NX; ++r) col[r] = PB[r][b];
    D::btx(pb, col, sb);
#pragma unroll
    for (int a = 0; a < NU; ++a) S[a][b] = sb[a] + ((a == b) ? hu[a] : R(0));
  }
  R M[NU][NX];  // row a of B'P A is A' (column a of P B)
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    R col[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) col[r] = PB[r][a];
    D::atx(pb, col, M[a]);
  }
  bool fr[NU];
  R ub[NU];
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    fr[a] = (wt[a] == 0);
    ub[a] = (wt[a] == 1) ? (R)lo[a] : ((wt[a] == 2) ? (R)hi[a] : R(0));
  }
  // Cholesky of S' (lower) with reciprocal diagonal
  R L[NU][NU], Li[NU];
#pragma unroll
  for (int a = 0; a < NU; ++a)
#pragma unroll
    for (int b = 0; b < NU; ++b) L[a][b] = R(0);
#pragma unroll
  for (int a = 0; a < NU; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      R v = (fr[a] && fr[b]) ? S[a][b] : (a == b ? R(1) : R(0));
#pragma unroll
      for (int k = 0; k < b; ++k) v = fma(-L[a][k], L[b][k], v);
      if (a == b) {
        const R d = sqrt(v);
        L[a][a] = d;
        Li[a] = R(1) / d;
      } else {
        L[a][b] = v * Li[b];
      }
    }
  }
  // Sv = S'^-1 column by column, fixed rows/columns zeroed
#pragma unroll
  for (int b = 0; b < NU; ++b) {
    R y[NU];
#pragma unroll
    for (int a = 0; a < NU; ++a) y[a] = (a == b) ? R(1) : R(0);
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      R v = y[a];
#pragma unroll
      for (int k = 0; k < a; ++k) v = fma(-L[a][k], y[k], v);
      y[a] = v * Li[a];
    }
#pragma unroll
    for (int a = NU - 1; a >= 0; --a) {
      R v = y[a];
#pragma unroll
      for (int k = a + 1; k < NU; ++k) v = fma(-L[k][a], y[k], v);
      y[a] = v * Li[a];
    }
#pragma unroll
    for (int a = 0; a < NU; ++a) Sv[a][b] = (fr[a] && fr[b]) ? y[a] : R(0);
  }
  R su[NU];  // (S ubar) on the free rows
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    R v = R(0);
#pragma unroll
    for (int b = 0; b < NU; ++b) v = fma(S[a][b], ub[b], v);
    su[a] = fr[a] ? v : R(0);
  }
#pragma unroll
  for (int a = 0; a < NU; ++a) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      R v = R(0);
#pragma unroll
      for (int b = 0; b < NU; ++b) v = fma(Sv[a][b], M[b][c], v);
      K[a][c] = -v;
    }
    R v = R(0);
#pragma unroll
    for (int b = 0; b < NU; ++b) v = fma(Sv[a][b], su[b], v);
    kc[a] = fr[a] ? -v : ub[a];
  }
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    R v = R(0);
#pragma unroll
    for (int a = 0; a < NU; ++a) v = fma(K[a][r], su[a], fma(M[a][r], ub[a], v));
    cc[r] = v;
  }
  if (want_P) {
    R PA[NX][NX];  // row r of P A is A' (row r of P)
#pragma unroll
    for (int r = 0; r < NX; ++r) D::atx(pb, Pn[r], PA[r]);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      R col[NX], apa[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) col[r] = PA[r][c];
      D::atx(pb, col, apa);   // column c of A'P A
#pragma unroll
      for (int r = 0; r <= c; ++r) {
        R v = apa[r] + ((r == c) ? hx[r] : R(0));
#pragma unroll
        for (int a = 0; a < NU; ++a) v = fma(M[a][r], K[a][c], v);
        Pt[r][c] = v;
        Pt[c][r] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Reference normal: the fallback when two positions coincide (< 1e-6) and the
// FROZEN default.  Normalised reference relative position; else the relative
// reference velocity turned by 90 degrees (2-D) or crossed with the axis of
// its smallest component (3-D); else e_1.
// ---------------------------------------------------------------------------
// Unit vector n = d / |d| of a position difference, by one hardware
// reciprocal square root (about 1 ulp) and NU products instead of a rounded
// square root and NU divisions; false (n untouched) when |d| < 1e-6.  The
// pair phase and the polish both take their normals from here, so a normal
// recomputed from the same positions is bitwise the same everywhere.
template <int NU>
__device__ __forceinline__ bool unit_normal(const float d[NU], float n[NU]) {
  float dd = 0.f;
#pragma unroll
  for (int c = 0; c < NU; ++c) dd = fmaf(d[c], d[c], dd);
  if (!(dd >= 1e-12f)) return false;
  const float r = __builtin_amdgcn_rsqf(dd);
#pragma unroll
  for (int c = 0; c < NU; ++c) n[c] = d[c] * r;
  return true;
}

template <int NX, int NU>
__device__ __forceinline__ void reference_normal(const WS &ws, const Scen &sc, int a, int b, int t, float n[NU]) {
  const float *ra = ws.xref + (sc.xo + (long long)a * (sc.T + 1) + t) * NX;
  const float *rb = ws.xref + (sc.xo + (long long)b * (sc.T + 1) + t) * NX;
  float d[NU], dd = 0.f;
#pragma unroll
  for (int c = 0; c < NU; ++c) { d[c] = ra[c] - rb[c]; dd = fmaf(d[c], d[c], dd); }
  dd = sqrtf(dd);
  if (dd >= 1e-6f) {
#pragma unroll
    for (int c = 0; c < NU; ++c) n[c] = d[c] / dd;
    return;
  }
  float v[3] = {0.f, 0.f, 0.f}, vv = 0.f;
#pragma unroll
  for (int c = 0; c < NU; ++c) { v[c] = ra[NU + c] - rb[NU + c]; vv = fmaf(v[c], v[c], vv); }
  vv = sqrtf(vv);
  if (vv >= 1e-6f) {
    float cr[3] = {0.f, 0.f, 0.f};
    if (NU == 2) {
      cr[0] = -v[1];
      cr[1] = v[0];
    } else {
      int km = 0;
      if (fabsf(v[1]) < fabsf(v[km])) km = 1;
      if (fabsf(v[2]) < fabsf(v[km])) km = 2;
      const float e0 = km == 0, e1 = km == 1, e2 = km == 2;
      cr[0] = v[1] * e2 - v[2] * e1;
      cr[1] = v[2] * e0 - v[0] * e2;
      cr[2] = v[0] * e1 - v[1] * e0;
    }
    float cn = 0.f;
#pragma unroll
    for (int c = 0; c < NU; ++c) cn = fmaf(cr[c], cr[c], cn);
    cn = sqrtf(cn);
    if (cn > 0.f) {
#pragma unroll
      for (int c = 0; c < NU; ++c) n[c] = cr[c] / cn;
      return;
    }
  }
#pragma unroll
  for (int c = 0; c < NU; ++c) n[c] = (c == 0) ? 1.f : 0.f;
}

}  // namespace tadmm
