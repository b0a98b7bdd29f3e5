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
  float ulo[3], uhi[3];
  float qT, dmin, rho, eps_abs, eps_rel, mu_tol;
  int max_iter, max_as, normal_mode, cache, warm, hot, refine;
};

// Per-scenario table columns (int64).
enum { TB_F = 0, TB_B, TB_L, TB_A, TB_XO, TB_UO, TB_PO, TB_LB, TB_D, TB_NCOL };
// Per-scenario int32 state columns.
enum { ST_STATUS = 0, ST_ITERS, ST_CAP, ST_DONE, ST_NCOL = 8 };
// Per-scenario float state columns.
enum { SN_R = 0, SN_S, SN_EPRI, SN_EDUAL, SN_NCOL = 4 };
// Per-scenario counters (int64).
enum { CT_PASSES = 0, CT_REFACTOR, CT_AFFINE, CT_PAIRS, CT_NCOL = 4 };

struct WS {
  const int *N, *T;                  // [S]
  const long long *tab;              // [S][TB_NCOL]
  const int *order;                  // [S] launch order (largest first)
  int *queue;                        // [1] next item of the persistent queue
  float *fr;                         // float regions
  double *dr;                        // FP64 refinement scratch [NX][N(T+1)] per scenario
  int8_t *wr;                        // working-set regions  [NU][N(T+1)] per scenario
  int *adirty;                       // [agents] highest stale factor stage (-1: none)
  float *lam;                        // [DP][T][N][N] per scenario
  uint8_t *pact;                     // [T][N][N] per scenario
  int *sst;                          // [S][ST_NCOL]
  float *snorm;                      // [S][SN_NCOL]
  unsigned long long *cnt;           // [S][CT_NCOL]
  // inputs (caller layouts)
  const float *x0, *xref, *qd, *rd, *normals;
};

// Field layout inside a scenario's float region: component f of agent i at
// stage t is at fr[F + f * GS + t * N + i], GS = N (T + 1).
template <int NX, int NU>
struct Fld {
  static constexpr int DP = NU;
  static constexpr int NS = NU * (NU + 1) / 2;  // packed symmetric NU x NU
  static constexpr int NP = NX * (NX + 1) / 2;  // packed symmetric NX x NX
  static constexpr int X = 0;                 // current iterate x_t        [NX]
  static constexpr int U = X + NX;            // current iterate u_t        [NU]
  static constexpr int XE = U + NU;           // equality-QP solution x_t   [NX]
  static constexpr int UE = XE + NX;          // equality-QP solution u_t   [NU]
  static constexpr int PV = UE + NU;          // affine value term p_t      [NX]
  static constexpr int KV = PV + NX;          // affine feedforward k_t     [NU]
  static constexpr int GQ = KV + NU;          // -2 Q_t r_t                 [NX]
  // linear term of the position block of the local QP:
  //   q_t = -2 Q_t r_t - sum_j (rho z_ij,t - lambda_ij,t)
  //       = GQ - rho n_nbr C x^k_t - sum_j (lambda_ij^(k-1) - 2 lambda_ij^k),
  // formed once per iteration from the small dual part (no long sums of
  // position-sized terms in FP32)
  static constexpr int QP = GQ + NX;          //                            [DP]
  static constexpr int XP = QP + DP;          // C x^k (positions of the previous iterate) [DP]
  static constexpr int ZD = XP + DP;          // sum_j z_ij - n_nbr C x^k   [DP]
  static constexpr int RED = ZD + DP;         // residual partial sums      [5]
  // cached Riccati factor of stage t for the current working set
  static constexpr int K = RED + 5;           // feedback gain K_t          [NU*NX]
  static constexpr int SV = K + NU * NX;      // S'^-1 (zero on fixed rows) [NS]
  static constexpr int KC = SV + NS;          // feedforward constant       [NU]
  static constexpr int CC = KC + NU;          // value-gradient constant    [NX]
  static constexpr int PU = CC + NX;          // value Hessian P_t (upper)  [NP]
  static constexpr int NF = PU + NP;
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
  long long fo, bo, lo, ao, xo, uo, po, lb, dof;
};

__device__ __forceinline__ Scen load_scen(const WS &ws, int s) {
  Scen sc;
  sc.s = s;
  sc.N = ws.N[s];
  sc.T = ws.T[s];
  sc.GS = sc.N * (sc.T + 1);
  const long long *tb = ws.tab + (long long)s * TB_NCOL;
  sc.fo = tb[TB_F]; sc.bo = tb[TB_B]; sc.lo = tb[TB_L]; sc.ao = tb[TB_A];
  sc.xo = tb[TB_XO]; sc.uo = tb[TB_UO]; sc.po = tb[TB_PO]; sc.lb = tb[TB_LB]; sc.dof = tb[TB_D];
  return sc;
}

// Stage weights (cost Eq. 1 without 1/2, penalty (rho/2)||.||^2 per partner):
// H_x,t = 2 Q_t + rho n_nbr C'C with Q_T = qT Q; H_u = 2 R.
template <int NX, int NU>
__device__ __forceinline__ void stage_hx(const Prob &pb, const float *qd, int t, int T, int n_nbr, float hx[NX]) {
  const float w = (t == T) ? pb.qT : 1.0f;
#pragma unroll
  for (int r = 0; r < NX; ++r) hx[r] = 2.0f * w * qd[r] + (r < NU ? pb.rho * (float)n_nbr : 0.0f);
}

// ---------------------------------------------------------------------------
// Riccati factor of one stage for a working set (Eq. 7 with inputs fixed)
// ---------------------------------------------------------------------------
// Given P_{t+1}, the free/fixed pattern of u_t and the bound values ubar:
//   S = H_u + B'P B,  M = B'P A,  S' = S on the free block, identity elsewhere,
//   Sv = S'^-1 with the fixed rows/columns zeroed (the inverse of S_ff),
//   K = -Sv M (zero rows on fixed inputs),
//   kc = -Sv (S ubar) on free rows, ubar on fixed rows,
//   c = K' (S ubar)_f + M' ubar,
//   P_t = H_x + A'P A + M'K (symmetric; only for t >= 1).
// With these, the affine terms of the sweep are
//   k_t = kc - Sv B'p_{t+1},   p_t = q_t + c + A'p_{t+1} + K' B'p_{t+1},
// since A + B K is the closed loop and -Sv B' the gain of k_t on p_{t+1}.
template <int NX, int NU>
__device__ __forceinline__ void factor_stage(const Prob &pb, const float hx[NX], const float hu[NU],
                                             const float Pn[NX][NX], const int8_t wt[NU], bool want_P,
                                             float Pt[NX][NX], float K[NU][NX], float Sv[NU][NU], float kc[NU],
                                             float cc[NX]) {
  const float *A = pb.A;
  const float *B = pb.B;
  float PB[NX][NU];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      float v = 0.f;
#pragma unroll
      for (int k = 0; k < NX; ++k) v = fmaf(Pn[r][k], B[k * NU + c], v);
      PB[r][c] = v;
    }
  float S[NU][NU];
#pragma unroll
  for (int a = 0; a < NU; ++a)
#pragma unroll
    for (int b = 0; b < NU; ++b) {
      float v = (a == b) ? hu[a] : 0.f;
#pragma unroll
      for (int r = 0; r < NX; ++r) v = fmaf(B[r * NU + a], PB[r][b], v);
      S[a][b] = v;
    }
  float M[NU][NX];  // B'P A = (P B)' A
#pragma unroll
  for (int a = 0; a < NU; ++a)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      float v = 0.f;
#pragma unroll
      for (int r = 0; r < NX; ++r) v = fmaf(PB[r][a], A[r * NX + c], v);
      M[a][c] = v;
    }
  bool fr[NU];
  float ub[NU];
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    fr[a] = (wt[a] == 0);
    ub[a] = (wt[a] == 1) ? pb.ulo[a] : ((wt[a] == 2) ? pb.uhi[a] : 0.f);
  }
  // Cholesky of S' (lower) with reciprocal diagonal
  float L[NU][NU], Li[NU];
#pragma unroll
  for (int a = 0; a < NU; ++a)
#pragma unroll
    for (int b = 0; b < NU; ++b) L[a][b] = 0.f;
#pragma unroll
  for (int a = 0; a < NU; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      float v = (fr[a] && fr[b]) ? S[a][b] : (a == b ? 1.f : 0.f);
#pragma unroll
      for (int k = 0; k < b; ++k) v = fmaf(-L[a][k], L[b][k], v);
      if (a == b) {
        const float d = sqrtf(v);
        L[a][a] = d;
        Li[a] = 1.0f / d;
      } else {
        L[a][b] = v * Li[b];
      }
    }
  }
  // Sv = S'^-1 column by column, fixed rows/columns zeroed
#pragma unroll
  for (int b = 0; b < NU; ++b) {
    float y[NU];
#pragma unroll
    for (int a = 0; a < NU; ++a) y[a] = (a == b) ? 1.f : 0.f;
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      float v = y[a];
#pragma unroll
      for (int k = 0; k < a; ++k) v = fmaf(-L[a][k], y[k], v);
      y[a] = v * Li[a];
    }
#pragma unroll
    for (int a = NU - 1; a >= 0; --a) {
      float v = y[a];
#pragma unroll
      for (int k = a + 1; k < NU; ++k) v = fmaf(-L[k][a], y[k], v);
      y[a] = v * Li[a];
    }
#pragma unroll
    for (int a = 0; a < NU; ++a) Sv[a][b] = (fr[a] && fr[b]) ? y[a] : 0.f;
  }
  float su[NU];  // (S ubar) on the free rows
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    float v = 0.f;
#pragma unroll
    for (int b = 0; b < NU; ++b) v = fmaf(S[a][b], ub[b], v);
    su[a] = fr[a] ? v : 0.f;
  }
#pragma unroll
  for (int a = 0; a < NU; ++a) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      float v = 0.f;
#pragma unroll
      for (int b = 0; b < NU; ++b) v = fmaf(Sv[a][b], M[b][c], v);
      K[a][c] = -v;
    }
    float v = 0.f;
#pragma unroll
    for (int b = 0; b < NU; ++b) v = fmaf(Sv[a][b], su[b], v);
    kc[a] = fr[a] ? -v : ub[a];
  }
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    float v = 0.f;
#pragma unroll
    for (int a = 0; a < NU; ++a) v = fmaf(K[a][r], su[a], fmaf(M[a][r], ub[a], v));
    cc[r] = v;
  }
  if (want_P) {
    float PA[NX][NX];
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < NX; ++k) v = fmaf(Pn[r][k], A[k * NX + c], v);
        PA[r][c] = v;
      }
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) {
        float v = (r == c) ? hx[r] : 0.f;
#pragma unroll
        for (int k = 0; k < NX; ++k) v = fmaf(A[k * NX + r], PA[k][c], v);
#pragma unroll
        for (int a = 0; a < NU; ++a) v = fmaf(M[a][r], K[a][c], v);
        Pt[r][c] = v;
        Pt[c][r] = v;
      }
  }
}

// ---------------------------------------------------------------------------
// Reference normal: the fallback when two positions coincide (< 1e-6) and the
// FROZEN default.  Normalised reference relative position; else the relative
// reference velocity turned by 90 degrees (2-D) or crossed with the axis of
// its smallest component (3-D); else e_1.
// ---------------------------------------------------------------------------
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
