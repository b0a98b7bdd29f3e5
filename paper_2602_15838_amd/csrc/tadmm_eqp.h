// Equality-QP solves behind the derivative of a converged solve (gfx950).
//
// The solution of the ADMM iterations is read as the solution of the
// centralized QP of Sec. III-A with its final active sets held as equalities:
// the inputs of the working sets W at their bounds, and the half-planes of
// the last consensus step that were violated (A_c) as n'(C x_i,t - C x_j,t) =
// d_min, with their normals n frozen.  That equality QP (EQP) is solved twice:
//
//   polish:  min sum_i J_i(w_i)            s.t. dynamics (x0), W at bounds, A_c
//   adjoint: min sum_i 1/2 w'H_i w - g'w   s.t. the same rows, homogeneous
//            (g = dL/dw; its solution wbar and costates give dL/dtheta by the
//            implicit function theorem).
//
// Both have the same structure: per agent an LQR with fixed inputs, coupled
// only through the held half-planes.  With multipliers nu on those rows, each
// agent's solution is an affine function of the linear term -D'nu on its
// positions (one Riccati sweep and rollout, factors of the agent QP without
// the consensus penalty), and the rows themselves give the Schur system
//   S nu = d - D w(0),   S = D H_W^-1 D'  (symmetric positive semidefinite),
// solved by MINRES: one sweep + rollout per agent per iteration, exact after
// |A_c| iterations in exact arithmetic, and a least-squares solution when the
// held rows cannot all hold (a solve stopped before convergence can leave
// such a set).  The polish starts from the multipliers of the last consensus
// step (nu = -n'lambda_ij = gamma).
//
// Work decomposition: one workgroup per scenario.  The sweeps run one lane per
// agent in the real type R (FP64, or FP32 on request), their stage data read
// in batches; the scatter of -D'nu one lane per agent-stage over the held rows
// of that agent-stage, listed once per polish in increasing partner order
// (the order of its sum); the Krylov vectors, scalars and the gradient
// reductions are FP64 with fixed-order reductions, so the result is
// deterministic.
#pragma once

#include "tadmm_device.h"

namespace tadmm {

// Per agent-stage fields of the EQP region (R values, each padded to 4).
template <int NX, int NU>
struct EFld {
  static constexpr int NS = NU * (NU + 1) / 2;
  static constexpr int K = 0;                   // feedback gain without the consensus penalty  [NU*NX]
  static constexpr int SV = K + pad4(NU * NX);  // S'^-1, packed symmetric                     [NS]
  static constexpr int KC = SV + pad4(NS);      // feedforward constant of the fixed inputs     [NU]
  static constexpr int CC = KC + pad4(NU);      // value-gradient constant of the fixed inputs  [NX]
  static constexpr int KV = CC + pad4(NX);      // affine feedforward k_t of the last sweep     [NU]
  static constexpr int E = KV + pad4(NU);       // -D'v on the positions (coupling term)        [NU]
  static constexpr int XT = E + pad4(NU);       // positions of the last rollout                [NU]
  static constexpr int XS = XT + pad4(NU);      // polished x_t                                 [NX]
  static constexpr int US = XS + pad4(NX);      // polished u_t                                 [NU]
  static constexpr int NF = US + pad4(NU);
};

// EQP workspace (pointers into the solve's workspace).  Pair-steps are
// indexed q = p T + (t - 1), p the lexicographic pair index (as the caller's
// normals); held half-planes are compacted per scenario in that order.
struct EWS {
  void *er;          // [sum N(T+1)][EFld::NF] R
  float *nrm;        // [sum P T][NU] frozen normals
  int *cidx;         // [sum P T] compact index of a held half-plane, -1 otherwise
  int2 *clist;       // [sum P T] (q, i N + j) of held half-plane k
  double *cg;        // [sum P T][6]: per scenario nu and five MINRES vectors, each P T long
  int *m;            // [S] number of held half-planes
  // the held rows of every agent-stage (i, t), t = 1..T, index a = (t-1) N + i:
  // entries coff[a] .. coff[a+1]-1 of cent, each (2 k + (i > j), q) for held
  // row k = (min(i,j), max(i,j), t) at pair-step q, partners j increasing
  int *coff;         // [sum N (T+1)] per scenario from its first agent-stage (N T + 1 used)
  int2 *cent;        // [2 sum P T] per scenario from 2 (its first pair-step)
};

enum { EQ_POLISH = 0, EQ_ADJOINT = 1 };
enum { EQK_INHOM = 0, EQK_HOM = 1, EQK_ADJ = 2 };
enum { ES_M = 0, ES_ITERS, ES_RES, ES_VIOL, ES_NCOL };

struct EqpIO {
  const float *gx, *gu;          // adjoint: upstream dL/dx, dL/du (caller layouts; gu may be null)
  float *x, *u;                  // polish: outputs (caller layouts)
  float *dx0, *dxref, *dlogq, *dlogr;   // adjoint outputs (any may be null)
  float *stats;                  // [S][ES_NCOL] or null
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Workgroup-wide sum (max) in a fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum_d(v);
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double block_max(double v, double *red) {
  v = wave_max_d(v);
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s = fmax(s, red[w]);
  return s;
}

__device__ __forceinline__ int pair_of(int f, int s, int N) { return f * N - f * (f + 1) / 2 + (s - f - 1); }

// Riccati factors of agent i for its working set, without the consensus
// penalty: H_x = 2 Q_t, H_T = 2 qT Q, H_u = 2 R (Eq. 7 with fixed inputs).
template <int NX, int NU, bool DI, class R>
__device__ void eqp_factor(const Prob &pb, const WS &ws, const Scen &sc, R *Er, int i) {
  using EF = EFld<NX, NU>;
  const int N = sc.N, T = sc.T;
  const float *qd = ws.qd + (long long)sc.s * NX;
  const float *rd = ws.rd + (long long)sc.s * NU;
  const int8_t *Wb = ws.wr + sc.bo;
  R hu[NU];
#pragma unroll
  for (int a = 0; a < NU; ++a) hu[a] = R(2) * (R)rd[a];
  R Pn[NX][NX];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) Pn[r][c] = (r == c) ? R(2) * (R)pb.qT * (R)qd[r] : R(0);
  for (int t = T - 1; t >= 0; --t) {
    R hx[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) hx[r] = R(2) * (R)qd[r];
    int8_t wt[NU];
#pragma unroll
    for (int a = 0; a < NU; ++a) wt[a] = Wb[(unsigned)(t * N + i) * 4u + a];
    R Pt[NX][NX], K[NU][NX], Sv[NU][NU], kc[NU], cc[NX];
    factor_stage<NX, NU, DI, R>(pb, hx, hu, Pn, wt, pb.ulo, pb.uhi, t >= 1, Pt, K, Sv, kc, cc);
    R *f = Er + (size_t)(t * N + i) * EF::NF;
#pragma unroll
    for (int a = 0; a < NU; ++a) {
#pragma unroll
      for (int c = 0; c < NX; ++c) f[EF::K + a * NX + c] = K[a][c];
#pragma unroll
      for (int b = a; b < NU; ++b) f[EF::SV + sym_idx<NU>(a, b)] = Sv[a][b];
      f[EF::KC + a] = kc[a];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) f[EF::CC + r] = cc[r];
    if (t >= 1) {
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int c = 0; c < NX; ++c) Pn[r][c] = Pt[r][c];
    }
  }
}

// One agent's EQP solve for the coupling term stored in the E field.
//   kind EQK_INHOM: x_0 = x0, fixed inputs at their bounds, tracking terms
//                   -2 Q_t r_t (the polish);
//   kind EQK_HOM:   x_0 = 0, fixed inputs 0, no other term (a product with S);
//   kind EQK_ADJ:   x_0 = 0, fixed inputs 0, linear terms -dL/dx_t, -dL/du_t.
// Backward sweep p_T = q_T; s = B'p_{t+1} + r_t; k_t = kc_t - Sv_t s;
// p_t = q_t + c_t + A'p_{t+1} + K_t' s (kc, c only for EQK_INHOM); then the
// rollout u_t = K_t x_t + k_t.  With `final` the solution is stored (polish)
// or turned into the parameter gradients (adjoint): with xbar, ubar the
// adjoint solution and p_0 its value gradient at stage 0,
//   dL/dx0      = dL/dx_0 - p_0,
//   dL/dxref_t  = 2 w_t q * xbar_t                       (t >= 1; 0 at t = 0),
//   dL/dlog q_k = -sum_t 2 w_t q_k xbar_t,k (x_t,k - r_t,k),
//   dL/dlog r_a = -sum_t 2 r_a ubar_t,a u_t,a,
// i.e. -wbar' dF/dtheta for the KKT map F = H w + c + E'y of the EQP.
template <int NX, int NU, bool DI, class R>
__device__ void eqp_agent(const Prob &pb, const WS &ws, const Scen &sc, R *Er, int i, int kind, bool final,
                          const EqpIO &io, double gq[NX], double gr[NU]) {
  using EF = EFld<NX, NU>;
  using D = Dyn<NX, NU, DI>;
  const int N = sc.N, T = sc.T;
  const float *qd = ws.qd + (long long)sc.s * NX;
  const float *rd = ws.rd + (long long)sc.s * NU;
  const long long xrow = sc.xo + (long long)i * (T + 1);   // caller row of (agent, t = 0)
  const long long urow = sc.uo + (long long)i * T;
  auto F = [&](int t) -> R * { return Er + (size_t)(t * N + i) * EF::NF; };
  auto qlin = [&](int t, R q[NX]) {
    const R *f = F(t);
    const R w = (t == T) ? (R)pb.qT : R(1);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      R v = R(0);
      if (kind == EQK_INHOM) v = R(-2) * w * (R)qd[c] * (R)ws.xref[(xrow + t) * NX + c];
      else if (kind == EQK_ADJ) v = -(R)io.gx[(xrow + t) * NX + c];
      if (c < NU) v += f[EF::E + c];
      q[c] = v;
    }
  };
  // stages per batch of the sweeps: every load of a batch is issued before
  // its first stage is computed (two stages for the 3-D FP64 blocks, whose
  // data fill many registers, four otherwise)
  constexpr int KB = (sizeof(R) == 8 && NX == 6) ? 2 : 4;
  constexpr int NS = EF::NS;
  struct BStage {
    R kc[NU], sv[NS], K[NU][NX], cc[NX], q[NX], gu[NU];
  };
  auto bload = [&](BStage &st, int t) {
    const R *f = F(t);
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      st.kc[a] = (kind == EQK_INHOM) ? f[EF::KC + a] : R(0);
      st.gu[a] = (kind == EQK_ADJ && io.gu) ? (R)io.gu[(urow + t) * NU + a] : R(0);
#pragma unroll
      for (int c = 0; c < NX; ++c) st.K[a][c] = f[EF::K + a * NX + c];
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) st.sv[k] = f[EF::SV + k];
#pragma unroll
    for (int c = 0; c < NX; ++c) st.cc[c] = (kind == EQK_INHOM) ? f[EF::CC + c] : R(0);
    if (t >= 1) qlin(t, st.q);
  };
  R p[NX];
  qlin(T, p);
  for (int t0 = T - 1; t0 >= 0; t0 -= KB) {
    BStage st[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b)
      if (t0 - b >= 0) bload(st[b], t0 - b);
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int t = t0 - b;
      if (t < 0) break;
      const BStage &cur = st[b];
      R s[NU];
      D::btx(pb, p, s);
      if (kind == EQK_ADJ && io.gu) {
#pragma unroll
        for (int a = 0; a < NU; ++a) s[a] -= cur.gu[a];
      }
      R pn[NX];
      D::atx(pb, p, pn);
#pragma unroll
      for (int a = 0; a < NU; ++a) {
        R k = cur.kc[a];
#pragma unroll
        for (int c2 = 0; c2 < NU; ++c2) k = fma(-cur.sv[a <= c2 ? sym_idx<NU>(a, c2) : sym_idx<NU>(c2, a)], s[c2], k);
        F(t)[EF::KV + a] = k;
#pragma unroll
        for (int c = 0; c < NX; ++c) pn[c] = fma(cur.K[a][c], s[a], pn[c]);
      }
      if (kind == EQK_INHOM) {
#pragma unroll
        for (int c = 0; c < NX; ++c) pn[c] += cur.cc[c];
      }
      if (t >= 1) {
#pragma unroll
        for (int c = 0; c < NX; ++c) pn[c] += cur.q[c];
      }
#pragma unroll
      for (int c = 0; c < NX; ++c) p[c] = pn[c];
    }
  }
  R x[NX];
#pragma unroll
  for (int c = 0; c < NX; ++c) x[c] = (kind == EQK_INHOM) ? (R)ws.x0[(sc.ao + i) * NX + c] : R(0);
  if (final && kind == EQK_INHOM) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      F(0)[EF::XS + c] = x[c];
      io.x[(xrow + 0) * NX + c] = (float)x[c];
    }
  }
  if (final && kind == EQK_ADJ) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      if (io.dx0) io.dx0[(sc.ao + i) * NX + c] = (float)((double)io.gx[(xrow + 0) * NX + c] - (double)p[c]);
      if (io.dxref) io.dxref[(xrow + 0) * NX + c] = 0.f;
    }
  }
  for (int t0 = 0; t0 < T; t0 += KB) {
   R kvb[KB][NU], Kb[KB][NU][NX];
#pragma unroll
   for (int b = 0; b < KB; ++b)
    if (t0 + b < T) {
      const R *f = F(t0 + b);
#pragma unroll
      for (int a = 0; a < NU; ++a) {
        kvb[b][a] = f[EF::KV + a];
#pragma unroll
        for (int c = 0; c < NX; ++c) Kb[b][a][c] = f[EF::K + a * NX + c];
      }
    }
#pragma unroll
   for (int b = 0; b < KB; ++b) {
    const int t = t0 + b;
    if (t >= T) break;
    R u[NU];
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      R v = kvb[b][a];
#pragma unroll
      for (int c = 0; c < NX; ++c) v = fma(Kb[b][a][c], x[c], v);
      u[a] = v;
    }
    R xn[NX];
    D::ax(pb, x, xn);
    D::add_bu(pb, u, xn);
    R *fn = F(t + 1);
#pragma unroll
    for (int c = 0; c < NU; ++c) fn[EF::XT + c] = xn[c];
    if (final && kind == EQK_INHOM) {
#pragma unroll
      for (int a = 0; a < NU; ++a) {
        F(t)[EF::US + a] = u[a];
        io.u[(urow + t) * NU + a] = (float)u[a];
      }
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        fn[EF::XS + c] = xn[c];
        io.x[(xrow + t + 1) * NX + c] = (float)xn[c];
      }
    }
    if (final && kind == EQK_ADJ) {
      const R *fs = F(t);
#pragma unroll
      for (int a = 0; a < NU; ++a) gr[a] -= 2.0 * (double)rd[a] * (double)u[a] * (double)fs[EF::US + a];
      const double w = (t + 1 == T) ? (double)pb.qT : 1.0;
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        const double wq = 2.0 * w * (double)qd[c];
        const double dev = (double)fn[EF::XS + c] - (double)ws.xref[(xrow + t + 1) * NX + c];
        gq[c] -= wq * (double)xn[c] * dev;
        if (io.dxref) io.dxref[(xrow + t + 1) * NX + c] = (float)(wq * (double)xn[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < NX; ++c) x[c] = xn[c];
   }
  }
}

// eqp_agent for one coordinate axis c of agent i, with double-integrator
// dynamics: the fixed-input LQR of the agent is then block diagonal over the
// axes (diagonal Q and R, a box and a coupling term per coordinate), and so
// are its factors (the cross-axis entries of K and S'^-1 are exact zeros), so
// the axis problem in (position c, velocity NU + c; input c) reads its own
// entries of the agent's records and performs, in the same order, the
// nonzero operations of eqp_agent: the results are those of the joint sweep.
// One lane per (agent, axis); 2 x 2 blocks, stages loaded four at a time.
template <int NX, int NU, class R>
__device__ void eqp_agent_axis(const Prob &pb, const WS &ws, const Scen &sc, R *Er, int i, int c, int kind,
                               bool final, const EqpIO &io, double gq[NX], double gr[NU]) {
  using EF = EFld<NX, NU>;
  constexpr int KB = 4;
  const int N = sc.N, T = sc.T, cv = NU + c;
  const float *qd = ws.qd + (long long)sc.s * NX;
  const float *rd = ws.rd + (long long)sc.s * NU;
  const long long xrow = sc.xo + (long long)i * (T + 1);
  const long long urow = sc.uo + (long long)i * T;
  const R dt = (R)pb.dt, h = (R)pb.h;
  const int svc = sym_idx<NU>(c, c);
  auto F = [&](int t) -> R * { return Er + (size_t)(t * N + i) * EF::NF; };
  // linear term of the stage on (position, velocity) of this axis
  auto qlin = [&](int t, R q[2]) {
    const R w = (t == T) ? (R)pb.qT : R(1);
    R v0 = R(0), v1 = R(0);
    if (kind == EQK_INHOM) {
      v0 = R(-2) * w * (R)qd[c] * (R)ws.xref[(xrow + t) * NX + c];
      v1 = R(-2) * w * (R)qd[cv] * (R)ws.xref[(xrow + t) * NX + cv];
    } else if (kind == EQK_ADJ) {
      v0 = -(R)io.gx[(xrow + t) * NX + c];
      v1 = -(R)io.gx[(xrow + t) * NX + cv];
    }
    q[0] = v0 + F(t)[EF::E + c];
    q[1] = v1;
  };
  struct BStage {
    R kc, sv, k0, k1, c0, c1, q[2], gu;
  };
  R p[2];
  qlin(T, p);
  for (int t0 = T - 1; t0 >= 0; t0 -= KB) {
    BStage st[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int t = t0 - b;
      if (t < 0) break;
      const R *f = F(t);
      st[b].kc = (kind == EQK_INHOM) ? f[EF::KC + c] : R(0);
      st[b].sv = f[EF::SV + svc];
      st[b].k0 = f[EF::K + c * NX + c];
      st[b].k1 = f[EF::K + c * NX + cv];
      st[b].c0 = (kind == EQK_INHOM) ? f[EF::CC + c] : R(0);
      st[b].c1 = (kind == EQK_INHOM) ? f[EF::CC + cv] : R(0);
      st[b].gu = (kind == EQK_ADJ && io.gu) ? (R)io.gu[(urow + t) * NU + c] : R(0);
      if (t >= 1) qlin(t, st[b].q);
    }
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int t = t0 - b;
      if (t < 0) break;
      const BStage &cur = st[b];
      R sa = fma(dt, p[1], h * p[0]);                 // B'p
      if (kind == EQK_ADJ && io.gu) sa -= cur.gu;
      R pn0 = p[0], pn1 = fma(dt, p[0], p[1]);        // A'p
      const R k = fma(-cur.sv, sa, cur.kc);
      F(t)[EF::KV + c] = k;
      pn0 = fma(cur.k0, sa, pn0);
      pn1 = fma(cur.k1, sa, pn1);
      if (kind == EQK_INHOM) {
        pn0 += cur.c0;
        pn1 += cur.c1;
      }
      if (t >= 1) {
        pn0 += cur.q[0];
        pn1 += cur.q[1];
      }
      p[0] = pn0;
      p[1] = pn1;
    }
  }
  R x0 = (kind == EQK_INHOM) ? (R)ws.x0[(sc.ao + i) * NX + c] : R(0);
  R x1 = (kind == EQK_INHOM) ? (R)ws.x0[(sc.ao + i) * NX + cv] : R(0);
  if (final && kind == EQK_INHOM) {
    F(0)[EF::XS + c] = x0;
    F(0)[EF::XS + cv] = x1;
    io.x[xrow * NX + c] = (float)x0;
    io.x[xrow * NX + cv] = (float)x1;
  }
  if (final && kind == EQK_ADJ) {
    if (io.dx0) {
      io.dx0[(sc.ao + i) * NX + c] = (float)((double)io.gx[xrow * NX + c] - (double)p[0]);
      io.dx0[(sc.ao + i) * NX + cv] = (float)((double)io.gx[xrow * NX + cv] - (double)p[1]);
    }
    if (io.dxref) {
      io.dxref[xrow * NX + c] = 0.f;
      io.dxref[xrow * NX + cv] = 0.f;
    }
  }
  for (int t0 = 0; t0 < T; t0 += KB) {
    R kv[KB], k0[KB], k1[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b)
      if (t0 + b < T) {
        const R *f = F(t0 + b);
        kv[b] = f[EF::KV + c];
        k0[b] = f[EF::K + c * NX + c];
        k1[b] = f[EF::K + c * NX + cv];
      }
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int t = t0 + b;
      if (t >= T) break;
      const R u = fma(k1[b], x1, fma(k0[b], x0, kv[b]));
      const R xn0 = fma(h, u, fma(dt, x1, x0));
      const R xn1 = fma(dt, u, x1);
      R *fn = F(t + 1);
      fn[EF::XT + c] = xn0;
      if (final && kind == EQK_INHOM) {
        F(t)[EF::US + c] = u;
        io.u[(urow + t) * NU + c] = (float)u;
        fn[EF::XS + c] = xn0;
        fn[EF::XS + cv] = xn1;
        io.x[(xrow + t + 1) * NX + c] = (float)xn0;
        io.x[(xrow + t + 1) * NX + cv] = (float)xn1;
      }
      if (final && kind == EQK_ADJ) {
        gr[c] -= 2.0 * (double)rd[c] * (double)u * (double)F(t)[EF::US + c];
        const double w = (t + 1 == T) ? (double)pb.qT : 1.0;
        const double wq0 = 2.0 * w * (double)qd[c], wq1 = 2.0 * w * (double)qd[cv];
        const double dev0 = (double)fn[EF::XS + c] - (double)ws.xref[(xrow + t + 1) * NX + c];
        const double dev1 = (double)fn[EF::XS + cv] - (double)ws.xref[(xrow + t + 1) * NX + cv];
        gq[c] -= wq0 * (double)xn0 * dev0;
        gq[cv] -= wq1 * (double)xn1 * dev1;
        if (io.dxref) {
          io.dxref[(xrow + t + 1) * NX + c] = (float)(wq0 * (double)xn0);
          io.dxref[(xrow + t + 1) * NX + cv] = (float)(wq1 * (double)xn1);
        }
      }
      x0 = xn0;
      x1 = xn1;
    }
  }
}

// The agents' EQP solves of a scenario: one lane per (agent, axis) with
// double-integrator dynamics, one lane per agent otherwise.
template <int NX, int NU, bool DI, class R>
__device__ __forceinline__ void eqp_agents(const Prob &pb, const WS &ws, const Scen &sc, R *Er, int kind, bool final,
                                           const EqpIO &io, double gq[NX], double gr[NU], int tid, int nth) {
  if constexpr (DI) {
    for (int l = tid; l < sc.N * NU; l += nth)
      eqp_agent_axis<NX, NU, R>(pb, ws, sc, Er, l / NU, l % NU, kind, final, io, gq, gr);
  } else {
    for (int i = tid; i < sc.N; i += nth) eqp_agent<NX, NU, DI, R>(pb, ws, sc, Er, i, kind, final, io, gq, gr);
  }
}

// E_i,t = -sum_j sigma_ij v_k n_k over the held half-planes k = (i, j, t)
// (sigma = +1 when i is the pair's first agent): the linear term -D'v.  The
// list of an agent-stage is read four entries at a time.
template <int NX, int NU, class R>
__device__ void eqp_scatter(const Scen &sc, R *Er, const float *nrm, const int *off, const int2 *ent,
                            const double *v, double scale, int tid, int nth) {
  using EF = EFld<NX, NU>;
  const int N = sc.N, T = sc.T;
  for (int idx = tid; idx < N * T; idx += nth) {
    const int t = idx / N + 1, i = idx % N;
    double e[NU];
#pragma unroll
    for (int c = 0; c < NU; ++c) e[c] = 0.0;
    const int b0 = off[idx], b1 = off[idx + 1];
    for (int b = b0; b < b1; b += 4) {
      int2 en[4];
      double vv[4];
      float nn[4][NU];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (b + q < b1) en[q] = ent[b + q];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (b + q < b1) {
          vv[q] = v[en[q].x >> 1];
#pragma unroll
          for (int c = 0; c < NU; ++c) nn[q][c] = nrm[(long long)en[q].y * NU + c];
        }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (b + q < b1) {
          const double sv = (en[q].x & 1) ? -scale * vv[q] : scale * vv[q];
#pragma unroll
          for (int c = 0; c < NU; ++c) e[c] -= sv * (double)nn[q][c];
        }
    }
    R *f = Er + (size_t)(t * N + i) * EF::NF;
#pragma unroll
    for (int c = 0; c < NU; ++c) f[EF::E + c] = (R)e[c];
  }
}

// (D xt)_k for the held half-planes k0 .. k0+3 (those below m), their list
// entries and positions read before any is used.
template <int NX, int NU, class R>
__device__ __forceinline__ void eqp_rows4(const Scen &sc, const R *Er, const float *nrm, const int2 *cl, int k0,
                                          int m, double g[4]) {
  using EF = EFld<NX, NU>;
  const int N = sc.N, T = sc.T;
  int2 en[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (k0 + q < m) en[q] = cl[k0 + q];
  R xi[4][NU], xj[4][NU];
  float nn[4][NU];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (k0 + q < m) {
      const int qq = en[q].x, i = en[q].y / N, j = en[q].y % N, t = qq % T + 1;
      const R *fi = Er + (size_t)(t * N + i) * EF::NF;
      const R *fj = Er + (size_t)(t * N + j) * EF::NF;
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        xi[q][c] = fi[EF::XT + c];
        xj[q][c] = fj[EF::XT + c];
        nn[q][c] = nrm[(long long)qq * NU + c];
      }
    }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double v = 0.0;
    if (k0 + q < m) {
#pragma unroll
      for (int c = 0; c < NU; ++c) v = fma((double)nn[q][c], (double)xi[q][c] - (double)xj[q][c], v);
    }
    g[q] = v;
  }
}


// Freeze the normals of the last consensus step and compact the held
// half-planes (contiguous chunks per thread, exclusive scan: a fixed order);
// the polish starts from nu = gamma of the last consensus step.
template <int NX, int NU>
__device__ void eqp_freeze(const Prob &pb, const WS &ws, const EWS &ew, const Scen &sc, int *scan, int tid, int nth) {
  using F = Fld<NX, NU>;
  const int N = sc.N, T = sc.T, P = N * (N - 1) / 2, TP = P * T;
  const float *R = ws.fr + sc.fo;
  float *nrm = ew.nrm + sc.po * NU;
  int *cidx = ew.cidx + sc.po;
  int2 *cl = ew.clist + sc.po;
  double *nu = ew.cg + 6 * sc.po;
  const float *gm = ws.gam + sc.lo;
  const int per = (TP + nth - 1) / nth;
  const int q0 = min(TP, tid * per), q1 = min(TP, q0 + per);
  int cnt = 0;
  for (int pass = 0; pass < 2; ++pass) {
    int k = (pass == 1) ? scan[tid] : 0;
    int i = 0, j = 1, pcur = -1;
    for (int q = q0; q < q1; ++q) {
      const int p = q / T, t = q % T + 1;
      if (p != pcur) {   // decode the pair (i, j) of index p
        int r = p;
        i = 0;
        while (r >= N - 1 - i) { r -= N - 1 - i; ++i; }
        j = i + 1 + r;
        pcur = p;
      }
      const int e = (t - 1) * N * N + j * N + i;   // ordered copy (i, j), i first
      const bool act = gm[e] > 0.f;   // violated at the last consensus step
      if (pass == 0) {
        float n[NU];
        if (pb.normal_mode == NORMAL_FROZEN) {
          if (ws.normals) {
            const float *nv = ws.normals + (sc.po + (long long)q) * NU;
#pragma unroll
            for (int c = 0; c < NU; ++c) n[c] = nv[c];
          } else {
            reference_normal<NX, NU>(ws, sc, i, j, t, n);
          }
        } else {   // the normal of the last consensus step, from the final positions
          float d[NU];
#pragma unroll
          for (int c = 0; c < NU; ++c)
            d[c] = R[fidx((unsigned)sc.GS, (unsigned)(t * N + i), F::X + c)] -
                   R[fidx((unsigned)sc.GS, (unsigned)(t * N + j), F::X + c)];
          if (!unit_normal<NU>(d, n)) reference_normal<NX, NU>(ws, sc, i, j, t, n);
        }
#pragma unroll
        for (int c = 0; c < NU; ++c) nrm[(long long)q * NU + c] = n[c];
        cnt += act;
      } else {
        if (act) {
          cidx[q] = k;
          cl[k] = make_int2(q, i * N + j);
          nu[k] = (double)gm[e];   // lambda_ij = -gamma n: the half-plane's multiplier
          ++k;
        } else {
          cidx[q] = -1;
        }
      }
    }
    if (pass == 0) {
      __syncthreads();
      scan[tid] = cnt;
      __syncthreads();
      if (tid == 0) {
        int acc = 0;
        for (int w = 0; w < nth; ++w) { const int c = scan[w]; scan[w] = acc; acc += c; }
        ew.m[sc.s] = acc;
        scan[nth] = acc;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // The held rows of every agent-stage, partners in increasing order:
  // contiguous chunks of agent-stages per thread, counted, scanned, filled.
  const int m = scan[nth];
  const int NT = N * T;
  int *off = ew.coff + sc.xo;
  int2 *ent = ew.cent + 2 * sc.po;
  const int per2 = (NT + nth - 1) / nth;
  const int a0 = min(NT, tid * per2), a1 = min(NT, a0 + per2);
  auto held = [&](int a, int j) -> int {   // compact index of (i, j, t) for agent-stage a, or -1
    const int t = a / N + 1, i = a % N;
    const int f = i < j ? i : j, s2 = i < j ? j : i;
    return cidx[pair_of(f, s2, N) * T + (t - 1)];
  };
  int cnt2 = 0;
  for (int a = a0; a < a1; ++a)
    for (int j = 0; j < N; ++j)
      if (j != a % N && held(a, j) >= 0) ++cnt2;
  __syncthreads();
  scan[tid] = cnt2;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int w = 0; w < nth; ++w) { const int c = scan[w]; scan[w] = acc; acc += c; }
    off[NT] = acc;
  }
  __syncthreads();
  int o = scan[tid];
  for (int a = a0; a < a1; ++a) {
    off[a] = o;
    const int t = a / N + 1, i = a % N;
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      const int k = held(a, j);
      if (k < 0) continue;
      const int f = i < j ? i : j, s2 = i < j ? j : i;
      ent[o++] = make_int2(2 * k + (i > j ? 1 : 0), pair_of(f, s2, N) * T + (t - 1));
    }
  }
  __syncthreads();
  if (tid == 0) scan[nth] = m;
  __syncthreads();
}

template <int NX, int NU, bool DI, class R>
__device__ void eqp_scenario(const Prob &pb, const WS &ws, const EWS &ew, const EqpIO &io, int s, int mode, int max_cg,
                             double tol, double *red, int *scan) {
  using EF = EFld<NX, NU>;
  const int tid = threadIdx.x, nth = blockDim.x;
  const Scen sc = load_scen(ws, s);
  const int N = sc.N, T = sc.T, TP = N * (N - 1) / 2 * T;
  R *Er = (R *)ew.er + (size_t)sc.xo * EF::NF;
  const float *nrm = ew.nrm + sc.po * NU;
  const int2 *cl = ew.clist + sc.po;
  const int *coff = ew.coff + sc.xo;
  const int2 *cent = ew.cent + 2 * sc.po;
  double *nu = ew.cg + 6 * sc.po, *sd = nu + TP;
  if (mode == EQ_POLISH) {
    eqp_freeze<NX, NU>(pb, ws, ew, sc, scan, tid, nth);
    for (int i = tid; i < N; i += nth) eqp_factor<NX, NU, DI, R>(pb, ws, sc, Er, i);
  }
  __syncthreads();
  const int m = (mode == EQ_POLISH) ? scan[nth] : ew.m[s];
  if (mode == EQ_ADJOINT)
    for (int k = tid; k < m; k += nth) nu[k] = 0.0;
  __syncthreads();
  const int kind = (mode == EQ_POLISH) ? EQK_INHOM : EQK_ADJ;
  const double dval = (mode == EQ_POLISH) ? (double)pb.dmin : 0.0;
  double gq[NX], gr[NU];
  // residual of the held rows at the starting multipliers
  eqp_scatter<NX, NU, R>(sc, Er, nrm, coff, cent, nu, 1.0, tid, nth);
  __syncthreads();
  eqp_agents<NX, NU, DI, R>(pb, ws, sc, Er, kind, false, io, gq, gr, tid, nth);
  __syncthreads();
  // MINRES (Paige and Saunders 1975) on S nu = d - D w(0): Lanczos vectors
  // r1, r2 (r2 = beta v), the product y = S v, and the directions w_{k-2},
  // w_{k-1}; the residual norm phibar never increases, and on a singular,
  // inconsistent system (held rows that cannot all hold with the fixed
  // inputs) the iterate tends to a least-squares solution.
  double *b0 = sd, *b1 = b0 + TP, *b2 = b1 + TP, *wa = b2 + TP, *wb = wa + TP;
  double *r1 = b0, *r2 = b1, *y = b2;
  double acc = 0.0;
  for (int k0 = 4 * tid; k0 < m; k0 += 4 * nth) {
    double g[4];
    eqp_rows4<NX, NU, R>(sc, Er, nrm, cl, k0, m, g);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k0 + q < m) {
        const double r = dval - g[q];
        r2[k0 + q] = r;
        r1[k0 + q] = 0.0;
        wa[k0 + q] = 0.0;
        wb[k0 + q] = 0.0;
        acc = fma(r, r, acc);
      }
  }
  const double beta1 = sqrt(block_sum(acc, red));
  const double ref = (mode == EQ_POLISH) ? fmax((double)pb.dmin * sqrt((double)m), beta1) : beta1;
  const int cap = min(max_cg, 2 * m + 20);
  const double ls_tol = fmax(sqrt(tol), 1e-4);
  double beta = beta1, oldb = 0.0, dbar = 0.0, epsln = 0.0, phibar = beta1, cs = -1.0, sn = 0.0, gmax = 0.0;
  double anorm2 = 0.0;   // Frobenius norm of the Lanczos tridiagonal so far, an estimate of ||S||^2
  int it = 0;
  while (m > 0 && it < cap && phibar > tol * ref && beta > 1e-30 * beta1) {
    eqp_scatter<NX, NU, R>(sc, Er, nrm, coff, cent, r2, 1.0 / beta, tid, nth);   // v = r2 / beta
    __syncthreads();
    eqp_agents<NX, NU, DI, R>(pb, ws, sc, Er, EQK_HOM, false, io, gq, gr, tid, nth);
    __syncthreads();
    acc = 0.0;
    for (int k0 = 4 * tid; k0 < m; k0 += 4 * nth) {
      double g[4];
      eqp_rows4<NX, NU, R>(sc, Er, nrm, cl, k0, m, g);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (k0 + q < m) {
          const int k = k0 + q;
          double v = g[q];
          if (it >= 1) v = fma(-beta / oldb, r1[k], v);
          y[k] = v;
          acc = fma(r2[k] / beta, v, acc);
        }
    }
    const double alfa = block_sum(acc, red);
    acc = 0.0;
    for (int k0 = 4 * tid; k0 < m; k0 += 4 * nth) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (k0 + q < m) {
          const int k = k0 + q;
          const double v = fma(-alfa / beta, r2[k], y[k]);
          y[k] = v;
          acc = fma(v, v, acc);
        }
    }
    { double *t = r1; r1 = r2; r2 = y; y = t; }   // r1 <- r2, r2 <- y
    oldb = beta;
    beta = sqrt(block_sum(acc, red));
    const double oldeps = epsln;
    const double delta = cs * dbar + sn * alfa;
    const double gbar = sn * dbar - cs * alfa;
    epsln = sn * beta;
    dbar = -cs * beta;
    // ||S r|| of the current iterate is phibar sqrt(gbar^2 + dbar^2) (the
    // MINRES estimate); once it is below sqrt(tol) ||S|| ||r||, the iterate
    // is a least-squares solution of an inconsistent system (held rows that
    // cannot all hold): further steps cannot lower ||r||, and on a singular
    // S their rounding only drifts the multipliers along its null space
    anorm2 += alfa * alfa + oldb * oldb + beta * beta;
    if (phibar * sqrt(gbar * gbar + dbar * dbar) <= ls_tol * sqrt(anorm2) * phibar) break;
    const double gamma = sqrt(gbar * gbar + beta * beta);
    gmax = fmax(gmax, gamma);
    if (!(gamma > 1e-13 * gmax)) break;   // the Krylov space is exhausted on a singular system
    cs = gbar / gamma;
    sn = beta / gamma;
    const double phi = cs * phibar;
    phibar = sn * phibar;
    for (int k0 = 4 * tid; k0 < m; k0 += 4 * nth) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (k0 + q < m) {
          const int k = k0 + q;
          const double w = (r1[k] / oldb - oldeps * wa[k] - delta * wb[k]) / gamma;   // w_k into the w_{k-2} slot
          wa[k] = w;
          nu[k] = fma(phi, w, nu[k]);
        }
    }
    { double *t = wa; wa = wb; wb = t; }
    ++it;
    __syncthreads();
  }
  // final solve with the converged multipliers
  eqp_scatter<NX, NU, R>(sc, Er, nrm, coff, cent, nu, 1.0, tid, nth);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NX; ++c) gq[c] = 0.0;
#pragma unroll
  for (int a = 0; a < NU; ++a) gr[a] = 0.0;
  eqp_agents<NX, NU, DI, R>(pb, ws, sc, Er, kind, true, io, gq, gr, tid, nth);
  __syncthreads();
  double viol = 0.0;
  for (int k0 = 4 * tid; k0 < m; k0 += 4 * nth) {
    double g[4];
    eqp_rows4<NX, NU, R>(sc, Er, nrm, cl, k0, m, g);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k0 + q < m) viol = fmax(viol, fabs(dval - g[q]));
  }
  viol = block_max(viol, red);
  if (mode == EQ_ADJOINT) {
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      const double g = block_sum(gq[c], red);
      if (tid == 0 && io.dlogq) io.dlogq[(long long)s * NX + c] = (float)g;
    }
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      const double g = block_sum(gr[a], red);
      if (tid == 0 && io.dlogr) io.dlogr[(long long)s * NU + a] = (float)g;
    }
  }
  if (tid == 0 && io.stats) {
    float *st = io.stats + (long long)s * ES_NCOL;
    st[ES_M] = (float)m;
    st[ES_ITERS] = (float)it;
    st[ES_RES] = (float)(ref > 0.0 ? phibar / ref : 0.0);
    st[ES_VIOL] = (float)viol;
  }
  __syncthreads();
}

// BT threads per workgroup: 256, or 512 where a scenario has more axis
// problems than 256 (every sweep of a MINRES iteration then runs all of them
// at once)
template <int NX, int NU, bool DI, class R, int BT = 256>
__global__ __launch_bounds__(BT) void k_eqp(Prob pb, WS ws, EWS ew, EqpIO io, int S, int mode, int max_cg,
                                            double tol) {
  __shared__ double red[BT / 64];
  __shared__ int scan[BT + 1];
  for (int s = blockIdx.x; s < S; s += gridDim.x)
    eqp_scenario<NX, NU, DI, R>(pb, ws, ew, io, s, mode, max_cg, tol, red, scan);
}

}  // namespace tadmm
