// turboadmm.hip -- HIP kernels and C-ABI host library of the ADMM hot path.
//
// Method (see include/turboadmm.h): per ADMM iteration, one input-bounded
// linear-quadratic local QP per agent (Sec. IV-A, Eq. 3) solved by a Riccati
// factor (Eq. 7), an affine backward sweep, a forward rollout (Eq. 8) and
// costates (Eq. 9) inside a primal active-set loop; then the consensus
// projection (Eq. 4), the dual update (Eq. 5) and the residual test (Sec. V-A).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/turboadmm.h"
#include "tadmm_device.h"
#include "tadmm_eqp.h"

namespace tadmm {

// ===========================================================================
// Local QP (x-update)
// ===========================================================================
// The x-update routines are written against a view V of one local QP: its
// dimensions (V::NX states, V::NU inputs), its fields at (component, stage),
// its input bounds, stage weights and working set.  There are two views.
//
// AgentView: the QP of agent i, for any dynamics.  Its fields are those of the
//   agent-stage region: agent-stage g = t * N + i, field f at R[fidx(GS, g, f)]
//   (32-bit offsets; the group base (f / 4) * 4 GS is uniform).
//
// AxisView: coordinate axis c of agent i's QP.  With double-integrator
//   dynamics the stage costs (diagonal Q, R), the consensus penalty (on the
//   positions, coordinate by coordinate) and the input box all act per
//   coordinate, so the local QP separates exactly into dp problems in the
//   (position, velocity; acceleration) of one axis.  Each one has its own
//   working set, factors and active-set loop and is solved by one lane; the
//   minimiser is unique, so together they give the joint QP's solution.  An
//   axis problem's private fields (factors, affine terms, equality-QP
//   inputs) live in a region of 16-byte groups over the axis-stages
//   a = (t * N + i) * dp + c, so consecutive lanes read consecutive groups;
//   its iterate, linear term, working set and FP64 scratch are the agent's
//   fields of that axis.
//
// V::kBatch stages are loaded per batch in the sweeps: all their loads are
// issued before the first one is used, so a batch costs about one memory
// round trip instead of one per stage.
// Arrays of the axis-stage region, each [a][width] floats over the
// axis-stages a, so that a pass writes whole contiguous spans: the factor
// (K_0, K_1, S'^-1, kc), the value constant (c_0, c_1), the affine value
// term (p_0, p_1; written where the input is fixed), the affine terms (k,
// the equality-QP input) and the packed value Hessian (P_00, P_01, P_11, -).
enum { AXA_FAC = 0, AXA_C = 4, AXA_PV = 6, AXA_AFF = 8, AXA_P = 10, AXA_W = 14 };   // offsets in units of GA floats
// floats of a scenario's axis-stage region (GS agent-stages, dp axes)
__host__ __device__ constexpr long long axis_region_floats(long long GS, int dp) { return (long long)AXA_W * GS * dp; }
// The inputs u are a dense [GS][NU] array after the axis-stage region (a pass
// writes every input of a stage: whole contiguous spans).
__host__ __device__ constexpr long long input_region_floats(long long GS, int nu) { return GS * nu; }
template <int NX, int NU>
__device__ __forceinline__ float &uref(float *R, unsigned GS, unsigned g, int c) {
  return R[(size_t)Fld<NX, NU>::NF * GS + (size_t)axis_region_floats(GS, NU) + (size_t)g * NU + c];
}
// The previous positions C x^k are a dense [GS][NU] array after the inputs
// (the consensus step commits every agent-stage's positions: whole spans).
template <int NX, int NU>
__device__ __forceinline__ float &xpref(float *R, unsigned GS, unsigned g, int c) {
  return R[(size_t)Fld<NX, NU>::NF * GS + (size_t)axis_region_floats(GS, NU) + (size_t)input_region_floats(GS, NU) +
           (size_t)g * NU + c];
}

// An agent's dynamics for the dynamics products: its own matrices when the
// batch gives them, else the shared ones of the kernel arguments.
struct DynSel {
  const Prob &pb;
  const float *A, *B;
  __device__ __forceinline__ float a(int k) const { return A ? A[k] : pb.A[k]; }
  __device__ __forceinline__ float b(int k) const { return B ? B[k] : pb.B[k]; }
};

template <int NX_, int NU_, bool DI_>
struct AgentView {
  static constexpr int NX = NX_, NU = NU_, NS = NU_ * (NU_ + 1) / 2, NP = NX_ * (NX_ + 1) / 2;
  static constexpr bool DI = DI_;
  static constexpr int kBatch = 2, kSweepBatch = 2, kRefineBatch = 1;
  using F = Fld<NX, NU>;
  float *__restrict__ R;
  int8_t *__restrict__ Wb;
  double *__restrict__ D;
  int *dirty;                 // highest stage whose factor is stale (-1: none)
  const float *qd;            // diagonal of Q
  unsigned GS, N, i;
  float lo[NU], hi[NU], hu[NU];
  float rho, rho_prev;        // penalty of this iteration, of the last one
  const float *Ad, *Bd;       // this agent's own dynamics (NULL: the shared ones)
  __device__ __forceinline__ AgentView(const Prob &pb, const WS &ws, const Scen &sc, int i_)
      : R(ws.fr + sc.fo), Wb(ws.wr + sc.bo), D(ws.dr + sc.dof), dirty(ws.adirty + (sc.ao + i_) * NU_),
        qd(ws.aq ? ws.aq + (sc.ao + i_) * NX : ws.qd + (long long)sc.s * NX), GS((unsigned)sc.GS),
        N((unsigned)sc.N), i((unsigned)i_), rho(pb.adapt ? ws.rhos[2 * sc.s] : pb.rho),
        rho_prev(pb.adapt ? ws.rhos[2 * sc.s + 1] : pb.rho),
        Ad(ws.aA ? ws.aA + (sc.ao + i_) * (NX * NX) : nullptr),
        Bd(ws.aB ? ws.aB + (sc.ao + i_) * (NX * NU) : nullptr) {
    const float *rd = ws.ar ? ws.ar + (sc.ao + i_) * NU : ws.rd + (long long)sc.s * NU;
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      lo[a] = ws.alo ? ws.alo[(sc.ao + i_) * NU + a] : pb.ulo[a];
      hi[a] = ws.ahi ? ws.ahi[(sc.ao + i_) * NU + a] : pb.uhi[a];
      hu[a] = 2.0f * rd[a];
    }
  }
  __device__ __forceinline__ unsigned g(int t) const { return (unsigned)t * N + i; }
  __device__ __forceinline__ float &f(int field, int t) const { return fref(R, GS, g(t), field); }
  __device__ __forceinline__ float &K(int a, int c, int t) const { return f(F::K + a * NX + c, t); }
  __device__ __forceinline__ float &SV(int k, int t) const { return f(F::SV + k, t); }
  __device__ __forceinline__ float &KC(int a, int t) const { return f(F::KC + a, t); }
  __device__ __forceinline__ float &CC(int r, int t) const { return f(F::CC + r, t); }
  __device__ __forceinline__ float &PU(int k, int t) const { return f(F::PU + k, t); }
  __device__ __forceinline__ float &PV(int r, int t) const { return f(F::PV + r, t); }
  __device__ __forceinline__ float &KV(int a, int t) const { return f(F::KV + a, t); }
  __device__ __forceinline__ float &UE(int a, int t) const { return f(F::UE + a, t); }
  __device__ __forceinline__ float &Q(int r, int t) const { return f(r < NU ? F::QZ + r : F::Q + r, t); }
  __device__ __forceinline__ float &ZD(int c, int t) const { return f(F::QZ + NU + c, t); }
  __device__ __forceinline__ float &X(int r, int t) const { return f(F::X + r, t); }
  __device__ __forceinline__ float &U(int a, int t) const { return uref<NX, NU>(R, GS, g(t), a); }
  __device__ __forceinline__ int8_t &w(int a, int t) const { return Wb[g(t) * 4u + a]; }
  __device__ __forceinline__ double &d(int r, int t) const { return D[g(t) * (unsigned)NX + r]; }
  __device__ __forceinline__ void hx(const Prob &pb, int t, int T, int n_nbr, float h[NX]) const {
    stage_hx<NX, NU>(pb, qd, t, T, n_nbr, rho, h);
  }
  __device__ __forceinline__ DynSel dyn(const Prob &pb) const { return DynSel{pb, Ad, Bd}; }
};

// LA: the affine feedforward k_t and the equality-QP input of the axis
// problem live in LDS ([t][2][nl] over the scenario's nl axis problems, this
// one at column l) instead of the axis-stage region: both are written and
// read only within one x-update, so they need not reach HBM.
template <int NXF, int NUF, bool LA = false>
struct AxisView {
  static constexpr int NX = 2, NU = 1, NS = 1, NP = 3;
  static constexpr bool DI = true;
  static constexpr int kBatch = 4, kSweepBatch = 4;
  // the refinement's stages per batch: 4 in the plain-option kernel, whose
  // LDS slots leave the registers for it, one elsewhere (the option paths'
  // registers would spill in the x-update)
  static constexpr int kRefineBatch = LA ? 4 : 1;
  using F = Fld<NXF, NUF>;
  float *__restrict__ R;      // agent-stage region
  float *__restrict__ AX;     // axis-stage region
  int8_t *__restrict__ Wb;
  double *__restrict__ D;
  int *dirty;
  unsigned GS, N, i, c;
  float qd[2], lo[1], hi[1], hu[1];
  float rho, rho_prev;        // penalty of this iteration, of the last one
  float *la = nullptr;        // LA: the LDS slots, [t][2][nl]
  unsigned nl = 0, l = 0;
  __device__ __forceinline__ AxisView(const Prob &pb, const WS &ws, const Scen &sc, int i_, int c_)
      : R(ws.fr + sc.fo), AX(ws.fr + sc.fo + (long long)Fld<NXF, NUF>::NF * sc.GS), Wb(ws.wr + sc.bo),
        D(ws.dr + sc.dof), dirty(ws.adirty + (sc.ao + i_) * NUF + c_), GS((unsigned)sc.GS), N((unsigned)sc.N),
        i((unsigned)i_), c((unsigned)c_), rho(pb.adapt ? ws.rhos[2 * sc.s] : pb.rho),
        rho_prev(pb.adapt ? ws.rhos[2 * sc.s + 1] : pb.rho) {
    const float *q = ws.aq ? ws.aq + (sc.ao + i_) * NXF : ws.qd + (long long)sc.s * NXF;
    const float *rd = ws.ar ? ws.ar + (sc.ao + i_) * NUF : ws.rd + (long long)sc.s * NUF;
    qd[0] = q[c];
    qd[1] = q[NUF + c];
    hu[0] = 2.0f * rd[c];
    if (ws.alo) {   // this agent's own box
      lo[0] = ws.alo[(sc.ao + i_) * NUF + c_];
      hi[0] = ws.ahi[(sc.ao + i_) * NUF + c_];
    } else {        // the bounds of this axis, selected without indexing the argument arrays
      float l = pb.ulo[0], h = pb.uhi[0];
#pragma unroll
      for (int a = 1; a < NUF; ++a)
        if (c_ == a) { l = pb.ulo[a]; h = pb.uhi[a]; }
      lo[0] = l;
      hi[0] = h;
    }
  }
  __device__ __forceinline__ unsigned g(int t) const { return (unsigned)t * N + i; }
  __device__ __forceinline__ unsigned st(int r) const { return r ? NUF + c : c; }   // state index in the agent
  // element `slot` of array `arr` (offset arr * GA floats, `width` floats per axis-stage)
  template <int ARR, int WIDTH>
  __device__ __forceinline__ float &ax(int slot, int t) const {
    float *base = AX + (size_t)((unsigned)ARR * (GS * (unsigned)NUF));
    return base[(g(t) * (unsigned)NUF + c) * (unsigned)WIDTH + (unsigned)slot];
  }
  __device__ __forceinline__ float &K(int, int col, int t) const { return ax<AXA_FAC, 4>(col, t); }
  __device__ __forceinline__ float &SV(int, int t) const { return ax<AXA_FAC, 4>(2, t); }
  __device__ __forceinline__ float &KC(int, int t) const { return ax<AXA_FAC, 4>(3, t); }
  __device__ __forceinline__ float &CC(int r, int t) const { return ax<AXA_C, 2>(r, t); }
  __device__ __forceinline__ float &PV(int r, int t) const { return ax<AXA_PV, 2>(r, t); }
  __device__ __forceinline__ float &KV(int, int t) const {
    if constexpr (LA) return la[(unsigned)t * 2u * nl + l];
    else return ax<AXA_AFF, 2>(0, t);
  }
  __device__ __forceinline__ float &UE(int, int t) const {
    if constexpr (LA) return la[((unsigned)t * 2u + 1u) * nl + l];
    else return ax<AXA_AFF, 2>(1, t);
  }
  __device__ __forceinline__ float &PU(int k, int t) const { return ax<AXA_P, 4>(k, t); }
  __device__ __forceinline__ float &Q(int r, int t) const {
    return fref(R, GS, g(t), r ? F::Q + NUF + (int)c : F::QZ + (int)c);
  }
  __device__ __forceinline__ float &ZD(int, int t) const { return fref(R, GS, g(t), F::QZ + NUF + (int)c); }
  __device__ __forceinline__ float &X(int r, int t) const { return fref(R, GS, g(t), F::X + (int)st(r)); }
  __device__ __forceinline__ float &U(int, int t) const { return uref<NXF, NUF>(R, GS, g(t), (int)c); }
  __device__ __forceinline__ int8_t &w(int, int t) const { return Wb[g(t) * 4u + c]; }
  __device__ __forceinline__ double &d(int r, int t) const { return D[g(t) * (unsigned)NXF + st(r)]; }
  // stage_hx of the axis: 2 w q_pos + rho n_nbr on the position, 2 w q_vel
  __device__ __forceinline__ void hx(const Prob &pb, int t, int T, int n_nbr, float h[2]) const {
    const float w = (t == T) ? pb.qT : 1.0f;
    h[0] = 2.0f * w * qd[0] + rho * (float)n_nbr + (pb.pbox ? pb.sigma : 0.0f);
    h[1] = 2.0f * w * qd[1] + (pb.sbox ? pb.sigma : 0.0f);
  }
  __device__ __forceinline__ const Prob &dyn(const Prob &pb) const { return pb; }
};

template <class V>
__device__ __forceinline__ void load_sym(const V &m, int t, float P[V::NX][V::NX]) {
#pragma unroll
  for (int r = 0; r < V::NX; ++r)
#pragma unroll
    for (int c = r; c < V::NX; ++c) {
      const float v = m.PU(sym_idx<V::NX>(r, c), t);
      P[r][c] = v;
      P[c][r] = v;
    }
}

// Refactor stages thi..0 for the current working set (Eq. 7 with fixed
// inputs).  The working-set entries of a batch of stages are read at once;
// the recurrence itself is in registers.
template <class V>
__device__ void refactor(const Prob &pb, const V &m, int T, int n_nbr, int thi) {
  constexpr int NX = V::NX, NU = V::NU, B = V::kBatch;
  float Pn[NX][NX];
  load_sym(m, thi + 1, Pn);
  for (int t0 = thi; t0 >= 0; t0 -= B) {
    int8_t wb[B][NU];
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
      for (int a = 0; a < NU; ++a) wb[q][a] = (t0 - q >= 0) ? m.w(a, t0 - q) : (int8_t)0;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int t = t0 - q;
      if (t < 0) break;
      float hx[NX];
      m.hx(pb, t, T, n_nbr, hx);
      float Pt[NX][NX], K[NU][NX], Sv[NU][NU], kc[NU], cc[NX];
      factor_stage<NX, NU, V::DI>(m.dyn(pb), hx, m.hu, Pn, wb[q], m.lo, m.hi, t >= 1, Pt, K, Sv, kc, cc);
#pragma unroll
      for (int a = 0; a < NU; ++a) {
#pragma unroll
        for (int c = 0; c < NX; ++c) m.K(a, c, t) = K[a][c];
#pragma unroll
        for (int b = a; b < NU; ++b) m.SV(sym_idx<NU>(a, b), t) = Sv[a][b];
        m.KC(a, t) = kc[a];
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) m.CC(r, t) = cc[r];
      if (t >= 1) {
#pragma unroll
        for (int r = 0; r < NX; ++r)
#pragma unroll
          for (int c = r; c < NX; ++c) m.PU(sym_idx<NX>(r, c), t) = Pt[r][c];
#pragma unroll
        for (int r = 0; r < NX; ++r)
#pragma unroll
          for (int c = 0; c < NX; ++c) Pn[r][c] = Pt[r][c];
      }
    }
  }
}

// Affine backward sweep with the cached factors:
//   p_T = q_T;  k_t = kc_t - Sv_t B'p_{t+1};  p_t = q_t + c_t + A'p_{t+1} + K_t' B'p_{t+1},
// storing k_t for the rollout and p_{t+1} where stage t has a fixed input,
// with q_t = -2 Q_t r_t - C' sum_j (rho z_ij,t - lambda_ij,t) (QP on positions).
template <class V>
struct SweepStage {
  float K[V::NU][V::NX], sv[V::NS], kc[V::NU], q[V::NX], cc[V::NX];
  int8_t wt[V::NU];
  __device__ __forceinline__ void load(const V &m, int t) {
#pragma unroll
    for (int a = 0; a < V::NU; ++a) {
      wt[a] = m.w(a, t);
#pragma unroll
      for (int c = 0; c < V::NX; ++c) K[a][c] = m.K(a, c, t);
      kc[a] = m.KC(a, t);
    }
#pragma unroll
    for (int k = 0; k < V::NS; ++k) sv[k] = m.SV(k, t);
#pragma unroll
    for (int c = 0; c < V::NX; ++c) {
      q[c] = m.Q(c, t);
      cc[c] = m.CC(c, t);
    }
  }
};

// Later passes of one x-update change neither q nor the factors above the
// highest stage ts whose working set changed (the refactor starts there), so
// p_t above ts is what the previous sweep computed: the sweep stores p at
// every stage that is a multiple of kSweepMark, and a sweep given ts < T - 1
// restarts from the first such stage above ts (ts < 0 or >= T - 1: from T).
constexpr int kSweepMark = 4;
template <class V>
__device__ __forceinline__ int affine_sweep(const Prob &pb, const V &m, int T, int ts = -1) {
  constexpr int NX = V::NX, NU = V::NU, B = V::kSweepBatch;
  using D = Dyn<NX, NU, V::DI>;
  const int top = (ts >= 0 && ts < T - 1) ? min(T, (ts + kSweepMark) / kSweepMark * kSweepMark) : T;
  float p[NX];
  if (top == T) {
#pragma unroll
    for (int r = 0; r < NX; ++r) p[r] = m.Q(r, T);
  } else {
#pragma unroll
    for (int r = 0; r < NX; ++r) p[r] = m.PV(r, top);
  }
  for (int t0 = top - 1; t0 >= 0; t0 -= B) {
    SweepStage<V> st[B];
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (t0 - q >= 0) st[q].load(m, t0 - q);
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int t = t0 - q;
      if (t < 0) break;
      const SweepStage<V> &cur = st[q];
      bool fixed = false;
#pragma unroll
      for (int a = 0; a < NU; ++a) fixed |= (cur.wt[a] != 0);
      // p_{t+1} is read back for the costates of a stage with a fixed input,
      // and by a restarted sweep at the marked stages
      if (fixed || (t + 1) % kSweepMark == 0) {
#pragma unroll
        for (int r = 0; r < NX; ++r) m.PV(r, t + 1) = p[r];
      }
      float bp[NU];
      D::btx(m.dyn(pb), p, bp);
#pragma unroll
      for (int a = 0; a < NU; ++a) {
        float v = cur.kc[a];
#pragma unroll
        for (int b = 0; b < NU; ++b) v = fmaf(-cur.sv[a <= b ? sym_idx<NU>(a, b) : sym_idx<NU>(b, a)], bp[b], v);
        m.KV(a, t) = v;
      }
      if (t >= 1) {
        float np[NX];
        D::atx(m.dyn(pb), p, np);
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          float v = (cur.q[c] + cur.cc[c]) + np[c];
#pragma unroll
          for (int a = 0; a < NU; ++a) v = fmaf(cur.K[a][c], bp[a], v);
          np[c] = v;
        }
#pragma unroll
        for (int r = 0; r < NX; ++r) p[r] = np[r];
      }
    }
  }
  return top;
}

// relative FP32 rounding allowance of a multiplier (about 64 ulps)
constexpr float kMuNoise = 4e-6f;

struct StepInfo {
  float alpha;   // largest feasible fraction of the step toward the EQP solution
  int blk;       // flat index t*nu+c of the blocking bound (-1: none)
  int side;      // 1 lower, 2 upper
  float mu_min;  // most negative multiplier of the working set (0 if none < 0)
  int drop;      // its flat index (-1: none)
};

// Forward rollout u_t = K_t x_t + k_t, x_{t+1} = A x_t + B u_t (Eq. 8) into
// (UE, X), with the ratio test against the current inputs and, on stages with
// fixed inputs, the multipliers from the costates nu_{t+1} = P x + p (Eq. 9):
// g = H_u u_t + B' nu_{t+1}; mu = g at a lower bound, -g at an upper bound.
// A batch first reads the working sets and the per-stage data, then the
// costate data of its stages with a fixed input.
template <class V>
struct RollStage {
  float K[V::NU][V::NX], kv[V::NU], uc[V::NU], P[V::NP], pv[V::NX];
  float ueo[V::NU];   // a pending partial step: the previous pass's UE
  int8_t wt[V::NU];
  __device__ __forceinline__ void load(const V &m, int t, bool pending) {
    if (pending) {
#pragma unroll
      for (int a = 0; a < V::NU; ++a) ueo[a] = m.UE(a, t);
    }
#pragma unroll
    for (int a = 0; a < V::NU; ++a) {
#pragma unroll
      for (int c = 0; c < V::NX; ++c) K[a][c] = m.K(a, c, t);
      kv[a] = m.KV(a, t);
      uc[a] = m.U(a, t);
    }
  }
  __device__ __forceinline__ bool fixed() const {
    bool f = false;
#pragma unroll
    for (int a = 0; a < V::NU; ++a) f |= (wt[a] != 0);
    return f;
  }
  // the costates are needed only where an input is fixed
  __device__ __forceinline__ void load_costate(const V &m, int t) {
    if (fixed()) {
#pragma unroll
      for (int k = 0; k < V::NP; ++k) P[k] = m.PU(k, t + 1);
#pragma unroll
      for (int r = 0; r < V::NX; ++r) pv[r] = m.PV(r, t + 1);
    }
  }
};

// A blocked active-set pass moves the inputs the fraction alpha toward its
// EQP solution and fixes the blocking input at its bound.  That update is
// applied by the next pass's rollout as it reaches each stage (the refactor
// and the sweep in between do not read U), or by settle_iterate() when the
// loop ends right after the blocked pass.  Inside the loop no pass reads the
// states X beyond x_0 (every rollout starts from x_0), so X is set once, when
// the loop ends.
struct PendingStep {
  bool on;
  float alpha;   // step fraction
  int bt, ba;    // stage and component of the blocking input
  float bound;   // its bound value
};

// The loop ended on a blocked pass (or at its cap): apply a pending step to U
// and roll the states out from the inputs.
template <class V>
__device__ void settle_iterate(const Prob &pb, const V &m, int T, const PendingStep &pd) {
  constexpr int NX = V::NX, NU = V::NU, B = V::kBatch;
  using D = Dyn<NX, NU, V::DI>;
  float x[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) x[r] = m.X(r, 0);
  for (int t0 = 0; t0 < T; t0 += B) {
    float ub[B][NU], ue[B][NU];
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (t0 + q < T) {
#pragma unroll
        for (int a = 0; a < NU; ++a) {
          ub[q][a] = m.U(a, t0 + q);
          ue[q][a] = pd.on ? m.UE(a, t0 + q) : 0.f;
        }
      }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int t = t0 + q;
      if (t >= T) break;
      float u[NU];
#pragma unroll
      for (int a = 0; a < NU; ++a) {
        u[a] = ub[q][a];
        if (pd.on) {
          u[a] = (t == pd.bt && a == pd.ba) ? pd.bound : fmaf(pd.alpha, ue[q][a] - u[a], u[a]);
          m.U(a, t) = u[a];
        }
      }
      float xn[NX];
      D::ax(m.dyn(pb), x, xn);
      D::add_bu(m.dyn(pb), u, xn);
#pragma unroll
      for (int r = 0; r < NX; ++r) { x[r] = xn[r]; m.X(r, t + 1) = xn[r]; }
    }
  }
}

// With `fp64_states` the same inputs are also rolled out in FP64 into the
// refinement scratch (the first step of refine_solution, done here when this
// pass turns out to be the last one).
template <class V>
__device__ __forceinline__ StepInfo forward_rollout(const Prob &pb, const V &m, int T, bool fp64_states,
                                                    const PendingStep &pd) {
  constexpr int NX = V::NX, NU = V::NU, B = V::kBatch;
  using D = Dyn<NX, NU, V::DI>;
  StepInfo si{1.0f, -1, 0, 0.0f, -1};
  float x[NX];
  double xd[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    x[r] = m.X(r, 0);
    xd[r] = (double)x[r];
    if (fp64_states) m.d(r, 0) = xd[r];
  }
  for (int t0 = 0; t0 < T; t0 += B) {
    RollStage<V> st[B];
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (t0 + q < T) {
#pragma unroll
        for (int a = 0; a < NU; ++a) st[q].wt[a] = m.w(a, t0 + q);
      }
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (t0 + q < T) st[q].load(m, t0 + q, pd.on);
#pragma unroll
    for (int q = 0; q < B; ++q)
      if (t0 + q < T) st[q].load_costate(m, t0 + q);
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int t = t0 + q;
      if (t >= T) break;
      RollStage<V> &cur = st[q];
      if (pd.on) {   // the previous pass's partial step, at this stage
#pragma unroll
        for (int a = 0; a < NU; ++a) {
          cur.uc[a] = (t == pd.bt && a == pd.ba) ? pd.bound : fmaf(pd.alpha, cur.ueo[a] - cur.uc[a], cur.uc[a]);
          m.U(a, t) = cur.uc[a];
        }
      }
      float ue[NU];
#pragma unroll
      for (int a = 0; a < NU; ++a) {
        float v = cur.kv[a];
#pragma unroll
        for (int c = 0; c < NX; ++c) v = fmaf(cur.K[a][c], x[c], v);
        ue[a] = v;
        m.UE(a, t) = v;
      }
      float xn[NX];
      D::ax(m.dyn(pb), x, xn);
      D::add_bu(m.dyn(pb), ue, xn);
#pragma unroll
      for (int r = 0; r < NX; ++r) m.X(r, t + 1) = xn[r];   // the states are read only at the loop's end
      if (fp64_states) {
        double ud[NU], xdn[NX];
#pragma unroll
        for (int a = 0; a < NU; ++a) ud[a] = (double)ue[a];
        D::ax(m.dyn(pb), xd, xdn);
        D::add_bu(m.dyn(pb), ud, xdn);
#pragma unroll
        for (int r = 0; r < NX; ++r) { xd[r] = xdn[r]; m.d(r, t + 1) = xdn[r]; }
      }
#pragma unroll
      for (int a = 0; a < NU; ++a) {
        if (cur.wt[a] != 0) continue;
        const float uc = cur.uc[a];
        if (ue[a] < m.lo[a]) {
          const float r = (uc <= m.lo[a]) ? 0.f : (m.lo[a] - uc) / (ue[a] - uc);
          if (r < si.alpha) { si.alpha = r; si.blk = t * NU + a; si.side = 1; }
        } else if (ue[a] > m.hi[a]) {
          const float r = (uc >= m.hi[a]) ? 0.f : (m.hi[a] - uc) / (ue[a] - uc);
          if (r < si.alpha) { si.alpha = r; si.blk = t * NU + a; si.side = 2; }
        }
      }
      if (cur.fixed()) {
        float nu[NX];
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          float v = cur.pv[r];
#pragma unroll
          for (int c = 0; c < NX; ++c) v = fmaf(cur.P[r <= c ? sym_idx<NX>(r, c) : sym_idx<NX>(c, r)], xn[c], v);
          nu[r] = v;
        }
        float bn[NU], an[NX], bs[NU];
        D::btx(m.dyn(pb), nu, bn);
#pragma unroll
        for (int r = 0; r < NX; ++r) an[r] = fabsf(nu[r]);
        D::btx(m.dyn(pb), an, bs);   // |B|'|nu| for the general form with nonnegative B
#pragma unroll
        for (int a = 0; a < NU; ++a) {
          if (cur.wt[a] == 0) continue;
          const float g = fmaf(m.hu[a], ue[a], bn[a]);
          // a multiplier is trusted to be negative only beyond the FP32
          // rounding of the terms it is formed from
          const float mu = ((cur.wt[a] == 1) ? g : -g) + kMuNoise * (fabsf(m.hu[a] * ue[a]) + fabsf(bs[a]));
          if (mu < si.mu_min) { si.mu_min = mu; si.drop = t * NU + a; }
        }
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) x[r] = xn[r];
    }
  }
  return si;
}

// One step of mixed-precision iterative refinement of the final equality-QP
// solution (working set fixed).  The reduced gradient of the local QP at the
// FP32 solution is evaluated in FP64 (exact rollout of the stored inputs and
// the adjoint recursion nu_T = H_T x_T + q_T, nu_t = H_x x_t + q_t + A'nu_{t+1},
// g_t = H_u u_t + B'nu_{t+1}); the correction min 1/2 d'Hd + g_f'du (du on free
// inputs, homogeneous dynamics) is solved with the cached FP32 factors
// (k_t = -Sv (B'p + g_t), p_t = A'p + K'(B'p + g_t), p_T = 0) and applied in
// FP64 before rounding the iterate back to FP32.
// FROM_UE: the inputs to refine are the equality-QP inputs UE (the last
// active-set pass took the full step and its EQP solution was not copied),
// else U (the refined solution is written to U and X either way).  With
// `states_ready` the FP64 rollout of those inputs is already in the scratch.
template <class V, bool FROM_UE>
__device__ void refine_solution(const Prob &pb, const V &m, int T, int n_nbr, bool states_ready) {
  constexpr int NX = V::NX, NU = V::NU, NS = V::NS;
  using D = Dyn<NX, NU, V::DI>;
  auto uin = [&](int a, int t) -> float { return FROM_UE ? m.UE(a, t) : m.U(a, t); };
  // every loop below reads the data of V::kRefineBatch stages before it
  // computes the first of them (one memory round trip per batch)
  constexpr int B = V::kRefineBatch;
  double x[NX];
  if (!states_ready) {
#pragma unroll
    for (int r = 0; r < NX; ++r) { x[r] = (double)m.X(r, 0); m.d(r, 0) = x[r]; }
    // (1) exact rollout of the stored inputs
    for (int t0 = 0; t0 < T; t0 += B) {
      float ub[B][NU];
#pragma unroll
      for (int q = 0; q < B; ++q)
        if (t0 + q < T) {
#pragma unroll
          for (int a = 0; a < NU; ++a) ub[q][a] = uin(a, t0 + q);
        }
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int t = t0 + q;
        if (t >= T) break;
        double u[NU], xn[NX];
#pragma unroll
        for (int a = 0; a < NU; ++a) u[a] = (double)ub[q][a];
        D::ax(m.dyn(pb), x, xn);
        D::add_bu(m.dyn(pb), u, xn);
#pragma unroll
        for (int r = 0; r < NX; ++r) { x[r] = xn[r]; m.d(r, t + 1) = xn[r]; }
      }
    }
  }
  // (2) backward: FP64 adjoint (reduced gradient) and the FP32 correction sweep
  double nu[NX];
  {
    float hx[NX];
    m.hx(pb, T, T, n_nbr, hx);
#pragma unroll
    for (int r = 0; r < NX; ++r) nu[r] = fma((double)hx[r], m.d(r, T), (double)m.Q(r, T));
  }
  float pc[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) pc[r] = 0.f;
  struct BStage {
    float u[NU], K[NU][NX], sv[NS], q[NX];
    double xd[NX];
    int8_t wt[NU];
  };
  auto bload = [&](BStage &st, int t) {
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      st.u[a] = uin(a, t);
      st.wt[a] = m.w(a, t);
#pragma unroll
      for (int c = 0; c < NX; ++c) st.K[a][c] = m.K(a, c, t);
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) st.sv[k] = m.SV(k, t);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      st.q[c] = m.Q(c, t);
      st.xd[c] = m.d(c, t);
    }
  };
  for (int t0 = T - 1; t0 >= 0; t0 -= B) {
   BStage bst[B];
#pragma unroll
   for (int q = 0; q < B; ++q)
     if (t0 - q >= 0) bload(bst[q], t0 - q);
#pragma unroll
   for (int q = 0; q < B; ++q) {
    const int t = t0 - q;
    if (t < 0) break;
    const BStage &cur = bst[q];
    double bnu[NU];
    float bpc[NU], sg[NU];
    D::btx(m.dyn(pb), nu, bnu);
    D::btx(m.dyn(pb), pc, bpc);
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      const double g = fma((double)m.hu[a], (double)cur.u[a], bnu[a]);
      sg[a] = ((cur.wt[a] == 0) ? (float)g : 0.f) + bpc[a];
    }
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      float v = 0.f;
#pragma unroll
      for (int b = 0; b < NU; ++b) v = fmaf(-cur.sv[a <= b ? sym_idx<NU>(a, b) : sym_idx<NU>(b, a)], sg[b], v);
      m.KV(a, t) = v;
    }
    if (t >= 1) {
      float hx[NX];
      m.hx(pb, t, T, n_nbr, hx);
      float np[NX];
      double nn[NX];
      D::atx(m.dyn(pb), pc, np);
      D::atx(m.dyn(pb), nu, nn);
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        float v = np[c];
#pragma unroll
        for (int a = 0; a < NU; ++a) v = fmaf(cur.K[a][c], sg[a], v);
        pc[c] = v;
        nu[c] = nn[c] + fma((double)hx[c], cur.xd[c], (double)cur.q[c]);
      }
    }
   }
  }
  // (3) correction rollout, update in FP64, round back to FP32
  float dx[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) { dx[r] = 0.f; x[r] = m.d(r, 0); }
  struct FStage {
    float K[NU][NX], kv[NU], u[NU];
  };
  auto fload = [&](FStage &st, int t) {
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      st.kv[a] = m.KV(a, t);
      st.u[a] = uin(a, t);
#pragma unroll
      for (int c = 0; c < NX; ++c) st.K[a][c] = m.K(a, c, t);
    }
  };
  for (int t0 = 0; t0 < T; t0 += B) {
   FStage fst[B];
#pragma unroll
   for (int q = 0; q < B; ++q)
     if (t0 + q < T) fload(fst[q], t0 + q);
#pragma unroll
   for (int q = 0; q < B; ++q) {
    const int t = t0 + q;
    if (t >= T) break;
    const FStage &cur = fst[q];
    float du[NU], uf[NU];
    double ud[NU];
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      float v = cur.kv[a];
#pragma unroll
      for (int c = 0; c < NX; ++c) v = fmaf(cur.K[a][c], dx[c], v);
      du[a] = v;
      // a free input refined past its bound by a rounding-level amount is
      // put back on the bound, so that the next active-set start is feasible
      uf[a] = fminf(fmaxf((float)((double)cur.u[a] + (double)v), m.lo[a]), m.hi[a]);
      ud[a] = (double)uf[a];
      m.U(a, t) = uf[a];
    }
    float dxn[NX];
    double xn[NX];
    D::ax(m.dyn(pb), dx, dxn);
    D::add_bu(m.dyn(pb), du, dxn);
    D::ax(m.dyn(pb), x, xn);
    D::add_bu(m.dyn(pb), ud, xn);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      dx[r] = dxn[r];
      x[r] = xn[r];
      m.X(r, t + 1) = (float)xn[r];
    }
   }
  }
}

// One local QP's x-update at ADMM iteration k.  Returns 1 if the active-set
// loop hit its cap.  cnt[] accumulates pass / stage counters (in units of the
// view's stages: agent-stages or axis-stages).
template <class V>
__device__ int agent_xupdate(const Prob &pb, const WS &ws, const Scen &sc, const V &m, int k,
                             unsigned cnt[CT_NXU]) {
  constexpr int NX = V::NX, NU = V::NU;
  using D = Dyn<NX, NU, V::DI>;
  const int T = sc.T;
  const int n_nbr = sc.N - 1;
  int td = *m.dirty;
  const int cap = pb.max_as > 0 ? pb.max_as : 10 * T * NU;
  // the FP64-residual refinement, every iteration or once the residuals of
  // the last test are within refine_band of their tolerances (before that the
  // FP32 rounding of the local QP is far below what the iteration resolves)
  const bool refine = pb.refine && (pb.refine_band <= 0.f || uni(ws.sst[(long long)sc.s * ST_NCOL + ST_NEAR]) != 0);

  if (m.rho != m.rho_prev) {
    // The penalty changed after the last test (residual balancing).  The
    // position part of the linear term, GQP - rho (n_nbr C x + ZD) +
    // sum_j lambda_ij, moves by (rho_prev - rho)(n_nbr C x + ZD); the stage
    // Hessians change, so every factor is stale, including P_T.
    const float d = m.rho_prev - m.rho;
    for (int t = 0; t <= T; ++t)
#pragma unroll
      for (int c = 0; c < NU; ++c) m.Q(c, t) = fmaf(d, fmaf((float)n_nbr, m.X(c, t), m.ZD(c, t)), m.Q(c, t));
    float hT[NX];
    m.hx(pb, T, T, n_nbr, hT);
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) m.PU(sym_idx<NX>(r, c), T) = (r == c) ? hT[r] : 0.f;
    td = T - 1;
  }

  if ((k == 1 && !pb.cont) || !pb.hot) {
    // fresh start: empty working set ...
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int a = 0; a < NU; ++a)
        if (m.w(a, t) != 0) { m.w(a, t) = 0; td = max(td, t); }
    if (pb.warm) {
      // ... from the unconstrained affine LQ solution (Sec. IV-B), clipped
      if (!pb.cache) td = T - 1;
      if (td >= 0) { refactor(pb, m, T, n_nbr, td); cnt[CT_REFACTOR] += td + 1; td = -1; }
      affine_sweep(pb, m, T);
      cnt[CT_AFFINE] += T;
      (void)forward_rollout(pb, m, T, false, PendingStep{false, 0.f, -1, 0, 0.f});
      cnt[CT_PASSES] += 1;
    }
    float x[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) x[r] = m.X(r, 0);
    constexpr int B = V::kBatch;
    for (int t0 = 0; t0 < T; t0 += B) {
      float ub[B][NU];
#pragma unroll
      for (int q = 0; q < B; ++q)
#pragma unroll
        for (int a = 0; a < NU; ++a) ub[q][a] = (pb.warm && t0 + q < T) ? m.UE(a, t0 + q) : 0.f;
#pragma unroll
      for (int q = 0; q < B; ++q) {
        const int t = t0 + q;
        if (t >= T) break;
        float ust[NU];
#pragma unroll
        for (int a = 0; a < NU; ++a) {
          float u = ub[q][a];
          int8_t s = 0;
          if (u < m.lo[a]) { u = m.lo[a]; s = 1; }
          else if (u > m.hi[a]) { u = m.hi[a]; s = 2; }
          if (s) { m.w(a, t) = s; td = max(td, t); }
          ust[a] = u;
          m.U(a, t) = u;
        }
        float xn[NX];
        D::ax(m.dyn(pb), x, xn);
        D::add_bu(m.dyn(pb), ust, xn);
#pragma unroll
        for (int r = 0; r < NX; ++r) { x[r] = xn[r]; m.X(r, t + 1) = xn[r]; }
      }
    }
  }

  int done = 0;
  bool full = false;   // the last pass took the full step: its EQP solution is in (UE, X)
  int last_drop = -1, last_side = 0;   // bound released by the previous pass
  PendingStep pd{false, 0.f, -1, 0, 0.f};
  for (int it = 0; it < cap; ++it) {
    if (!pb.cache) td = T - 1;
    // the first pass sweeps every stage (q changed with the consensus step);
    // a later one from the highest stage whose working set changed
    const int ts = it == 0 ? -1 : td;
    if (td >= 0) { refactor(pb, m, T, n_nbr, td); cnt[CT_REFACTOR] += td + 1; td = -1; }
    const int swept = affine_sweep(pb, m, T, ts);
    cnt[CT_AFFINE] += (T + swept) / 2;   // (rollout stages + sweep stages) / 2
    const StepInfo si = forward_rollout(pb, m, T, refine, pd);
    pd.on = false;
    cnt[CT_PASSES] += 1;
    if (si.blk >= 0) {
      // blocked: move the fraction alpha toward the EQP solution and fix the
      // bound (the move itself is applied by the next rollout)
      const int bt = si.blk / NU, ba = si.blk % NU;
      float bnd = 0.f;   // the bound, selected without indexing the bound arrays
#pragma unroll
      for (int a = 0; a < NU; ++a)
        if (a == ba) bnd = (si.side == 1) ? m.lo[a] : m.hi[a];
      pd = PendingStep{true, fmaxf(si.alpha, 0.f), bt, ba, bnd};
      m.w(ba, bt) = (int8_t)si.side;
      td = max(td, bt);
      if (si.blk == last_drop && si.side == last_side) {
        // the bound released by the previous pass blocks again on the same
        // side right away: its multiplier was negative only at rounding
        // level; keep it and stop
        done = 1;
        break;
      }
      last_drop = -1;
      continue;
    }
    // full step: the EQP solution becomes the iterate (copied unless the
    // refinement below reads it from (UE, X) and writes the result)
    const bool drop = si.drop >= 0 && si.mu_min < -pb.mu_tol;
    if (drop || !refine) {   // (the rollout wrote its states into X already)
      // 8 stages per batch: their loads are all in flight before the stores
      for (int t0 = 0; t0 < T; t0 += 8) {
        float ub[8][NU];
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
          for (int a = 0; a < NU; ++a) ub[q][a] = (t0 + q < T) ? m.UE(a, t0 + q) : 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (t0 + q < T) {
#pragma unroll
            for (int a = 0; a < NU; ++a) m.U(a, t0 + q) = ub[q][a];
          }
      }
    }
    if (drop) {
      const int dt = si.drop / NU, da = si.drop % NU;
      last_side = m.w(da, dt);
      last_drop = si.drop;
      m.w(da, dt) = 0;
      td = max(td, dt);
      continue;
    }
    done = 1;
    full = true;
    break;
  }
  if (!full) settle_iterate(pb, m, T, pd);   // ended on a blocked pass or at the cap
  if (done && refine) {
    if (td >= 0) { refactor(pb, m, T, n_nbr, td); cnt[CT_REFACTOR] += td + 1; td = -1; }
    if (full) refine_solution<V, true>(pb, m, T, n_nbr, true);
    else refine_solution<V, false>(pb, m, T, n_nbr, false);
    cnt[CT_AFFINE] += 2 * T;
  }
  *m.dirty = td;
  return done ? 0 : 1;
}

// Lanes of a scenario's x-update: one per agent, or, with the separable
// double-integrator QP, one per (agent, axis), agents outer.
template <int NX, int NU, bool DI>
__host__ __device__ constexpr int xupdate_lanes(int N) { return DI ? N * NU : N; }

// LA (with DI): the axis problems' k and EQP-input slots in LDS at la,
// 2 T N NU floats.
template <int NX, int NU, bool DI, bool LA = false>
__device__ __forceinline__ int local_xupdate(const Prob &pb, const WS &ws, const Scen &sc, int l, int k,
                                             unsigned cnt[CT_NXU], float *la = nullptr) {
  if constexpr (DI) {
    AxisView<NX, NU, LA> m(pb, ws, sc, l / NU, l % NU);
    if constexpr (LA) {
      m.la = la;
      m.nl = (unsigned)(sc.N * NU);
      m.l = (unsigned)l;
    }
    return agent_xupdate(pb, ws, sc, m, k, cnt);
  } else {
    const AgentView<NX, NU, false> m(pb, ws, sc, l);
    return agent_xupdate(pb, ws, sc, m, k, cnt);
  }
}

// ===========================================================================
// Consensus (Eq. 4) + dual update (Eq. 5) for agent i at step t, all partners
// ===========================================================================
// Ordered copy (i, j) of a pair, positions p_i, p_j, lambda_ij (lambda_ji =
// -lambda_ij): a = p_i + lambda_ij/rho, b = p_j - lambda_ij/rho,
// v = d_min - n_ij'(a - b); the projection onto {n_ij'(a-b) >= d_min} moves a
// and b by +-(v+/2) n_ij, and Eq. 5 then gives lambda_ij <- -(rho/2) max(v, 0)
// n_ij = -gamma n_ij, which is evaluated in this closed form (no
// cancellation); the copy follows from Eq. 5 as z_ij = p_i + (lambda_ij -
// lambda_ij_new)/rho.  Lane (i, t) handles its own copies; the copy (j, i)
// computes every vector exactly negated and the same gamma, so only gamma is
// stored (one float per ordered copy, both equal).  lambda_ij of the previous
// step is rebuilt as -gamma n_prev with n_prev the normal of that step,
// recomputed from the previous positions C x^k (XP) with the same arithmetic,
// so the rebuilt value is bitwise the stored one of a vector layout.
// Normal of the ordered copy (i, j): n_ij = (p_i - p_j) / |p_i - p_j|, the
// negation of n_ji.  The given normals and the reference fallback are those
// of the canonical pair (f < s), negated for i > j.  Negation, subtraction
// and rounding commute exactly, so the two copies of a pair compute exactly
// opposite normals and, below, the same dual.
template <int NX, int NU>
__device__ __forceinline__ void pair_normal(const Prob &pb, const WS &ws, const Scen &sc, int i, int j, int t,
                                            const float pi[NU], const float pj[NU], float n[NU]) {
  const bool first = i < j;
  const int f = first ? i : j, s = first ? j : i;
  bool canonical = true;
  if (pb.normal_mode == NORMAL_FROZEN) {
    if (ws.normals) {
      const int pidx = f * sc.N - f * (f + 1) / 2 + (s - f - 1);
      const float *nv = ws.normals + (sc.po + (long long)pidx * sc.T + (t - 1)) * NU;
#pragma unroll
      for (int c = 0; c < NU; ++c) n[c] = nv[c];
    } else {
      reference_normal<NX, NU>(ws, sc, f, s, t, n);
    }
  } else {
    float d[NU];
#pragma unroll
    for (int c = 0; c < NU; ++c) d[c] = pi[c] - pj[c];
    canonical = !unit_normal<NU>(d, n);
    if (canonical) reference_normal<NX, NU>(ws, sc, f, s, t, n);
  }
  if (canonical && !first) {
#pragma unroll
    for (int c = 0; c < NU; ++c) n[c] = -n[c];
  }
}

// One agent-stage's consensus step over its partners.  REL: over-relaxation
// (Boyd et al. 2011, Sec. 3.4.3).  The z- and dual updates take
// xh = alpha C x^(k+1) + (1 - alpha) z^k for C x^(k+1), so the copies' z is
// kept: D = z_ij - z_ji (both orientations store exact negatives, as with
// gamma) and e = z_ij - C x_i (offsets stay small).  The duals keep their
// collapsed form lambda_ij = -gamma n, since the projection still moves the
// pair symmetrically about its midpoint.
// Partner masks (every scenario of at most 64 agents; MASK: known to hold
// for the whole launch): the agent-stage keeps a bit mask of its partners j
// whose gamma (ordered copy (i, j)) is nonzero, in the residual slots RED+5
// (j < 32) and RED+6; gamma is read only where the bit is set and written
// only where it was or becomes nonzero.  The stored gammas stay exact (zero
// where the bit is clear), so every other reader sees the same values, and
// every mode computes the same iterates, while an inactive pair, most of
// them, costs no memory access.  A set bit whose gamma was cleared by other
// code only costs a read of that zero.
template <int NX, int NU, bool REL, bool MASK = false>
__device__ void pair_agent_stage_impl(const Prob &pb, const WS &ws, const Scen &sc, int i, int t,
                                      const float *__restrict__ lpos, const float *__restrict__ lprev, int lofs) {
  using F = Fld<NX, NU>;
  const int N = sc.N;
  float *R = ws.fr + sc.fo;
  const unsigned GS = (unsigned)sc.GS, gi = (unsigned)(t * N + i);   // this agent-stage
  auto Ri = [&](int f) -> float & { return fref(R, GS, gi, f); };
  float pi[NU], qi[NU];   // positions of this step and of the previous one
  bool bad = false;
#pragma unroll
  for (int c = 0; c < NU; ++c) { pi[c] = Ri(F::X + c); qi[c] = xpref<NX, NU>(R, GS, gi, c); }
#pragma unroll
  for (int c = 0; c < NX; ++c) bad |= !isfinite(Ri(F::X + c));
  // the last step's ZD and this stage's tracking term, read with the
  // positions (one memory round trip rather than another after the partners)
  float zdo[NU], gqp[NU];
#pragma unroll
  for (int c = 0; c < NU; ++c) { zdo[c] = Ri(F::QZ + NU + c); gqp[c] = Ri(F::GQP + c); }
  float *gm = ws.gam + sc.lo;
  // (the per-scenario penalty equals pb.rho unless it adapts)
  const float rho = pb.adapt ? ws.rhos[2 * sc.s] : pb.rho, irho = 1.0f / rho;
  const bool frozen = pb.normal_mode == NORMAL_FROZEN;
  float es[NU], zd[NU], ls[NU];   // sum (lam_old - 2 lam_new), sum (z - C x), sum lam_new
#pragma unroll
  for (int c = 0; c < NU; ++c) { es[c] = 0.f; zd[c] = 0.f; ls[c] = 0.f; }
  float r2 = 0.f, z2 = 0.f;
  // partner positions (this step and the previous one) from LDS when the
  // scenario's positions (from agent-stage lofs on) are staged there
  auto partner = [&](int j, float pj[NU], float qj[NU]) {
    if (lpos) {
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        pj[c] = lpos[(t * N + j - lofs) * NU + c];
        qj[c] = lprev[(t * N + j - lofs) * NU + c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        pj[c] = R[fidx(GS, (unsigned)(t * N + j), F::X + c)];
        qj[c] = xpref<NX, NU>(R, GS, (unsigned)(t * N + j), c);
      }
    }
  };
  auto partner_pos = [&](int j, float pj[NU]) {
    if (lpos) {
#pragma unroll
      for (int c = 0; c < NU; ++c) pj[c] = lpos[(t * N + j - lofs) * NU + c];
    } else {
#pragma unroll
      for (int c = 0; c < NU; ++c) pj[c] = R[fidx(GS, (unsigned)(t * N + j), F::X + c)];
    }
  };
  const int gbase = (t - 1) * N * N + i;        // + j * N: this lane's ordered copy (i, j)
  // The partner loop skips j == i and runs in batches of kPB partners: the
  // duals and positions of a batch are all read before the first is used
  // (each dual is read before this loop stores its own word).
  constexpr int kPB = REL ? 4 : 8;
  const int np = N - 1;
  auto jof = [&](int jj) { return jj + (jj >= i); };
  const long long LS = (long long)sc.T * N * N;
  float *ob = REL ? ws.orx + 2LL * NU * sc.lo : nullptr;   // plane c at ob + c LS
  const float al = pb.alpha, bl = 1.0f - pb.alpha;
  // squared distance beyond which an inactive pair cannot become active
  // (a margin of 0.1% over d_min covers the rounding of the normal); never
  // below the distance at which the normal falls back to the references
  // (unit_normal), whose half-plane does not follow the positions
  const float far2 = fmaxf((1.001f * pb.dmin) * (1.001f * pb.dmin), 1e-12f);
  const bool msk = MASK || N <= 64;
  unsigned mw0 = 0u, mw1 = 0u, nm0 = 0u, nm1 = 0u;   // msk: partners with gamma != 0, before / after
  if (msk) {
    mw0 = __float_as_uint(Ri(F::RED + 5));
    if (N > 32) mw1 = __float_as_uint(Ri(F::RED + 6));
  }
  auto was_on = [&](int j) -> bool { return (((j < 32) ? (mw0 >> j) : (mw1 >> (j - 32))) & 1u) != 0u; };
  // The full consensus step of partner j: gold is its dual before the step,
  // pj and qj its positions of this step and of the previous one, Dq and eq
  // its relaxed planes (REL).
  auto full = [&](int j, float gold, const float *pj, const float *qj, const float *Dq, const float *eq) {
    float n[NU];
    pair_normal<NX, NU>(pb, ws, sc, i, j, t, pi, pj, n);
    // lambda_ij of the previous step, -gamma_prev n_prev
    float lown[NU];
    {
      float np_[NU];
      if (frozen) {
#pragma unroll
        for (int c = 0; c < NU; ++c) np_[c] = n[c];
      } else if (gold != 0.f) {
        pair_normal<NX, NU>(pb, ws, sc, i, j, t, qi, qj, np_);
      } else {
        // an inactive pair's dual is zero whatever its normal
#pragma unroll
        for (int c = 0; c < NU; ++c) np_[c] = 0.f;
      }
#pragma unroll
      for (int c = 0; c < NU; ++c) lown[c] = -gold * np_[c];
    }
    const int li = gbase + j * N;  // this lane's ordered copy (i, j)
    float g = 0.f;
    float abv[NU];
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      // a - b; relaxed: xh_i - xh_j = alpha (p_i - p_j) + (1 - alpha) D
      float dx;
      if constexpr (REL) dx = fmaf(al, pi[c] - pj[c], bl * Dq[c]);
      else dx = pi[c] - pj[c];
      abv[c] = dx + 2.0f * irho * lown[c];
      g = fmaf(n[c], abv[c], g);
    }
    const float v = pb.dmin - g;
    const float gam = 0.5f * rho * fmaxf(v, 0.f);
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      const float lo = -gam * n[c];                  // lambda_ij after Eq. 5
      const float dl = (lown[c] - lo) * irho;        // z_ij - xh_i
      if constexpr (REL) {
        // e' = z_ij - C x_i = (1 - alpha)(z^k_ij - C x_i) + dl, z^k_ij = C x^k_i + e
        const float en = fmaf(bl, (qi[c] + eq[c]) - pi[c], dl);
        const float zo = pi[c] + en;
        ob[c * LS + li] = fmaf(fmaxf(v, 0.f), n[c], abv[c]);   // z_ij - z_ji after the projection
        ob[(NU + c) * LS + li] = en;
        es[c] += fmaf(rho, en, -lo);                 // rho (z_ij - C x_i) - lam_new
        zd[c] += en;
        ls[c] += lo;
        r2 = fmaf(en, en, r2);
        z2 = fmaf(zo, zo, z2);
      } else {
        const float zo = pi[c] + dl;
        es[c] += lown[c] - 2.0f * lo;                // rho z_ij - lam_new - rho C x_i
        zd[c] += dl;
        ls[c] += lo;
        r2 = fmaf(dl, dl, r2);
        z2 = fmaf(zo, zo, z2);
      }
    }
    // (the half-plane is active at this step iff gam > 0)
    if (msk) {
      const bool on = gam > 0.f;
      if (on || gold != 0.f) gm[li] = gam;
      if (on) {
        if (j < 32) nm0 |= 1u << j;
        else nm1 |= 1u << (j - 32);
      }
    } else {
      gm[li] = gam;
    }
  };
  if (REL || frozen) {
    // every partner takes the full step, in batches of kPB
    for (int j0 = 0; j0 < np; j0 += kPB) {
      float gb[kPB], pjb[kPB][NU], qjb[kPB][NU];
      float Db[REL ? kPB : 1][NU], eb[REL ? kPB : 1][NU];
#pragma unroll
      for (int q = 0; q < kPB; ++q)
        if (j0 + q < np) {
          gb[q] = (!msk || was_on(jof(j0 + q))) ? gm[gbase + jof(j0 + q) * N] : 0.f;
          partner(jof(j0 + q), pjb[q], qjb[q]);
          if constexpr (REL) {
#pragma unroll
            for (int c = 0; c < NU; ++c) {
              Db[q][c] = ob[c * LS + gbase + jof(j0 + q) * N];
              eb[q][c] = ob[(NU + c) * LS + gbase + jof(j0 + q) * N];
            }
          }
        }
#pragma unroll
      for (int q = 0; q < kPB; ++q) {
        if (j0 + q >= np) break;
        full(jof(j0 + q), gb[q], pjb[q], qjb[q], Db[REL ? q : 0], eb[REL ? q : 0]);
      }
    }
  } else {
    // Normals of the iterates, partners in chunks of 32.  A scan finds the
    // partners that need the full step: a nonzero dual before the step, or
    // a squared distance of at most far2.  The others were inactive and are
    // clearly apart, so the half-plane about their separation direction
    // holds with room to spare and they stay inactive: z_ij = C x_i and
    // every dual term is zero, and the scan records only the copy's norm
    // (and, without the mask, the zero dual).  The partners found then take
    // the full step in increasing order, up to four per lane at a time.  A
    // wave's lanes thus run the full step together: in a crossing, most
    // partner slots of a wave hold a near partner of some lane, while each
    // lane has few.
    for (int c0 = 0; c0 < np; c0 += 32) {
      const int cn = min(32, np - c0);
      unsigned need = 0u;
      for (int q0 = 0; q0 < cn; q0 += kPB) {
        float gb[kPB], pjb[kPB][NU];
#pragma unroll
        for (int q = 0; q < kPB; ++q)
          if (q0 + q < cn) {
            const int j = jof(c0 + q0 + q);
            gb[q] = msk ? (was_on(j) ? 1.f : 0.f) : gm[gbase + j * N];
            partner_pos(j, pjb[q]);
          }
#pragma unroll
        for (int q = 0; q < kPB; ++q) {
          if (q0 + q >= cn) break;
          float d2 = 0.f;
#pragma unroll
          for (int c = 0; c < NU; ++c) d2 = fmaf(pi[c] - pjb[q][c], pi[c] - pjb[q][c], d2);
          if (gb[q] == 0.f && d2 > far2) {
            // (its dual stays zero: the word already holds +0, the only zero
            // any step writes)
#pragma unroll
            for (int c = 0; c < NU; ++c) z2 = fmaf(pi[c], pi[c], z2);
          } else {
            need |= 1u << (q0 + q);
          }
        }
      }
      while (need) {
        int jb[4];
        float gb[4], pjb[4][NU], qjb[4][NU];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          jb[b] = -1;
          if (need) {
            const int j = jof(c0 + __builtin_ctz(need));
            need &= need - 1u;
            jb[b] = j;
            gb[b] = (!msk || was_on(j)) ? gm[gbase + j * N] : 0.f;
            partner(j, pjb[b], qjb[b]);
          }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (jb[b] >= 0) full(jb[b], gb[b], pjb[b], qjb[b], nullptr, nullptr);
      }
    }
  }
  if (msk) {
    Ri(F::RED + 5) = __uint_as_float(nm0);
    if (N > 32) Ri(F::RED + 6) = __uint_as_float(nm1);
  }
  float s2 = 0.f, ax2 = 0.f, aty2 = 0.f;
  const float nn = (float)(N - 1);
#pragma unroll
  for (int c = 0; c < NU; ++c) {
    // rho sum_j (z_ij^(k+1) - z_ij^k) = rho (n_nbr (C x^(k+1) - C x^k) + ZD^(k+1) - ZD^k)
    const float ds = rho * fmaf(nn, pi[c] - qi[c], zd[c] - zdo[c]);
    s2 = fmaf(ds, ds, s2);
    ax2 = fmaf(pi[c], pi[c], ax2);
    aty2 = fmaf(ls[c], ls[c], aty2);
    Ri(F::QZ + c) = fmaf(-rho * nn, pi[c], gqp[c]) - es[c];
    Ri(F::QZ + NU + c) = zd[c];
  }
  ax2 *= nn;
  if (pb.pbox) {
    // the position box block, as below; its linear term joins the consensus
    // part of q written above
    const float sg = pb.sigma;
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      const float yo = Ri(F::YP + c), mo = Ri(F::YP + NU + c);
      const float yn = fminf(fmaxf(pi[c] + mo / sg, pb.plo[c]), pb.phi[c]);
      const float mn = fmaf(sg, pi[c] - yn, mo);
      const float ds = sg * (yn - yo);
      Ri(F::YP + c) = yn;
      Ri(F::YP + NU + c) = mn;
      Ri(F::QZ + c) -= fmaf(sg, yn, -mn);
      r2 = fmaf(pi[c] - yn, pi[c] - yn, r2);
      s2 = fmaf(ds, ds, s2);
      ax2 = fmaf(pi[c], pi[c], ax2);
      z2 = fmaf(yn, yn, z2);
      aty2 = fmaf(mn, mn, aty2);
    }
  }
  if (pb.sbox) {
    // the state box block: y = clip(x + mu / sigma), mu += sigma (x - y), and
    // the next linear term -2 Q r - (sigma y - mu) on those states
    const float sg = pb.sigma;
#pragma unroll
    for (int c = 0; c < NX - NU; ++c) {
      const float xv = Ri(F::X + NU + c), yo = Ri(F::YM + c), mo = Ri(F::YM + NU + c);
      const float yn = fminf(fmaxf(xv + mo / sg, pb.slo[c]), pb.shi[c]);
      const float mn = fmaf(sg, xv - yn, mo);
      const float ds = sg * (yn - yo);
      Ri(F::YM + c) = yn;
      Ri(F::YM + NU + c) = mn;
      Ri(F::Q + NU + c) = Ri(F::GQV + c) - fmaf(sg, yn, -mn);
      r2 = fmaf(xv - yn, xv - yn, r2);
      s2 = fmaf(ds, ds, s2);
      ax2 = fmaf(xv, xv, ax2);
      z2 = fmaf(yn, yn, z2);
      aty2 = fmaf(mn, mn, aty2);
    }
  }
  if (bad) r2 = NAN;
  Ri(F::RED + 0) = r2;
  Ri(F::RED + 1) = s2;
  Ri(F::RED + 2) = ax2;
  Ri(F::RED + 3) = z2;
  Ri(F::RED + 4) = aty2;
}

// Momentum ADMM (the fast ADMM with restart of Goldstein et al. 2014, Alg. 8)
// on the consensus block.  Iteration k's x-update took the extrapolated
// copies zh and duals lh; its consensus step projects C x_i + lh_ij / rho
// (the pair still moves symmetrically about its midpoint, so lambda_ij =
// -gamma n again) and keeps z_k, lambda_k and the previous ones per ordered
// copy.  Planes (each shaped like the gamma region, copy (i, j) at
// [t][j][i]): MP_LH lh, MP_ZH zh, MP_ZK z_k, MP_ZK1 z_(k-1), MP_LK lambda_k,
// MP_LK1 lambda_(k-1), NU planes each.  Both orientations of a pair store
// exact negatives of each other's differences, as with gamma.
enum { MP_LH = 0, MP_ZH, MP_ZK, MP_ZK1, MP_LK, MP_LK1, MP_N };

template <int NX, int NU>
__device__ void pair_agent_stage_mom(const Prob &pb, const WS &ws, const Scen &sc, int i, int t,
                                     const float *__restrict__ lpos, int lofs = 0) {
  using F = Fld<NX, NU>;
  const int N = sc.N;
  float *R = ws.fr + sc.fo;
  const unsigned GS = (unsigned)sc.GS, gi = (unsigned)(t * N + i);
  auto Ri = [&](int f) -> float & { return fref(R, GS, gi, f); };
  float pi[NU];
  bool bad = false;
#pragma unroll
  for (int c = 0; c < NU; ++c) pi[c] = Ri(F::X + c);
#pragma unroll
  for (int c = 0; c < NX; ++c) bad |= !isfinite(Ri(F::X + c));
  float *gm = ws.gam + sc.lo;
  const long long LS = (long long)sc.T * N * N;
  float *mp = ws.mom + (long long)MP_N * NU * sc.lo;
  auto plane = [&](int which, int c) { return mp + (long long)(which * NU + c) * LS; };
  const float rho = pb.rho, irho = 1.0f / rho;
  float szk[NU], szh[NU], ls[NU];
#pragma unroll
  for (int c = 0; c < NU; ++c) { szk[c] = 0.f; szh[c] = 0.f; ls[c] = 0.f; }
  float r2 = 0.f, z2 = 0.f, c2 = 0.f;
  const int gbase = (t - 1) * N * N + i;
  // partners in batches of kPB: a batch's loads are all issued before the
  // first is used
  constexpr int kPB = 4;
  const int np = N - 1;
  for (int j0 = 0; j0 < np; j0 += kPB) {
   float pjb[kPB][NU], lhb[kPB][NU], zhb[kPB][NU], zkb[kPB][NU], lkb[kPB][NU];
#pragma unroll
   for (int q = 0; q < kPB; ++q)
    if (j0 + q < np) {
      const int j = (j0 + q) + ((j0 + q) >= i);
      const int li = gbase + j * N;
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        pjb[q][c] = lpos ? lpos[(t * N + j - lofs) * NU + c] : R[fidx(GS, (unsigned)(t * N + j), F::X + c)];
        lhb[q][c] = plane(MP_LH, c)[li];
        zhb[q][c] = plane(MP_ZH, c)[li];
        zkb[q][c] = plane(MP_ZK, c)[li];
        lkb[q][c] = plane(MP_LK, c)[li];
      }
    }
#pragma unroll
   for (int q = 0; q < kPB; ++q) {
    if (j0 + q >= np) break;
    const int j = (j0 + q) + ((j0 + q) >= i);
    const int li = gbase + j * N;
    const float *pj = pjb[q], *lh = lhb[q], *zh = zhb[q], *zk = zkb[q], *lk = lkb[q];
    float n[NU];
    pair_normal<NX, NU>(pb, ws, sc, i, j, t, pi, pj, n);
    float ab[NU], g = 0.f;
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      ab[c] = (pi[c] - pj[c]) + 2.0f * irho * lh[c];   // a - b with the extrapolated duals
      g = fmaf(n[c], ab[c], g);
    }
    const float v = pb.dmin - g;
    const float gam = 0.5f * rho * fmaxf(v, 0.f);
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      const float lo = -gam * n[c];                     // lambda_k
      const float z = pi[c] + (lh[c] - lo) * irho;      // z_k
      plane(MP_ZK1, c)[li] = zk[c];
      plane(MP_ZK, c)[li] = z;
      plane(MP_LK1, c)[li] = lk[c];
      plane(MP_LK, c)[li] = lo;
      const float dl = lo - lh[c], dz = z - zh[c];
      c2 = fmaf(dl * dl, irho, fmaf(rho * dz, dz, c2));
      r2 = fmaf(pi[c] - z, pi[c] - z, r2);
      z2 = fmaf(z, z, z2);
      szk[c] += z;
      szh[c] += zh[c];
      ls[c] += lo;
    }
    gm[li] = gam;
   }
  }
  float s2 = 0.f, ax2 = 0.f, aty2 = 0.f;
#pragma unroll
  for (int c = 0; c < NU; ++c) {
    // rho sum_j (z_k - zh_k): the x-update took zh
    const float ds = rho * (szk[c] - szh[c]);
    s2 = fmaf(ds, ds, s2);
    ax2 = fmaf(pi[c], pi[c], ax2);
    aty2 = fmaf(ls[c], ls[c], aty2);
  }
  ax2 *= (float)(N - 1);
  if (bad) r2 = NAN;
  Ri(F::RED + 0) = r2;
  Ri(F::RED + 1) = s2;
  Ri(F::RED + 2) = ax2;
  Ri(F::RED + 3) = z2;
  Ri(F::RED + 4) = aty2;
  Ri(F::RED + 5) = c2;
}

// After the stopping test of an unfinished iteration: the next iteration's
// extrapolated duals and copies (or the previous ones, after a restart), and
// the position part of the next linear term, GQP - sum_j (rho zh - lh).
template <int NX, int NU>
__device__ void mom_extrapolate(const Prob &pb, const WS &ws, const Scen &sc, int i, int t) {
  using F = Fld<NX, NU>;
  const int N = sc.N;
  float *R = ws.fr + sc.fo;
  const unsigned GS = (unsigned)sc.GS, gi = (unsigned)(t * N + i);
  auto Ri = [&](int f) -> float & { return fref(R, GS, gi, f); };
  const long long LS = (long long)sc.T * N * N;
  float *mp = ws.mom + (long long)MP_N * NU * sc.lo;
  auto plane = [&](int which, int c) { return mp + (long long)(which * NU + c) * LS; };
  const float *st = ws.momst + 4LL * sc.s;
  const float beta = st[2];
  const bool restart = st[3] != 0.f;
  float szh[NU], slh[NU];
#pragma unroll
  for (int c = 0; c < NU; ++c) { szh[c] = 0.f; slh[c] = 0.f; }
  const int gbase = (t - 1) * N * N + i;
  for (int jj = 0; jj < N - 1; ++jj) {
    const int li = gbase + (jj + (jj >= i)) * N;
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      const float zk = plane(MP_ZK, c)[li], zk1 = plane(MP_ZK1, c)[li];
      const float lk = plane(MP_LK, c)[li], lk1 = plane(MP_LK1, c)[li];
      const float zh = restart ? zk1 : fmaf(beta, zk - zk1, zk);
      const float lh = restart ? lk1 : fmaf(beta, lk - lk1, lk);
      plane(MP_ZH, c)[li] = zh;
      plane(MP_LH, c)[li] = lh;
      szh[c] += zh;
      slh[c] += lh;
    }
  }
#pragma unroll
  for (int c = 0; c < NU; ++c) Ri(F::QZ + c) = fmaf(-pb.rho, szh[c], Ri(F::GQP + c)) + slh[c];
}

template <int NX, int NU>
__device__ __forceinline__ void pair_agent_stage(const Prob &pb, const WS &ws, const Scen &sc, int i, int t,
                                                 const float *__restrict__ lpos, const float *__restrict__ lprev,
                                                 int lofs = 0) {
  if (pb.mom) pair_agent_stage_mom<NX, NU>(pb, ws, sc, i, t, lpos, lofs);
  else if (pb.relax) pair_agent_stage_impl<NX, NU, true>(pb, ws, sc, i, t, lpos, lprev, lofs);
  else pair_agent_stage_impl<NX, NU, false>(pb, ws, sc, i, t, lpos, lprev, lofs);
}

// After a consensus step: the positions of this step become the previous
// positions (XP) of the next one.  Kept out of the partner loop, which reads
// every partner's previous positions.
template <int NX, int NU>
__device__ __forceinline__ void commit_positions(const WS &ws, const Scen &sc, int tid, int nthreads) {
  using F = Fld<NX, NU>;
  float *R = ws.fr + sc.fo;
  const unsigned GS = (unsigned)sc.GS;
  for (int idx = sc.N + tid; idx < sc.GS; idx += nthreads)
#pragma unroll
    for (int c = 0; c < NU; ++c) xpref<NX, NU>(R, GS, (unsigned)idx, c) = fref(R, GS, (unsigned)idx, F::X + c);
}

// The stopping test's sums over agent-stages run in blocks of kTestBlock
// consecutive agent-stages (t >= 1, agent fastest): in block b, lane l adds
// the block's stages l, l + 64, ... in that order, starting from zero; the
// lane then adds the block sums in block order, and a fixed butterfly adds
// the lanes.  Every mode keeps this order (the many-workgroup mode forms the
// blocks in parallel), so every mode computes the same residuals.
constexpr int kTestBlock = 512;

template <int NX, int NU>
__device__ __forceinline__ void test_block(const WS &ws, const Scen &sc, int b0, int lane, float p[5]) {
  using F = Fld<NX, NU>;
  const float *R = ws.fr + sc.fo;
  const int NT = sc.N * sc.T;
  constexpr int U = kTestBlock / 64;
  float v[U][5];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int idx = b0 + lane + 64 * u;
    if (idx < NT) {
#pragma unroll
      for (int q = 0; q < 5; ++q) v[u][q] = R[fidx((unsigned)sc.GS, (unsigned)(sc.N + idx), F::RED + q)];
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) p[q] = 0.f;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (b0 + lane + 64 * u < NT) {
#pragma unroll
      for (int q = 0; q < 5; ++q) p[q] += v[u][q];
    }
}

// Residual norms and the stopping test of Sec. V-A (Boyd et al. 2011, Sec.
// 3.3.1): p = 2 P T dp consensus rows, n = N T dp position variables.
// Executed by one full wavefront, summing in the block order above; `part`:
// the block sums already formed ([b][5][64]), else formed here.
// MOM: the momentum variant's combined residual and extrapolation decision.
template <int NX, int NU, bool MOM = false>
__device__ int scenario_test(const Prob &pb, const WS &ws, const Scen &sc, int k, int lane, int cap_hit,
                             const float *part = nullptr) {
  using F = Fld<NX, NU>;
  const float *R = ws.fr + sc.fo;
  const int NT = sc.N * sc.T;
  float a[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  for (int b0 = 0, b = 0; b0 < NT; b0 += kTestBlock, ++b) {
    float p[5];
    if (part) {
#pragma unroll
      for (int q = 0; q < 5; ++q) p[q] = part[(b * 5 + q) * 64 + lane];
    } else {
      test_block<NX, NU>(ws, sc, b0, lane, p);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) a[q] += p[q];
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) a[q] = wave_sum(a[q]);
  float cmom = 0.f;   // momentum: the combined residual of the iteration
  if constexpr (MOM) {
    for (int idx = lane; idx < NT; idx += 64) cmom += R[fidx((unsigned)sc.GS, (unsigned)(sc.N + idx), F::RED + 5)];
    cmom = wave_sum(cmom);
  }
  int done = 0;
  if (lane == 0) {
    const float P = 0.5f * (float)sc.N * (float)(sc.N - 1);
    const float rn = sqrtf(a[0]), sn = sqrtf(a[1]);
    // the state box block adds N T (NX - NU) rows and coupled states
    const float nbox = (float)sc.N * (float)sc.T * (float)NU * (float)(pb.sbox + pb.pbox);
    const float epri = sqrtf(fmaf(2.0f * P, (float)sc.T * (float)NU, nbox)) * pb.eps_abs +
                       pb.eps_rel * fmaxf(sqrtf(a[2]), sqrtf(a[3]));
    const float edual = sqrtf(fmaf((float)sc.N, (float)sc.T * (float)NU, nbox)) * pb.eps_abs +
                        pb.eps_rel * sqrtf(a[4]);
    int *st = ws.sst + (long long)sc.s * ST_NCOL;
    float *sn_out = ws.snorm + (long long)sc.s * SN_NCOL;
    int status = SCEN_MAX_ITER;
    if (cap_hit) { status = SCEN_CAP; done = 1; }
    else if (!isfinite(rn) || !isfinite(sn)) { status = SCEN_NONFINITE; done = 1; }
    // (a continuing SQP round's first x-update still used the linear term of
    // the previous round's normals: its residuals prove nothing yet)
    else if (rn <= epri && sn <= edual && (k >= 2 || !pb.cont)) { status = SCEN_CONVERGED; done = 1; }
    else if (k >= pb.max_iter) { done = 1; }
    if (!cap_hit) {
      sn_out[SN_R] = rn; sn_out[SN_S] = sn; sn_out[SN_EPRI] = epri; sn_out[SN_EDUAL] = edual;
      if (ws.hist) {
        float *h = ws.hist + 2 * ((long long)sc.s * pb.max_iter + (k - 1));
        h[0] = rn;
        h[1] = sn;
      }
    }
    st[ST_NEAR] = (rn <= pb.refine_band * epri && sn <= pb.refine_band * edual) ? 1 : 0;
    // residual balancing (Boyd et al. 2011, Sec. 3.4.1): the next iteration's
    // penalty; the last one is kept for the x-update's correction
    float *rh = ws.rhos + 2 * sc.s;
    rh[1] = rh[0];
    if (!done && pb.adapt && k % pb.rho_every == 0) {
      if (rn > pb.rho_mu * sn) rh[0] = rh[1] * pb.rho_tau;
      else if (sn > pb.rho_mu * rn) rh[0] = rh[1] / pb.rho_tau;
    }
    // momentum (Goldstein et al. 2014, Alg. 8): extrapolate if the combined
    // residual fell by mom_eta, else restart from the previous iterates
    if (MOM && !done) {
      float *ms = ws.momst + 4LL * sc.s;
      const float a0 = ms[0], cp = ms[1];
      if (cmom < pb.mom_eta * cp) {
        const float an = 0.5f * (1.0f + sqrtf(fmaf(4.0f * a0, a0, 1.0f)));
        ms[2] = (a0 - 1.0f) / an;
        ms[3] = 0.f;
        ms[0] = an;
        ms[1] = cmom;
      } else {
        ms[2] = 0.f;
        ms[3] = 1.f;
        ms[0] = 1.f;
        ms[1] = cp / pb.mom_eta;
      }
    }
    st[ST_STATUS] = status;
    st[ST_ITERS] = k;
    st[ST_DONE] = done;
  }
  return __shfl(done, 0, 64);
}

// Per-scenario initial state: z^(0) = C r, lambda^(0) = 0 (the position
// linear term starts at -2 Q r - rho n_nbr C r), P_T = H_T, empty working
// sets, every factor stale.
template <int NX, int NU, bool MOM = false>
__device__ void scenario_setup(const Prob &pb, const WS &ws, const Scen &sc, int tid, int nthreads) {
  using F = Fld<NX, NU>;
  const int N = sc.N, T = sc.T, GS = sc.GS;
  float *R = ws.fr + sc.fo;
  int8_t *Wb = ws.wr + sc.bo;
  const float *qd = ws.qd + (long long)sc.s * NX;
  const int n_nbr = N - 1;
  if (pb.cont) {
    // A later SQP round: the iterate, working sets and factors carry over,
    // and so do the duals if the previous round converged.  Otherwise (its
    // half-planes may have been infeasible, the duals grown without bound)
    // the duals restart at zero with z = C x: gamma = 0, ZD = 0 and the
    // position part of the linear term -2 Q r - rho n_nbr C x.
    if (uni(ws.sst[(long long)sc.s * ST_NCOL + ST_COLD])) {
      for (int idx = tid; idx < GS; idx += nthreads) {
        auto Rg = [&](int f) -> float & { return R[fidx((unsigned)GS, (unsigned)idx, f)]; };
#pragma unroll
        for (int c = 0; c < NU; ++c) {
          Rg(F::QZ + c) = fmaf(-ws.rhos[2 * sc.s] * (float)n_nbr, Rg(F::X + c), Rg(F::GQP + c));
          Rg(F::QZ + NU + c) = 0.f;
          if (pb.pbox && idx >= N) {
            const float y0 = fminf(fmaxf(Rg(F::X + c), pb.plo[c]), pb.phi[c]);
            Rg(F::YP + c) = y0;
            Rg(F::YP + NU + c) = 0.f;
            Rg(F::QZ + c) -= pb.sigma * y0;
          }
        }
        // and the state box block restarts at y = clip(x), mu = 0
        if (pb.sbox && idx >= N) {
#pragma unroll
          for (int c = 0; c < NX - NU; ++c) {
            const float y0 = fminf(fmaxf(Rg(F::X + NU + c), pb.slo[c]), pb.shi[c]);
            Rg(F::YM + c) = y0;
            Rg(F::YM + NU + c) = 0.f;
            Rg(F::Q + NU + c) = fmaf(-pb.sigma, y0, Rg(F::GQV + c));
          }
        }
      }
      float *gm = ws.gam + sc.lo;
      for (int idx = tid; idx < T * N * N; idx += nthreads) gm[idx] = 0.f;
      if (pb.relax) {
        // the copies restart at z = C x: D = C x_i - C x_j, e = 0
        const long long LS = (long long)T * N * N;
        float *ob = ws.orx + 2LL * NU * sc.lo;
        for (int idx = tid; idx < T * N * N; idx += nthreads) {
          const int i = idx % N, j = (idx / N) % N, t = idx / (N * N) + 1;
#pragma unroll
          for (int c = 0; c < NU; ++c) {
            ob[c * LS + idx] = R[fidx((unsigned)GS, (unsigned)(t * N + i), F::X + c)] -
                               R[fidx((unsigned)GS, (unsigned)(t * N + j), F::X + c)];
            ob[(NU + c) * LS + idx] = 0.f;
          }
        }
      }
    }
    if (tid == 0) {
      int *st = ws.sst + (long long)sc.s * ST_NCOL;
      st[ST_STATUS] = SCEN_MAX_ITER;
      st[ST_ITERS] = 0;
      st[ST_CAP] = 0;
      st[ST_DONE] = 0;
      st[ST_NEAR] = 0;
      float *sn = ws.snorm + (long long)sc.s * SN_NCOL;
      sn[SN_R] = sn[SN_S] = sn[SN_EPRI] = sn[SN_EDUAL] = 0.f;
    }
    return;
  }
  for (int idx = tid; idx < GS; idx += nthreads) {
    const int t = idx / N, i = idx % N;
    auto Rg = [&](int f) -> float & { return R[fidx((unsigned)GS, (unsigned)idx, f)]; };
    const float *r = ws.xref + (sc.xo + (long long)i * (T + 1) + t) * NX;
    const float w = (t == T) ? pb.qT : 1.0f;
    const float *qi = ws.aq ? ws.aq + (sc.ao + i) * NX : qd;   // this agent's weights
    float gq[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      gq[c] = (t >= 1) ? -2.0f * w * qi[c] * r[c] : 0.f;
      if (c >= NU) {
        // the state box: y^0 = the reference's states clipped, mu^0 = 0, and
        // the linear term -2 Q r - (sigma y - mu)
        const float y0 = fminf(fmaxf(r[c], pb.slo[c - NU]), pb.shi[c - NU]);
        Rg(F::GQV + c - NU) = gq[c];
        Rg(F::YM + c - NU) = y0;
        Rg(F::YM + NU + c - NU) = 0.f;
        Rg(F::Q + c) = (pb.sbox && t >= 1) ? fmaf(-pb.sigma, y0, gq[c]) : gq[c];
      }
    }
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      // x^0 := r so that z^0 = C r, lambda^0 = 0
      Rg(F::GQP + c) = gq[c];
      float qz = fmaf(-pb.rho * (float)n_nbr, r[c], gq[c]);
      // the position box: y^0 = the reference clipped, mu^0 = 0
      const float y0 = fminf(fmaxf(r[c], pb.plo[c]), pb.phi[c]);
      Rg(F::YP + c) = y0;
      Rg(F::YP + NU + c) = 0.f;
      if (pb.pbox && t >= 1) qz -= pb.sigma * y0;
      Rg(F::QZ + c) = qz;
      xpref<NX, NU>(R, (unsigned)GS, (unsigned)idx, c) = r[c];
      Rg(F::QZ + NU + c) = 0.f;
      uref<NX, NU>(R, (unsigned)GS, (unsigned)idx, c) = 0.f;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) Wb[(unsigned)idx * 4u + c] = 0;
    Rg(F::RED + 5) = 0.f;   // no partner with a nonzero gamma (the consensus step's mask)
    Rg(F::RED + 6) = 0.f;
    if (t == 0) {
      const float *x0 = ws.x0 + (sc.ao + i) * NX;
#pragma unroll
      for (int c = 0; c < NX; ++c) Rg(F::X + c) = x0[c];
#pragma unroll
      for (int c = 0; c < NU; ++c) ws.adirty[(sc.ao + i) * NU + c] = T - 1;
    }
    if (t == T) {
      float hx[NX];
      stage_hx<NX, NU>(pb, qi, T, T, n_nbr, pb.rho, hx);
#pragma unroll
      for (int r2 = 0; r2 < NX; ++r2)
#pragma unroll
        for (int c = r2; c < NX; ++c) Rg(F::PU + sym_idx<NX>(r2, c)) = (r2 == c) ? hx[r2] : 0.f;
      // and of each axis problem (the axis-stage region follows the fields)
      float *AP = R + (size_t)F::NF * GS + (size_t)AXA_P * GS * NU;
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        float *e = AP + ((size_t)idx * NU + c) * 4;
        e[0] = hx[c];
        e[1] = 0.f;
        e[2] = hx[NU + c];
      }
    }
  }
  const int LS = T * N * N;
  float *gm = ws.gam + sc.lo;
  for (int idx = tid; idx < LS; idx += nthreads) gm[idx] = 0.f;
  if constexpr (MOM) {
    // momentum: zh = z_0 = z_(-1) = C r, lh = lambda_0 = lambda_(-1) = 0;
    // alpha_1 = 1, c_0 = inf
    float *mp = ws.mom + (long long)MP_N * NU * sc.lo;
    for (int idx = tid; idx < LS; idx += nthreads) {
      const int i = idx % N, t = idx / (N * N) + 1;
      const float *ri = ws.xref + (sc.xo + (long long)i * (T + 1) + t) * NX;
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        mp[(long long)(MP_LH * NU + c) * LS + idx] = 0.f;
        mp[(long long)(MP_ZH * NU + c) * LS + idx] = ri[c];
        mp[(long long)(MP_ZK * NU + c) * LS + idx] = ri[c];
        mp[(long long)(MP_ZK1 * NU + c) * LS + idx] = ri[c];
        mp[(long long)(MP_LK * NU + c) * LS + idx] = 0.f;
        mp[(long long)(MP_LK1 * NU + c) * LS + idx] = 0.f;
      }
    }
    if (tid == 0) {
      float *ms = ws.momst + 4LL * sc.s;
      ms[0] = 1.f;
      ms[1] = INFINITY;
      ms[2] = 0.f;
      ms[3] = 0.f;
    }
  }
  if (pb.relax) {
    // the copies' z^0 = C r: D = r_i - r_j, e = 0 (copy (i, j) at [t][j][i])
    float *ob = ws.orx + 2LL * NU * sc.lo;
    for (int idx = tid; idx < LS; idx += nthreads) {
      const int i = idx % N, j = (idx / N) % N, t = idx / (N * N) + 1;
      const float *ri = ws.xref + (sc.xo + (long long)i * (T + 1) + t) * NX;
      const float *rj = ws.xref + (sc.xo + (long long)j * (T + 1) + t) * NX;
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        ob[(long long)c * LS + idx] = ri[c] - rj[c];
        ob[(long long)(NU + c) * LS + idx] = 0.f;
      }
    }
  }
  if (tid == 0) {
    int *st = ws.sst + (long long)sc.s * ST_NCOL;
    st[ST_STATUS] = SCEN_MAX_ITER;
    st[ST_ITERS] = 0;
    st[ST_CAP] = 0;
    st[ST_DONE] = 0;
    st[ST_NEAR] = 0;
    float *sn = ws.snorm + (long long)sc.s * SN_NCOL;
    sn[SN_R] = sn[SN_S] = sn[SN_EPRI] = sn[SN_EDUAL] = 0.f;
    ws.rhos[2 * sc.s] = ws.rhos[2 * sc.s + 1] = pb.rho;
  }
}

__device__ __forceinline__ void add_counters(const WS &ws, int s, const long long c[CT_NCOL]) {
#pragma unroll
  for (int q = 0; q < CT_NCOL; ++q)
    if (c[q]) atomicAdd(ws.cnt + (long long)s * CT_NCOL + q, (unsigned long long)c[q]);
}

// the x-update's own counters of one lane (the first CT_NXU columns)
__device__ __forceinline__ void add_counters(const WS &ws, int s, const unsigned c[CT_NXU]) {
#pragma unroll
  for (int q = 0; q < CT_NXU; ++q)
    if (c[q]) atomicAdd(ws.cnt + (long long)s * CT_NCOL + q, (unsigned long long)c[q]);
}

// ===========================================================================
// Kernels: plain path (one scenario, host loop)
// ===========================================================================
template <int NX, int NU>
__global__ __launch_bounds__(256) void k_setup(Prob pb, WS ws, int s) {
  const Scen sc = load_scen(ws, s);
  if (pb.mom) scenario_setup<NX, NU, true>(pb, ws, sc, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
  else scenario_setup<NX, NU>(pb, ws, sc, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
  if (!pb.cont && blockIdx.x == 0 && threadIdx.x < CT_NCOL) ws.cnt[(long long)s * CT_NCOL + threadIdx.x] = 0ull;
}

template <int NX, int NU, bool DI>
__global__ __launch_bounds__(64) void k_xupdate(Prob pb, WS ws, int s, int k) {
  const Scen sc = load_scen(ws, s);
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= xupdate_lanes<NX, NU, DI>(sc.N)) return;
  unsigned cnt[CT_NXU] = {};
  const int capped = local_xupdate<NX, NU, DI>(pb, ws, sc, l, k, cnt);
  if (capped) atomicOr(ws.sst + (long long)s * ST_NCOL + ST_CAP, 1);
  add_counters(ws, s, cnt);
}

template <int NX, int NU>
__global__ __launch_bounds__(256) void k_pair(Prob pb, WS ws, int s) {
  const Scen sc = load_scen(ws, s);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= sc.N * sc.T) return;
  pair_agent_stage<NX, NU>(pb, ws, sc, idx % sc.N, idx / sc.N + 1, nullptr, nullptr);
  if (idx == 0) {
    long long c[CT_NCOL] = {};
    c[CT_PAIRS] = (long long)sc.N * (sc.N - 1) / 2 * sc.T;
    add_counters(ws, s, c);
  }
}

template <int NX, int NU>
__global__ __launch_bounds__(64) void k_resid(Prob pb, WS ws, int s, int k, int *done_out) {
  const Scen sc = load_scen(ws, s);
  const int cap = ws.sst[(long long)s * ST_NCOL + ST_CAP];
  const int done = pb.mom ? scenario_test<NX, NU, true>(pb, ws, sc, k, threadIdx.x, cap)
                          : scenario_test<NX, NU>(pb, ws, sc, k, threadIdx.x, cap);
  if (threadIdx.x == 0) *done_out = done;
  if (!cap) commit_positions<NX, NU>(ws, sc, threadIdx.x, blockDim.x);
}

// Momentum: the next iteration's extrapolated duals and copies of a scenario
// whose stopping test did not end it (one lane per agent-stage).
template <int NX, int NU>
__global__ __launch_bounds__(256) void k_extrap(Prob pb, WS ws, int s) {
  if (uni(ws.sst[(long long)s * ST_NCOL + ST_DONE])) return;
  const Scen sc = load_scen(ws, s);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < sc.N * sc.T) mom_extrapolate<NX, NU>(pb, ws, sc, idx % sc.N, idx / sc.N + 1);
}

// ===========================================================================
// Kernel: batched persistent solve
// ===========================================================================
// Workgroups take scenarios from an atomic counter in the host-given order
// (largest estimated work first) and iterate ADMM on chip until the
// scenario's own stopping test passes; the three phases are separated by
// workgroup barriers.  Every wave reaches the queue read, so the grid drains
// once the counter passes S.
// VAR: 0 plain ADMM, 1 over-relaxed, 2 momentum (each a kernel of its own);
// 3 plain ADMM without the options (normals of the iterates, shared weights
// and boxes, fixed penalty, no state boxes, not a continuing SQP round): the
// option flags and pointers are constants here, so their code and registers
// drop out of the kernel, and with double-integrator dynamics the x-update
// keeps its per-pass slots (k, EQP input) in the LDS that the consensus step
// uses for the positions (the host sizes it for both, 2 T N NU floats).
template <int NX, int NU, bool DI, int VAR>
__device__ __forceinline__ void persistent_body(Prob pb, WS ws, int S, int lds_floats) {
  if constexpr (VAR == 3) {
    pb.sbox = 0; pb.pbox = 0; pb.adapt = 0; pb.relax = 0; pb.mom = 0; pb.cont = 0;
    pb.normal_mode = NORMAL_PER_ITER;
    ws.aq = nullptr; ws.ar = nullptr; ws.alo = nullptr; ws.ahi = nullptr; ws.aA = nullptr; ws.aB = nullptr;
    ws.normals = nullptr; ws.orx = nullptr; ws.mom = nullptr; ws.momst = nullptr;
  }
  extern __shared__ float lds_pos[];  // positions of the scenario and the previous ones, [t][i][c] each
  __shared__ int s_item;
  __shared__ int s_cap;
  __shared__ int s_done;
  __shared__ long long s_tc[CT_NCOL];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (;;) {
    if (tid == 0) s_item = atomicAdd(ws.queue, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= S) return;
    const int s = __builtin_amdgcn_readfirstlane(ws.order[item]);
    if (pb.cont && uni(ws.skip[s])) continue;   // converged in an earlier SQP round
    const Scen sc = load_scen(ws, s);
    scenario_setup<NX, NU, VAR == 2>(pb, ws, sc, tid, nt);
    if (tid == 0) { s_cap = 0; s_done = 0; }
    // each lane's x-update counters in registers (32 bits: one scenario's
    // counts fit), the workgroup's pair count and phase times in LDS, kept by
    // thread 0
    unsigned cnt[CT_NXU] = {};
    if (tid == 0)
      for (int q = 0; q < CT_NCOL; ++q) s_tc[q] = 0;
    __syncthreads();
    for (int k = 1; k <= pb.max_iter; ++k) {
      const unsigned long long c0 = wall_clock64();
      for (int l = tid; l < xupdate_lanes<NX, NU, DI>(sc.N); l += nt)
        if (local_xupdate<NX, NU, DI, VAR == 3 && DI>(pb, ws, sc, l, k, cnt, lds_pos)) atomicOr(&s_cap, 1);
      __syncthreads();
      const unsigned long long c1 = wall_clock64();
      const int cap = s_cap;
      if (!cap) {
        // stage every position of the scenario in LDS (the partner loop reads
        // them N-1 times each), then the consensus and dual updates
        const bool staged = 2 * sc.GS * NU <= lds_floats;
        float *lds_prev = lds_pos + sc.GS * NU;
        if (staged) {
          float *R = ws.fr + sc.fo;
          const unsigned GS = (unsigned)sc.GS;
          for (int idx = tid; idx < sc.GS; idx += nt)
#pragma unroll
            for (int c = 0; c < NU; ++c) {
              lds_pos[idx * NU + c] = fref(R, GS, (unsigned)idx, Fld<NX, NU>::X + c);
              lds_prev[idx * NU + c] = xpref<NX, NU>(R, GS, (unsigned)idx, c);
            }
          __syncthreads();
        }
        for (int idx = tid; idx < sc.N * sc.T; idx += nt) {
          if constexpr (VAR == 2)
            pair_agent_stage_mom<NX, NU>(pb, ws, sc, idx % sc.N, idx / sc.N + 1, staged ? lds_pos : nullptr);
          else
            pair_agent_stage_impl<NX, NU, VAR == 1, VAR == 3>(pb, ws, sc, idx % sc.N, idx / sc.N + 1,
                                                    staged ? lds_pos : nullptr, staged ? lds_prev : nullptr, 0);
        }
        if (tid == 0) s_tc[CT_PAIRS] += (long long)sc.N * (sc.N - 1) / 2 * sc.T;
        __syncthreads();
        if (staged) {
          // the positions of this step are in LDS already
          float *R = ws.fr + sc.fo;
          const unsigned GS = (unsigned)sc.GS;
          for (int idx = sc.N + tid; idx < sc.GS; idx += nt)
#pragma unroll
            for (int c = 0; c < NU; ++c) xpref<NX, NU>(R, GS, (unsigned)idx, c) = lds_pos[idx * NU + c];
        } else {
          commit_positions<NX, NU>(ws, sc, tid, nt);
        }
      }
      __syncthreads();
      const unsigned long long c2 = wall_clock64();
      if (tid < 64) {
        const int d = scenario_test<NX, NU, VAR == 2>(pb, ws, sc, k, tid, cap);
        if (tid == 0) s_done = d;
      }
      __syncthreads();
      if constexpr (VAR == 2) {
        // momentum: the next iteration's extrapolated duals and copies
        if (!s_done) {
          for (int idx = tid; idx < sc.N * sc.T; idx += nt)
            mom_extrapolate<NX, NU>(pb, ws, sc, idx % sc.N, idx / sc.N + 1);
          __syncthreads();
        }
      }
      if (tid == 0) {
        s_tc[CT_T_X] += (long long)(c1 - c0);
        s_tc[CT_T_PAIR] += (long long)(c2 - c1);
        s_tc[CT_T_TEST] += (long long)(wall_clock64() - c2);
      }
      if (s_done) break;
    }
    add_counters(ws, s, cnt);
    if (tid == 0) {
      long long c[CT_NCOL];
      for (int q = 0; q < CT_NCOL; ++q) c[q] = s_tc[q];
      add_counters(ws, s, c);
    }
    __syncthreads();
  }
}

// Two launch shapes of the same persistent loop: workgroups of 128-256
// threads (several waves share a scenario's consensus step), and one-wave
// workgroups held to at most 128 VGPRs so that four waves fit per SIMD and a
// whole batch of a few thousand scenarios is resident at once.  REL:
// over-relaxation, a kernel of its own so that the plain kernel's code and
// register allocation stay as they are.
template <int NX, int NU, bool DI, int VAR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_admm_persistent(Prob pb, WS ws, int S, int lds_floats) {
  persistent_body<NX, NU, DI, VAR>(pb, ws, S, lds_floats);
}

template <int NX, int NU, bool DI, int VAR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_admm_persistent_lean(
    Prob pb, WS ws, int S, int lds_floats) {
  persistent_body<NX, NU, DI, VAR>(pb, ws, S, lds_floats);
}

template <int NX, int NU, bool DI>
const void *persistent_kernel(bool lean, int var) {
  if (lean) return var == 3 ? (const void *)k_admm_persistent_lean<NX, NU, DI, 3>
                 : var == 2 ? (const void *)k_admm_persistent_lean<NX, NU, DI, 2>
                 : var == 1 ? (const void *)k_admm_persistent_lean<NX, NU, DI, 1>
                            : (const void *)k_admm_persistent_lean<NX, NU, DI, 0>;
  return var == 3 ? (const void *)k_admm_persistent<NX, NU, DI, 3>
         : var == 2 ? (const void *)k_admm_persistent<NX, NU, DI, 2>
         : var == 1 ? (const void *)k_admm_persistent<NX, NU, DI, 1>
                    : (const void *)k_admm_persistent<NX, NU, DI, 0>;
}

// The persistent kernel variant of a solve (VAR of persistent_body).
int persistent_variant(const Prob &pb, const WS &w) {
  if (pb.mom) return 2;
  if (pb.relax) return 1;
  const bool plain = !pb.sbox && !pb.pbox && !pb.adapt && !pb.cont && pb.normal_mode == NORMAL_PER_ITER &&
                     !w.aq && !w.ar && !w.alo && !w.ahi && !w.aA && !w.aB;
  return plain ? 3 : 0;
}

__global__ void k_fill_i32(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// ===========================================================================
// Kernels: one scenario spread over many workgroups (few, large scenarios)
// ===========================================================================
// The plain path's phases without its per-iteration host round trip: the
// scenario index and the iteration number live in device memory (wide[1],
// wide[0]) so that a captured graph of several iterations serves every
// scenario of the batch; once a scenario has stopped, the remaining kernels
// of the graph return at once.
template <int NX, int NU>
__global__ __launch_bounds__(256) void k_wide_setup(Prob pb, WS ws, int *wide) {
  const Scen sc = load_scen(ws, uni(wide[1]));
  if (pb.mom) scenario_setup<NX, NU, true>(pb, ws, sc, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
  else scenario_setup<NX, NU>(pb, ws, sc, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
  if (!pb.cont && blockIdx.x == 0 && threadIdx.x < CT_NCOL) ws.cnt[(long long)sc.s * CT_NCOL + threadIdx.x] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) wide[0] = 1;
}

template <int NX, int NU, bool DI>
__global__ __launch_bounds__(64) void k_wide_x(Prob pb, WS ws, const int *wide) {
  const int s = uni(wide[1]);
  int *st = ws.sst + (long long)s * ST_NCOL;
  if (uni(st[ST_DONE])) return;
  const Scen sc = load_scen(ws, s);
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= xupdate_lanes<NX, NU, DI>(sc.N)) return;
  unsigned cnt[CT_NXU] = {};
  if (local_xupdate<NX, NU, DI>(pb, ws, sc, l, uni(wide[0]), cnt)) atomicOr(st + ST_CAP, 1);
  add_counters(ws, s, cnt);
}

// one lane per agent-stage; a block stages the current and previous
// positions of the stages its agent-stages belong to (every partner of
// agent-stage (i, t) is at stage t)
template <int NX, int NU>
__global__ __launch_bounds__(256) void k_wide_pair(Prob pb, WS ws, const int *wide, int lds_floats) {
  extern __shared__ float lds_pos[];
  const int s = uni(wide[1]);
  const int *st = ws.sst + (long long)s * ST_NCOL;
  if (uni(st[ST_DONE]) | uni(st[ST_CAP])) return;
  const Scen sc = load_scen(ws, s);
  const int N = sc.N, NT = N * sc.T;
  const int idx0 = blockIdx.x * blockDim.x;
  if (idx0 >= NT) return;
  const int idx1 = min(NT, idx0 + (int)blockDim.x);
  const int g0 = (idx0 / N + 1) * N, g1 = ((idx1 - 1) / N + 2) * N;   // agent-stages of those stages
  const int ng = g1 - g0;
  const bool staged = 2 * ng * NU <= lds_floats;
  float *lds_prev = lds_pos + ng * NU;
  if (staged) {
    float *R = ws.fr + sc.fo;
    const unsigned GS = (unsigned)sc.GS;
    for (int e = threadIdx.x; e < ng; e += blockDim.x)
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        lds_pos[e * NU + c] = fref(R, GS, (unsigned)(g0 + e), Fld<NX, NU>::X + c);
        lds_prev[e * NU + c] = xpref<NX, NU>(R, GS, (unsigned)(g0 + e), c);
      }
    __syncthreads();
  }
  const int idx = idx0 + threadIdx.x;
  if (idx < idx1)
    pair_agent_stage<NX, NU>(pb, ws, sc, idx % N, idx / N + 1, staged ? lds_pos : nullptr,
                             staged ? lds_prev : nullptr, g0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    long long c[CT_NCOL] = {};
    c[CT_PAIRS] = (long long)N * (N - 1) / 2 * sc.T;
    add_counters(ws, s, c);
  }
}

// one wave per block of the stopping test's sums (kTestBlock agent-stages):
// the block's sums into ws.tpart, and the positions of the block's
// agent-stages committed as the previous ones
template <int NX, int NU>
__global__ __launch_bounds__(64) void k_wide_tpart(Prob pb, WS ws, const int *wide) {
  const int s = uni(wide[1]);
  const int *st = ws.sst + (long long)s * ST_NCOL;
  if (uni(st[ST_DONE])) return;
  const Scen sc = load_scen(ws, s);
  const int b = blockIdx.x, b0 = b * kTestBlock, lane = threadIdx.x;
  if (b0 >= sc.N * sc.T) return;
  float p[5];
  test_block<NX, NU>(ws, sc, b0, lane, p);
#pragma unroll
  for (int q = 0; q < 5; ++q) ws.tpart[(b * 5 + q) * 64 + lane] = p[q];
  if (!uni(st[ST_CAP])) {
    using F = Fld<NX, NU>;
    float *R = ws.fr + sc.fo;
    const unsigned GS = (unsigned)sc.GS;
    const int e = min(sc.N * sc.T, b0 + kTestBlock);
    constexpr int U = kTestBlock / 64;
    float xv[U][NU];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = b0 + lane + 64 * u;
      if (idx < e)
#pragma unroll
        for (int c = 0; c < NU; ++c) xv[u][c] = fref(R, GS, (unsigned)(sc.N + idx), F::X + c);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = b0 + lane + 64 * u;
      if (idx < e)
#pragma unroll
        for (int c = 0; c < NU; ++c) xpref<NX, NU>(R, GS, (unsigned)(sc.N + idx), c) = xv[u][c];
    }
  }
}

template <int NX, int NU>
__global__ __launch_bounds__(64) void k_wide_test(Prob pb, WS ws, const int *wide) {
  const int s = uni(wide[1]);
  const int *st = ws.sst + (long long)s * ST_NCOL;
  if (uni(st[ST_DONE])) return;
  const Scen sc = load_scen(ws, s);
  const int cap = uni(st[ST_CAP]);
  if (pb.mom) (void)scenario_test<NX, NU, true>(pb, ws, sc, uni(wide[0]), threadIdx.x, cap, ws.tpart);
  else (void)scenario_test<NX, NU>(pb, ws, sc, uni(wide[0]), threadIdx.x, cap, ws.tpart);
}

// Momentum in the many-workgroup mode: the extrapolation after the test.
template <int NX, int NU>
__global__ __launch_bounds__(256) void k_wide_extrap(Prob pb, WS ws, const int *wide) {
  const int s = uni(wide[1]);
  if (uni(ws.sst[(long long)s * ST_NCOL + ST_DONE])) return;
  const Scen sc = load_scen(ws, s);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < sc.N * sc.T) mom_extrapolate<NX, NU>(pb, ws, sc, idx % sc.N, idx / sc.N + 1);
}

__global__ void k_wide_next(int *wide) {
  if (blockIdx.x == 0 && threadIdx.x == 0) wide[0] += 1;
}

// ===========================================================================
// Input checks and output write-back
// ===========================================================================
template <int NX, int NU>
__global__ void k_check(Prob pb, WS ws, int S, int *flags) {
  for (int s = blockIdx.x; s < S; s += gridDim.x) {
    const Scen sc = load_scen(ws, s);
    const int N = sc.N, T = sc.T;
    int bad = 0, close = 0;
    for (int e = threadIdx.x; e < N * NX; e += blockDim.x) bad |= !isfinite(ws.x0[sc.ao * NX + e]);
    for (long long e = threadIdx.x; e < (long long)N * (T + 1) * NX; e += blockDim.x) bad |= !isfinite(ws.xref[sc.xo * NX + e]);
    if (threadIdx.x < NX) { const float q = ws.qd[(long long)s * NX + threadIdx.x]; bad |= !(isfinite(q) && q > 0.f); }
    if (threadIdx.x < NU) { const float r = ws.rd[(long long)s * NU + threadIdx.x]; bad |= !(isfinite(r) && r > 0.f); }
    if (ws.aq)
      for (int e = threadIdx.x; e < N * NX; e += blockDim.x) {
        const float q = ws.aq[sc.ao * NX + e];
        bad |= !(isfinite(q) && q > 0.f);
      }
    if (ws.ar)
      for (int e = threadIdx.x; e < N * NU; e += blockDim.x) {
        const float r = ws.ar[sc.ao * NU + e];
        bad |= !(isfinite(r) && r > 0.f);
      }
    if (ws.alo)
      for (int e = threadIdx.x; e < N * NU; e += blockDim.x) {
        const float l = ws.alo[sc.ao * NU + e], h = ws.ahi[sc.ao * NU + e];
        bad |= !(isfinite(l) && isfinite(h) && l < h);
      }
    if (ws.aA) {
      for (int e = threadIdx.x; e < N * NX * NX; e += blockDim.x) bad |= !isfinite(ws.aA[sc.ao * NX * NX + e]);
      for (int e = threadIdx.x; e < N * NX * NU; e += blockDim.x) bad |= !isfinite(ws.aB[sc.ao * NX * NU + e]);
    }
    if (ws.normals && pb.normal_mode == NORMAL_FROZEN)
      for (long long e = threadIdx.x; e < (long long)N * (N - 1) / 2 * T * NU; e += blockDim.x)
        bad |= !isfinite(ws.normals[sc.po * NU + e]);
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
      const int i = e / N, j = e % N;
      if (j <= i) continue;
      float d2 = 0.f;
#pragma unroll
      for (int c = 0; c < NU; ++c) {
        const float d = ws.x0[(sc.ao + i) * NX + c] - ws.x0[(sc.ao + j) * NX + c];
        d2 = fmaf(d, d, d2);
      }
      close |= (sqrtf(d2) < pb.dmin);
    }
    if (bad) atomicOr(flags + 0, 1);
    if (close) atomicOr(flags + 1, 1);
  }
}

// ===========================================================================
// SQP outer loop: the half-planes re-linearized about each round's solution
// ===========================================================================
// The separation constraints of Eq. 1 are convexified as half-planes with
// frozen normals (Sec. III-A); every round solves that QP with the ADMM, and
// the next one re-linearizes about its solution.  A scenario leaves the loop,
// as under the stopping rule of Sec. V-A, once the objective of Eq. 1 moved
// by at most rtol (relative) since the previous round and every pair is at
// least d_min - sep_tol apart at every step t = 1..T.

__device__ __forceinline__ float block_min_f(float v, float *red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float m = red[0];
  for (int w = 1; w < nw; ++w) m = fminf(m, red[w]);
  return m;
}

// Normals of the next round for the scenarios still in the loop: every pair
// (i < j) and step t, n = (p_i - p_j)/|p_i - p_j| at the current positions
// (the reference normal where they coincide), written to nrm in the layout
// of the caller's frozen normals, [pair-step po + p T + t - 1][NU].
template <int NX, int NU>
__global__ __launch_bounds__(256) void k_sqp_relin(WS ws, float *nrm, int S) {
  using F = Fld<NX, NU>;
  for (int s = blockIdx.x; s < S; s += gridDim.x) {
    if (uni(ws.skip[s])) continue;
    const Scen sc = load_scen(ws, s);
    const int N = sc.N, T = sc.T;
    const float *R = ws.fr + sc.fo;
    for (int e = threadIdx.x; e < N * T; e += blockDim.x) {
      const int t = e / N + 1, i = e % N;
      float pi[NU];
#pragma unroll
      for (int c = 0; c < NU; ++c) pi[c] = R[fidx((unsigned)sc.GS, (unsigned)(t * N + i), F::X + c)];
      const int base = i * N - i * (i + 1) / 2;   // pair index of (i, i + 1)
      for (int j = i + 1; j < N; ++j) {
        float d[NU], n[NU];
#pragma unroll
        for (int c = 0; c < NU; ++c) d[c] = pi[c] - R[fidx((unsigned)sc.GS, (unsigned)(t * N + j), F::X + c)];
        if (!unit_normal<NU>(d, n)) reference_normal<NX, NU>(ws, sc, i, j, t, n);
        float *o = nrm + (sc.po + (long long)(base + j - i - 1) * T + (t - 1)) * NU;
#pragma unroll
        for (int c = 0; c < NU; ++c) o[c] = n[c];
      }
    }
  }
}

// End of a round for the scenarios still in the loop: the objective of Eq. 1
// at the solution, sum_i sum_{t<T} ||x - r||_Q^2 + ||u||_R^2 + ||x_T - r_T||_{Q_T}^2
// (FP64, fixed-order sums), the smallest distance between two agents over
// t = 1..T, and the stopping rule.  jprev: objective of the previous round;
// rounds: rounds solved; *active: scenarios still in the loop.
template <int NX, int NU>
__global__ __launch_bounds__(256) void k_sqp_eval(Prob pb, WS ws, double *jprev, int *rounds, float *minsep, int S,
                                                  int round, float rtol, float sep_tol, int *active) {
  using F = Fld<NX, NU>;
  __shared__ double red[4];
  __shared__ float redf[4];
  for (int s = blockIdx.x; s < S; s += gridDim.x) {
    if (uni(ws.skip[s])) continue;
    const Scen sc = load_scen(ws, s);
    const int N = sc.N, T = sc.T;
    const unsigned GS = (unsigned)sc.GS;
    const float *R = ws.fr + sc.fo;
    double J = 0.0;
    for (int e = threadIdx.x; e < sc.GS; e += blockDim.x) {
      const int t = e / N, i = e % N;
      const float *r = ws.xref + (sc.xo + (long long)i * (T + 1) + t) * NX;
      const float *qd = ws.aq ? ws.aq + (sc.ao + i) * NX : ws.qd + (long long)s * NX;
      const float *rd = ws.ar ? ws.ar + (sc.ao + i) * NU : ws.rd + (long long)s * NU;
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        const double d = (double)R[fidx(GS, (unsigned)e, F::X + c)] - (double)r[c];
        v = fma((double)qd[c] * d, d, v);
      }
      if (t == T) {
        v *= (double)pb.qT;
      } else {
#pragma unroll
        for (int a = 0; a < NU; ++a) {
          const double u = (double)uref<NX, NU>(const_cast<float *>(R), GS, (unsigned)e, a);
          v = fma((double)rd[a] * u, u, v);
        }
      }
      J += v;
    }
    J = block_sum(J, red);
    float m2 = INFINITY;   // smallest squared distance
    for (int e = threadIdx.x; e < N * T; e += blockDim.x) {
      const int t = e / N + 1, i = e % N;
      float pi[NU];
#pragma unroll
      for (int c = 0; c < NU; ++c) pi[c] = R[fidx(GS, (unsigned)(t * N + i), F::X + c)];
      for (int j = i + 1; j < N; ++j) {
        float d2 = 0.f;
#pragma unroll
        for (int c = 0; c < NU; ++c) {
          const float d = pi[c] - R[fidx(GS, (unsigned)(t * N + j), F::X + c)];
          d2 = fmaf(d, d, d2);
        }
        m2 = fminf(m2, d2);
      }
    }
    m2 = block_min_f(m2, redf);
    if (threadIdx.x == 0) {
      const float sep = sqrtf(m2);
      const bool done = round >= 1 && fabs(J - jprev[s]) <= (double)rtol * fmax(fabs(J), 1e-300) &&
                        sep >= pb.dmin - sep_tol;
      int *sst = ws.sst + (long long)s * ST_NCOL;
      sst[ST_COLD] = sst[ST_STATUS] != SCEN_CONVERGED;   // for the next round's setup
      jprev[s] = J;
      rounds[s] = round + 1;
      minsep[s] = sep;
      ws.skip[s] = done ? 1 : 0;
      if (!done) atomicAdd(active, 1);
    }
    __syncthreads();
  }
}

// stats [S][4]: rounds solved, 1 if the stopping rule was met, the objective
// of the last round, its smallest distance between two agents
__global__ void k_sqp_stats(WS ws, const double *jprev, const int *rounds, const float *minsep, int S, float *stats) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
    stats[4 * s + 0] = (float)rounds[s];
    stats[4 * s + 1] = (float)ws.skip[s];
    stats[4 * s + 2] = (float)jprev[s];
    stats[4 * s + 3] = minsep[s];
  }
}

template <int NX, int NU>
__global__ void k_writeback(WS ws, int S, tadmm_out out) {
  using F = Fld<NX, NU>;
  for (int s = blockIdx.x; s < S; s += gridDim.x) {
    const Scen sc = load_scen(ws, s);
    const int N = sc.N, T = sc.T;
    const float *R = ws.fr + sc.fo;
    const int8_t *Wb = ws.wr + sc.bo;
    if (out.x)
      for (int e = threadIdx.x; e < N * (T + 1) * NX; e += blockDim.x) {
        const int c = e % NX, it = e / NX, t = it % (T + 1), i = it / (T + 1);
        out.x[sc.xo * NX + e] = R[fidx((unsigned)sc.GS, (unsigned)(t * N + i), F::X + c)];
      }
    if (out.u || out.w)
      for (int e = threadIdx.x; e < N * T * NU; e += blockDim.x) {
        const int c = e % NU, it = e / NU, t = it % T, i = it / T;
        if (out.u) out.u[sc.uo * NU + e] = uref<NX, NU>(const_cast<float *>(R), (unsigned)sc.GS, (unsigned)(t * N + i), c);
        if (out.w) out.w[sc.uo * NU + e] = Wb[(unsigned)(t * N + i) * 4u + c];
      }
    if (out.pair_active)
      for (int e = threadIdx.x; e < N * N * T; e += blockDim.x) {
        const int i = e % N, j = (e / N) % N, t = e / (N * N) + 1;
        if (j <= i) continue;
        const int p = i * N - i * (i + 1) / 2 + (j - i - 1);
        out.pair_active[sc.po + (long long)p * T + (t - 1)] = (uint8_t)(ws.gam[sc.lo + e] > 0.f);
      }
    if (threadIdx.x == 0) {
      const int *st = ws.sst + (long long)s * ST_NCOL;
      const float *sn = ws.snorm + (long long)s * SN_NCOL;
      if (out.status) out.status[s] = st[ST_STATUS];
      if (out.iters) out.iters[s] = st[ST_ITERS];
      if (out.r_norm) out.r_norm[s] = sn[SN_R];
      if (out.s_norm) out.s_norm[s] = sn[SN_S];
      if (out.eps_pri) out.eps_pri[s] = sn[SN_EPRI];
      if (out.eps_dual) out.eps_dual[s] = sn[SN_EDUAL];
    }
    if (out.counters && threadIdx.x < CT_NCOL)
      out.counters[(long long)s * CT_NCOL + threadIdx.x] = (int64_t)ws.cnt[(long long)s * CT_NCOL + threadIdx.x];
  }
}

}  // namespace tadmm

// ===========================================================================
// Host library
// ===========================================================================

// The workspace of tadmm_solve_noalloc(): a fixed device array, one per GPU
// (each device that loads the library holds its own copy until the process
// ends).  Host code never passes its name to a kernel: the name is a host-side
// stand-in, and the device address comes from hipGetSymbolAddress, resolved
// once per device when a context is created on it.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

using namespace tadmm;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device).
hipError_t scratch_address(int dev, void **ptr) {
  *ptr = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipSuccess;   // no static workspace on this device
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  int S = 0, nx = 0, nu = 0, NF = 0;
  long long A = 0, sumGS = 0, sumL = 0;
  size_t o_N = 0, o_T = 0, o_tab = 0, o_order = 0, o_queue = 0, o_sst = 0, o_snorm = 0, o_cnt = 0, o_flags = 0;
  size_t o_adirty = 0, o_fr = 0, o_dr = 0, o_wr = 0, o_gam = 0, bytes = 0;
  size_t o_er = 0, o_nrm = 0, o_cidx = 0, o_clist = 0, o_cg = 0, o_m = 0, o_coff = 0, o_cent = 0;
  size_t o_wide = 0;   // wide mode: iteration number, scenario index
  size_t o_tpart = 0;  // wide mode: block sums of the stopping test, [blocks][5][64]
  size_t o_sqpj = 0, o_sqpi = 0, o_sqpf = 0;   // SQP: objective [S] (FP64); skip, rounds [2][S]; min distance [S]
  size_t o_rho = 0;    // [S][2] penalty of the next / last iteration
  size_t o_orx = 0;    // over-relaxation: [2 nu] planes shaped like the gamma region
  size_t o_mom = 0, o_momst = 0;   // momentum: [6 nu] planes shaped like the gamma region; [S][4]
  long long sumPT = 0;
  std::vector<long long> tab;
  std::vector<int> order;
};

// over-relaxation requested (alpha = 0 reads as 1: plain ADMM)
bool relaxed(const tadmm_params &p) { return p.alpha != 0.f && p.alpha != 1.f; }

int fields_per_stage(int nx, int nu) {
  return (nx == 4) ? Fld<4, 2>::NF : Fld<6, 3>::NF;
  (void)nu;
}

int eqp_fields_per_stage(int nx) { return (nx == 4) ? EFld<4, 2>::NF : EFld<6, 3>::NF; }

const char *kStatusStr[] = {"ok", "invalid argument", "shape error", "non-finite input", "infeasible start",
                            "HIP runtime error", "workspace error", "state error"};

bool params_ok(const tadmm_params *p, std::string &err) {
  if (!p) { err = "params is NULL"; return false; }
  if (!((p->nx == 4 && p->nu == 2) || (p->nx == 6 && p->nu == 3))) { err = "nx/nu must be 4/2 or 6/3"; return false; }
  for (int k = 0; k < p->nx * p->nx; ++k) if (!std::isfinite(p->A[k])) { err = "A not finite"; return false; }
  for (int k = 0; k < p->nx * p->nu; ++k) if (!std::isfinite(p->B[k])) { err = "B not finite"; return false; }
  for (int c = 0; c < p->nu; ++c)
    if (!(std::isfinite(p->u_lo[c]) && std::isfinite(p->u_hi[c]) && p->u_lo[c] < p->u_hi[c])) {
      err = "need finite u_lo < u_hi"; return false;
    }
  if (!(std::isfinite(p->rho) && p->rho > 0.f)) { err = "rho must be > 0"; return false; }
  if (!(std::isfinite(p->qT_scale) && p->qT_scale > 0.f)) { err = "qT_scale must be > 0"; return false; }
  if (!(std::isfinite(p->d_min) && p->d_min >= 0.f)) { err = "d_min must be >= 0"; return false; }
  if (!(std::isfinite(p->eps_abs) && p->eps_abs >= 0.f && std::isfinite(p->eps_rel) && p->eps_rel >= 0.f)) {
    err = "eps_abs/eps_rel must be >= 0"; return false;
  }
  if (!(std::isfinite(p->mu_tol) && p->mu_tol >= 0.f)) { err = "mu_tol must be >= 0"; return false; }
  if (!(std::isfinite(p->refine_band) && p->refine_band >= 0.f)) { err = "refine_band must be >= 0"; return false; }
  if (p->adaptive_rho && !(std::isfinite(p->rho_mu) && p->rho_mu >= 1.f && std::isfinite(p->rho_tau) &&
                           p->rho_tau > 1.f && p->rho_every >= 1)) {
    err = "adaptive_rho needs rho_mu >= 1, rho_tau > 1 and rho_every >= 1"; return false;
  }
  if (p->state_box)
    for (int c = 0; c < p->nu; ++c) {
      if (std::isnan(p->s_lo[c]) || std::isnan(p->s_hi[c]) || !(p->s_lo[c] < p->s_hi[c])) {
        err = "state_box needs s_lo < s_hi (infinite ends allowed)"; return false;
      }
      if (std::isnan(p->p_lo[c]) || std::isnan(p->p_hi[c]) || !(p->p_lo[c] < p->p_hi[c])) {
        err = "state_box needs p_lo < p_hi (infinite ends allowed)"; return false;
      }
    }
  if (!(p->alpha >= 0.f && p->alpha < 2.f)) { err = "alpha must be in (0, 2) (0: plain ADMM)"; return false; }
  if (p->momentum) {
    if (!(p->mom_eta > 0.f && p->mom_eta < 1.f)) { err = "momentum needs 0 < mom_eta < 1"; return false; }
    if (p->adaptive_rho || relaxed(*p) || p->state_box) {
      err = "momentum is not combined with adaptive_rho, alpha != 1 or state_box"; return false;
    }
  }
  if (p->max_iter < 1) { err = "max_iter must be >= 1"; return false; }
  if (p->normal_mode != TADMM_NORMAL_PER_ITER && p->normal_mode != TADMM_NORMAL_FROZEN) {
    err = "unknown normal_mode"; return false;
  }
  if (p->block_threads != 0 && (p->block_threads < 64 || p->block_threads > 256 || p->block_threads % 64 != 0)) {
    err = "block_threads must be 0, 64, 128, 192 or 256"; return false;
  }
  return true;
}

bool make_layout(const tadmm_params *p, int S, const int32_t *N, const int32_t *T, Layout &L, std::string &err) {
  if (S < 0) { err = "n_scen < 0"; return false; }
  if (S > 0 && (!N || !T)) { err = "n_agents / horizon are NULL"; return false; }
  L = Layout();
  L.S = S; L.nx = p->nx; L.nu = p->nu; L.NF = fields_per_stage(p->nx, p->nu);
  L.tab.assign((size_t)S * TB_NCOL, 0);
  long long fo = 0, bo = 0, lo = 0, ao = 0, xo = 0, uo = 0, po = 0, dof = 0, max_nt = 1;
  for (int s = 0; s < S; ++s) {
    const long long n = N[s], t = T[s];
    max_nt = std::max(max_nt, n * t);
    if (n < 1 || t < 1) { err = "every scenario needs N >= 1 and T >= 1"; return false; }
    if (n > 4096 || t > 65536) { err = "scenario too large (N <= 4096, T <= 65536)"; return false; }
    const long long GS = n * (t + 1);
    if ((long long)L.NF * GS + axis_region_floats(GS, p->nu) + 2 * input_region_floats(GS, p->nu) >= (1ll << 31) ||
        (long long)p->nu * t * n * n >= (1ll << 31) ||
        (long long)p->nx * GS >= (1ll << 31)) {
      err = "scenario too large for 32-bit in-scenario offsets"; return false;
    }
    long long *tb = &L.tab[(size_t)s * TB_NCOL];
    tb[TB_F] = fo; tb[TB_B] = bo; tb[TB_L] = lo; tb[TB_A] = ao; tb[TB_XO] = xo; tb[TB_UO] = uo; tb[TB_PO] = po;
    tb[TB_D] = dof;
    fo += (long long)L.NF * GS + axis_region_floats(GS, p->nu) + 2 * input_region_floats(GS, p->nu);
    dof += (long long)p->nx * GS;
    bo += 4ll * GS;
    lo += t * n * n;
    ao += n;
    xo += GS;
    uo += n * t;
    po += n * (n - 1) / 2 * t;
  }
  L.A = ao; L.sumGS = xo; L.sumL = lo;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + std::max<size_t>(bytes, 1)); return o; };
  L.o_N = take(sizeof(int) * S);
  L.o_T = take(sizeof(int) * S);
  L.o_tab = take(sizeof(long long) * S * TB_NCOL);
  L.o_order = take(sizeof(int) * S);
  L.o_queue = take(sizeof(int) * 64);
  L.o_sst = take(sizeof(int) * S * ST_NCOL);
  L.o_snorm = take(sizeof(float) * S * SN_NCOL);
  L.o_cnt = take(sizeof(unsigned long long) * S * CT_NCOL);
  L.o_flags = take(sizeof(int) * 64);
  L.o_adirty = take(sizeof(int) * (size_t)ao * (size_t)p->nu);
  L.o_fr = take(sizeof(float) * (size_t)fo);
  L.o_dr = take(sizeof(double) * (size_t)dof);
  L.o_wr = take((size_t)bo);
  L.o_gam = take(sizeof(float) * (size_t)lo);
  // equality-QP solves of the derivative (sized for FP64)
  L.sumPT = po;
  L.o_er = take(sizeof(double) * (size_t)eqp_fields_per_stage(p->nx) * (size_t)xo);
  L.o_nrm = take(sizeof(float) * (size_t)p->nu * (size_t)po);
  L.o_cidx = take(sizeof(int) * (size_t)po);
  L.o_clist = take(sizeof(int2) * (size_t)po);
  L.o_coff = take(sizeof(int) * (size_t)xo);
  L.o_cent = take(sizeof(int2) * 2 * (size_t)po);
  L.o_cg = take(sizeof(double) * 6 * (size_t)po);
  L.o_m = take(sizeof(int) * S);
  L.o_wide = take(sizeof(int) * 64);
  L.o_tpart = take(sizeof(float) * 5 * 64 * (size_t)((max_nt + kTestBlock - 1) / kTestBlock));
  L.o_sqpj = take(sizeof(double) * S);
  L.o_sqpi = take(sizeof(int) * 2 * S);
  L.o_sqpf = take(sizeof(float) * S);
  L.o_rho = take(sizeof(float) * 2 * S);
  if (relaxed(*p)) L.o_orx = take(sizeof(float) * 2 * (size_t)p->nu * (size_t)lo);
  if (p->momentum) {
    L.o_mom = take(sizeof(float) * 6 * (size_t)p->nu * (size_t)lo);
    L.o_momst = take(sizeof(float) * 4 * (size_t)S);
  }
  L.bytes = off;
  // launch order for the persistent queue: largest N^2 T first (LPT)
  L.order.resize(S);
  std::iota(L.order.begin(), L.order.end(), 0);
  std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) {
    return (long long)N[a] * N[a] * T[a] > (long long)N[b] * N[b] * T[b];
  });
  return true;
}

// A = [[I, dt I], [0, I]] and B = [[h I], [dt I]] (positions first; h is
// the caller's value, dt^2/2 for the exact zero-order hold): the dynamics of
// every workload here; it selects the structured products (two FMAs per
// position instead of dense 4x4 / 6x6 products).
bool is_double_integrator(const tadmm_params &p);

bool is_double_integrator(const tadmm_params &p, const tadmm_batch *b) {
  if (b && (b->agent_A || b->agent_B)) return false;   // per-agent dynamics: the general path
  return is_double_integrator(p);
}

bool is_double_integrator(const tadmm_params &p) {
  const int nx = p.nx, nu = p.nu;
  const float dt = p.A[0 * nx + nu];
  const float h = p.B[0];
  for (int r = 0; r < nx; ++r)
    for (int c = 0; c < nx; ++c) {
      float want = (r == c) ? 1.f : 0.f;
      if (r < nu && c == r + nu) want = dt;
      if (p.A[r * nx + c] != want) return false;
    }
  for (int r = 0; r < nx; ++r)
    for (int a = 0; a < nu; ++a) {
      float want = 0.f;
      if (r == a) want = h;
      if (r == a + nu) want = dt;
      if (p.B[r * nu + a] != want) return false;
    }
  return dt != 0.f;
}

Prob to_prob(const tadmm_params &p) {
  Prob pb;
  std::memset(&pb, 0, sizeof(pb));
  std::memcpy(pb.A, p.A, sizeof(pb.A));
  std::memcpy(pb.B, p.B, sizeof(pb.B));
  pb.dt = p.A[0 * p.nx + p.nu];
  pb.h = p.B[0];
  for (int c = 0; c < 3; ++c) { pb.ulo[c] = p.u_lo[c]; pb.uhi[c] = p.u_hi[c]; }
  pb.qT = p.qT_scale; pb.dmin = p.d_min; pb.rho = p.rho; pb.eps_abs = p.eps_abs; pb.eps_rel = p.eps_rel;
  pb.mu_tol = p.mu_tol; pb.max_iter = p.max_iter; pb.max_as = p.max_as_iter; pb.normal_mode = p.normal_mode;
  pb.cache = p.cache_factors ? 1 : 0; pb.warm = p.riccati_warmstart ? 1 : 0; pb.hot = p.hotstart ? 1 : 0;
  pb.refine = p.refine ? 1 : 0;
  pb.refine_band = p.refine_band;
  pb.adapt = p.adaptive_rho ? 1 : 0;
  pb.rho_every = std::max(p.rho_every, 1);
  pb.rho_mu = p.rho_mu;
  pb.rho_tau = p.rho_tau;
  pb.mom = p.momentum ? 1 : 0;
  pb.mom_eta = p.mom_eta;
  pb.relax = relaxed(p) ? 1 : 0;
  pb.alpha = pb.relax ? p.alpha : 1.0f;
  // each group of states is split only where one of its bounds is finite
  auto bounded = [&](const float *lo, const float *hi) {
    for (int c = 0; c < p.nu; ++c)
      if (std::isfinite(lo[c]) || std::isfinite(hi[c])) return true;
    return false;
  };
  pb.sbox = (p.state_box && bounded(p.s_lo, p.s_hi)) ? 1 : 0;
  pb.pbox = (p.state_box && bounded(p.p_lo, p.p_hi)) ? 1 : 0;
  for (int c = 0; c < 3; ++c) { pb.plo[c] = p.p_lo[c]; pb.phi[c] = p.p_hi[c]; }
  pb.sigma = p.rho;
  for (int c = 0; c < 3; ++c) { pb.slo[c] = p.s_lo[c]; pb.shi[c] = p.s_hi[c]; }
  return pb;
}

struct GraphKey {
  const void *ws = nullptr;
  tadmm_out out{};
  const float *x0 = nullptr, *xref = nullptr, *qd = nullptr, *rd = nullptr, *normals = nullptr;
  const float *aq = nullptr, *ar = nullptr, *alo = nullptr, *ahi = nullptr, *aA = nullptr, *aB = nullptr;
  int S = 0, threads = 0, grid = 0;
  int variant = 0;   // 0: a solve; SQP rounds: 2 (first) or 3 (later, continuing)
  size_t bytes = 0;
  tadmm_params prm{};
  bool operator==(const GraphKey &o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

}  // namespace

struct tadmm_ctx {
  tadmm_params prm{};
  hipStream_t stream = nullptr;      // caller's stream: every launch is ordered on it
  hipStream_t cap_stream = nullptr;  // private stream used only to capture the graph
  int device = 0, n_cu = 256;
  std::string err;
  int tuned_threads = 128;
  void *h_stage = nullptr;
  size_t h_stage_bytes = 0;
  int *h_flags = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  GraphKey key{};
  // wide mode: a setup graph and a graph of kWideChunk iterations
  hipGraph_t wgraph[2] = {nullptr, nullptr};
  hipGraphExec_t wexec[2] = {nullptr, nullptr};
  GraphKey wkey{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  float last_ms = -1.f;
  void *scratch = nullptr;           // device address of this device's static workspace
  // derivative bookkeeping: the last successful solve and its polish
  bool solved = false, polished = false;
  const void *solved_ws = nullptr;
  size_t solved_bytes = 0;
  tadmm_batch solved_batch{};
  std::vector<int> solved_N, solved_T;
};

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ctx->err = std::string(#expr) + " failed: " + hipGetErrorString(e_);      \
      return TADMM_ERR_HIP;                                                       \
    }                                                                             \
  } while (0)

namespace {

tadmm_status fail(tadmm_ctx *ctx, tadmm_status s, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return s;
}

tadmm_status stage_tables(tadmm_ctx *ctx, const Layout &L, const int32_t *N, const int32_t *T, char *ws,
                          bool noalloc = false) {
  if (noalloc) {
    // straight from the caller's and the layout's host arrays (no staging
    // buffer); they outlive the solve, which synchronizes the stream
    HIPCHK(hipMemcpyAsync(ws + L.o_N, N, sizeof(int) * L.S, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ws + L.o_T, T, sizeof(int) * L.S, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ws + L.o_tab, L.tab.data(), sizeof(long long) * L.S * TB_NCOL, hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(ws + L.o_order, L.order.data(), sizeof(int) * L.S, hipMemcpyHostToDevice, ctx->stream));
    return TADMM_OK;
  }
  const size_t need = L.o_order + sizeof(int) * std::max(L.S, 1);
  if (ctx->h_stage_bytes < need) {
    if (ctx->h_stage) HIPCHK(hipHostFree(ctx->h_stage));
    ctx->h_stage = nullptr;
    HIPCHK(hipHostMalloc(&ctx->h_stage, need, hipHostMallocDefault));
    ctx->h_stage_bytes = need;
  }
  char *h = (char *)ctx->h_stage;
  std::memcpy(h + L.o_N, N, sizeof(int) * L.S);
  std::memcpy(h + L.o_T, T, sizeof(int) * L.S);
  std::memcpy(h + L.o_tab, L.tab.data(), sizeof(long long) * L.S * TB_NCOL);
  std::memcpy(h + L.o_order, L.order.data(), sizeof(int) * L.S);
  HIPCHK(hipMemcpyAsync(ws, h, need, hipMemcpyHostToDevice, ctx->stream));
  return TADMM_OK;
}

WS make_ws(const Layout &L, char *ws, const tadmm_batch *b) {
  WS w;
  w.N = (const int *)(ws + L.o_N);
  w.T = (const int *)(ws + L.o_T);
  w.tab = (const long long *)(ws + L.o_tab);
  w.order = (const int *)(ws + L.o_order);
  w.queue = (int *)(ws + L.o_queue);
  w.fr = (float *)(ws + L.o_fr);
  w.dr = (double *)(ws + L.o_dr);
  w.wr = (int8_t *)(ws + L.o_wr);
  w.adirty = (int *)(ws + L.o_adirty);
  w.gam = (float *)(ws + L.o_gam);
  w.sst = (int *)(ws + L.o_sst);
  w.snorm = (float *)(ws + L.o_snorm);
  w.cnt = (unsigned long long *)(ws + L.o_cnt);
  w.x0 = b->x0; w.xref = b->xref; w.qd = b->q_diag; w.rd = b->r_diag;
  w.normals = (b->normals && true) ? b->normals : nullptr;
  w.aq = b->agent_q; w.ar = b->agent_r; w.alo = b->agent_lo; w.ahi = b->agent_hi;
  w.aA = b->agent_A; w.aB = b->agent_B;
  w.skip = (int *)(ws + L.o_sqpi);
  w.rhos = (float *)(ws + L.o_rho);
  w.orx = L.o_orx ? (float *)(ws + L.o_orx) : nullptr;
  w.mom = L.o_mom ? (float *)(ws + L.o_mom) : nullptr;
  w.momst = L.o_momst ? (float *)(ws + L.o_momst) : nullptr;
  w.hist = nullptr;
  w.tpart = (float *)(ws + L.o_tpart);
  return w;
}

template <int NX, int NU>
tadmm_status run_checks(tadmm_ctx *ctx, const Prob &pb, const WS &w, int S, int *d_flags) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, ctx->stream, d_flags, 64, 0);
  hipLaunchKernelGGL((k_check<NX, NU>), dim3(std::min(S, 4096)), dim3(256), 0, ctx->stream, pb, w, S, d_flags);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(ctx->h_flags, d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->h_flags[0]) return fail(ctx, TADMM_ERR_NONFINITE, "non-finite input or non-positive weight");
  if (ctx->h_flags[1]) return fail(ctx, TADMM_ERR_INFEASIBLE_START, "two agents start closer than d_min");
  return TADMM_OK;
}

template <int NX, int NU, bool DI>
tadmm_status run_plain(tadmm_ctx *ctx, const Prob &pb, const WS &w, const Layout &L, const int32_t *N,
                       const int32_t *T, int *d_flags, const tadmm_out &out, const int *skip = nullptr) {
  HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
  for (int s = 0; s < L.S; ++s) {
    if (skip && skip[s]) continue;
    const int n = N[s], t = T[s];
    const long long work = std::max<long long>((long long)n * (t + 1), (long long)t * n * n);
    const int gsetup = (int)std::min<long long>((work + 255) / 256, 4096);
    hipLaunchKernelGGL((k_setup<NX, NU>), dim3(gsetup), dim3(256), 0, ctx->stream, pb, w, s);
    for (int k = 1; k <= pb.max_iter; ++k) {
      hipLaunchKernelGGL((k_xupdate<NX, NU, DI>), dim3((xupdate_lanes<NX, NU, DI>(n) + 63) / 64), dim3(64), 0,
                         ctx->stream, pb, w, s, k);
      hipLaunchKernelGGL((k_pair<NX, NU>), dim3((n * t + 255) / 256), dim3(256), 0, ctx->stream, pb, w, s);
      hipLaunchKernelGGL((k_resid<NX, NU>), dim3(1), dim3(64), 0, ctx->stream, pb, w, s, k, d_flags + 2);
      if (pb.mom)
        hipLaunchKernelGGL((k_extrap<NX, NU>), dim3((n * t + 255) / 256), dim3(256), 0, ctx->stream, pb, w, s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(ctx->h_flags + 2, d_flags + 2, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (ctx->h_flags[2]) break;
    }
  }
  hipLaunchKernelGGL((k_writeback<NX, NU>), dim3(std::min(L.S, 4096)), dim3(256), 0, ctx->stream, w, L.S, out);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1));
  return TADMM_OK;
}

template <int NX, int NU, bool DI>
tadmm_status run_batched(tadmm_ctx *ctx, const Prob &pb, const WS &w, const Layout &L, const tadmm_batch *b,
                         const tadmm_out &out, void *ws, size_t bytes, int variant = 0, bool direct = false) {
  const int threads = ctx->prm.block_threads ? ctx->prm.block_threads : ctx->tuned_threads;
  // LDS for the positions of the largest scenario, up to 32 KB per workgroup
  // (larger scenarios read positions from global memory)
  long long max_gs = 0, max_tn = 0;
  for (int s = 0; s < L.S; ++s) {
    max_gs = std::max<long long>(max_gs, (long long)b->n_agents[s] * (b->horizon[s] + 1));
    max_tn = std::max<long long>(max_tn, (long long)b->n_agents[s] * b->horizon[s]);
  }
  const bool lean = (threads == 64);
  const long long cap_floats = lean ? 4096 : 8192;
  int var = persistent_variant(pb, w);
  // variant 3 keeps the x-update's slots of every scenario in LDS and a
  // 64-bit partner mask per agent-stage
  long long max_n = 0;
  for (int s = 0; s < L.S; ++s) max_n = std::max<long long>(max_n, b->n_agents[s]);
  if (var == 3 && ((DI && 2 * max_tn * NU > cap_floats) || max_n > 64)) var = 0;
  const long long want = std::max<long long>(2 * max_gs * NU, (var == 3 && DI) ? 2 * max_tn * NU : 0);
  const int lds_floats = (int)std::min<long long>(want, cap_floats);
  const size_t lds_bytes = sizeof(float) * (size_t)lds_floats;
  const void *kfn = persistent_kernel<NX, NU, DI>(lean, var);
  int per_cu = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, threads, lds_bytes));
  if (per_cu < 1) return fail(ctx, TADMM_ERR_HIP, "persistent kernel does not fit on a compute unit");
  const int grid = std::max(1, std::min(L.S, per_cu * ctx->n_cu));
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.ws = ws; key.out = out; key.x0 = b->x0; key.xref = b->xref; key.qd = b->q_diag; key.rd = b->r_diag;
  key.normals = w.normals; key.S = L.S; key.threads = threads; key.grid = grid; key.bytes = bytes; key.prm = ctx->prm;
  key.aq = w.aq; key.ar = w.ar; key.alo = w.alo; key.ahi = w.ahi; key.aA = w.aA; key.aB = w.aB;
  key.variant = variant;
  // the launches of one solve: counters and the queue are cleared by fill
  // kernels (no memset nodes), then the persistent kernel and the write-back
  auto launch = [&](hipStream_t cs) -> hipError_t {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, cs, w.queue, 1, 0);
    const long long nc = (long long)L.S * CT_NCOL;
    if (!pb.cont)   // a continuing SQP round keeps counting
      hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, cs, w.cnt, nc);
    Prob kpb = pb;
    WS kw = w;
    int kS = L.S, klds = lds_floats;
    void *args[] = {&kpb, &kw, &kS, &klds};
    const hipError_t lk = hipLaunchKernel(kfn, dim3(grid), dim3(threads), args, lds_bytes, cs);
    hipLaunchKernelGGL((k_writeback<NX, NU>), dim3(std::min(L.S, 4096)), dim3(256), 0, cs, w, L.S, out);
    const hipError_t le = hipGetLastError();
    return le != hipSuccess ? le : lk;
  };
  if (direct) {
    // no graph (its instantiation may allocate): the launches straight on the
    // caller's stream
    HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
    HIPCHK(launch(ctx->stream));
    HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1));
    return TADMM_OK;
  }
  if (!(ctx->gexec && key == ctx->key)) {
    if (ctx->gexec) { (void)hipGraphExecDestroy(ctx->gexec); ctx->gexec = nullptr; }
    if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
    // Captured on the context's private stream (the caller's stream may be the
    // legacy default stream, which cannot be captured); launched on the
    // caller's stream below.
    hipStream_t cs = ctx->cap_stream;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const hipError_t le = launch(cs);
    hipError_t ce = hipStreamEndCapture(cs, &ctx->graph);
    if (le != hipSuccess || ce != hipSuccess) {
      ctx->err = std::string("graph capture failed: ") + hipGetErrorString(le != hipSuccess ? le : ce);
      return TADMM_ERR_HIP;
    }
    HIPCHK(hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
    ctx->key = key;
  }
  HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
  HIPCHK(hipGraphLaunch(ctx->gexec, ctx->stream));
  HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1));
  return TADMM_OK;
}

constexpr int kWideChunk = 8;   // ADMM iterations per launch of the wide-mode graph

// One scenario at a time, every phase over many workgroups
// (TADMM_MODE_WIDE): per scenario a setup graph, then a graph of kWideChunk
// iterations launched until the scenario has stopped (its done flag read back
// once per launch).
template <int NX, int NU, bool DI>
tadmm_status run_wide(tadmm_ctx *ctx, const Prob &pb, const WS &w, const Layout &L, const tadmm_batch *b,
                      const tadmm_out &out, void *ws, size_t bytes, int variant = 0, const int *skip = nullptr) {
  char *w8 = (char *)ws;
  int *d_wide = (int *)(w8 + L.o_wide);
  long long max_n = 1, max_nt = 1, max_work = 1;
  for (int s = 0; s < L.S; ++s) {
    const long long n = b->n_agents[s], t = b->horizon[s];
    max_n = std::max(max_n, n);
    max_nt = std::max(max_nt, n * t);
    max_work = std::max(max_work, std::max(n * (t + 1), t * n * n));
  }
  const int gx = (int)((xupdate_lanes<NX, NU, DI>((int)max_n) + 63) / 64), gp = (int)((max_nt + 255) / 256);
  const int gt = (int)((max_nt + kTestBlock - 1) / kTestBlock);   // blocks of the stopping test's sums
  const int gsetup = (int)std::min<long long>((max_work + 255) / 256, 4096);
  // LDS of a pair block: the stages of 256 agent-stages, current and previous positions
  long long max_ng = 0;
  for (int s = 0; s < L.S; ++s) {
    const long long n = b->n_agents[s];
    max_ng = std::max(max_ng, (256 / n + 2) * n);
  }
  const int lds_floats = (int)std::min<long long>(2 * max_ng * NU, 8192);
  const size_t lds_bytes = sizeof(float) * (size_t)lds_floats;
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.ws = ws; key.out = out; key.x0 = b->x0; key.xref = b->xref; key.qd = b->q_diag; key.rd = b->r_diag;
  key.normals = w.normals; key.S = L.S; key.threads = gp; key.grid = gx; key.bytes = bytes; key.prm = ctx->prm;
  key.aq = w.aq; key.ar = w.ar; key.alo = w.alo; key.ahi = w.ahi; key.aA = w.aA; key.aB = w.aB;
  key.variant = variant;
  if (!(ctx->wexec[0] && key == ctx->wkey)) {
    for (int q = 0; q < 2; ++q) {
      if (ctx->wexec[q]) { (void)hipGraphExecDestroy(ctx->wexec[q]); ctx->wexec[q] = nullptr; }
      if (ctx->wgraph[q]) { (void)hipGraphDestroy(ctx->wgraph[q]); ctx->wgraph[q] = nullptr; }
    }
    hipStream_t cs = ctx->cap_stream;
    for (int q = 0; q < 2; ++q) {
      HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      if (q == 0) {
        hipLaunchKernelGGL((k_wide_setup<NX, NU>), dim3(gsetup), dim3(256), 0, cs, pb, w, d_wide);
      } else {
        for (int it = 0; it < kWideChunk; ++it) {
          hipLaunchKernelGGL((k_wide_x<NX, NU, DI>), dim3(gx), dim3(64), 0, cs, pb, w, (const int *)d_wide);
          hipLaunchKernelGGL((k_wide_pair<NX, NU>), dim3(gp), dim3(256), lds_bytes, cs, pb, w, (const int *)d_wide,
                             lds_floats);
          hipLaunchKernelGGL((k_wide_tpart<NX, NU>), dim3(gt), dim3(64), 0, cs, pb, w, (const int *)d_wide);
          hipLaunchKernelGGL((k_wide_test<NX, NU>), dim3(1), dim3(64), 0, cs, pb, w, (const int *)d_wide);
          if (pb.mom)
            hipLaunchKernelGGL((k_wide_extrap<NX, NU>), dim3(gp), dim3(256), 0, cs, pb, w, (const int *)d_wide);
          hipLaunchKernelGGL(k_wide_next, dim3(1), dim3(64), 0, cs, d_wide);
        }
      }
      hipError_t le = hipGetLastError();
      hipError_t ce = hipStreamEndCapture(cs, &ctx->wgraph[q]);
      if (le != hipSuccess || ce != hipSuccess) {
        ctx->err = std::string("graph capture failed: ") + hipGetErrorString(le != hipSuccess ? le : ce);
        return TADMM_ERR_HIP;
      }
      HIPCHK(hipGraphInstantiate(&ctx->wexec[q], ctx->wgraph[q], nullptr, nullptr, 0));
    }
    ctx->wkey = key;
  }
  HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
  for (int s = 0; s < L.S; ++s) {
    if (skip && skip[s]) continue;
    ctx->h_flags[8] = s;
    HIPCHK(hipMemcpyAsync(d_wide + 1, ctx->h_flags + 8, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipGraphLaunch(ctx->wexec[0], ctx->stream));
    for (int done_iters = 0; done_iters < pb.max_iter; done_iters += kWideChunk) {
      HIPCHK(hipGraphLaunch(ctx->wexec[1], ctx->stream));
      HIPCHK(hipMemcpyAsync(ctx->h_flags + 9, w.sst + (long long)s * ST_NCOL + ST_DONE, sizeof(int),
                            hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      if (ctx->h_flags[9]) break;
    }
  }
  hipLaunchKernelGGL((k_writeback<NX, NU>), dim3(std::min(L.S, 4096)), dim3(256), 0, ctx->stream, w, L.S, out);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1));
  return TADMM_OK;
}

// noalloc: the workspace is the device's static array (ws, bytes), the
// tables go straight from host arrays, the batched mode launches without a
// graph and the wide mode (graphs) is not offered.
template <int NX, int NU, bool DI>
tadmm_status solve_impl(tadmm_ctx *ctx, const tadmm_batch *b, const tadmm_out *out, void *ws, size_t bytes, int mode,
                        bool noalloc = false) {
  Layout L;
  if (!make_layout(&ctx->prm, b->n_scen, b->n_agents, b->horizon, L, ctx->err)) return TADMM_ERR_SHAPE;
  if (noalloc && mode != TADMM_MODE_PLAIN && mode != TADMM_MODE_BATCHED)
    return fail(ctx, TADMM_ERR_INVALID_ARG, "tadmm_solve_noalloc takes TADMM_MODE_PLAIN or TADMM_MODE_BATCHED");
  if (noalloc && !ws) return fail(ctx, TADMM_ERR_WORKSPACE, "no static workspace on this device");
  if (noalloc && L.bytes > bytes)
    return fail(ctx, TADMM_ERR_WORKSPACE, "batch needs " + std::to_string(L.bytes) +
                                              " bytes of workspace; the static workspace of tadmm_solve_noalloc holds " +
                                              std::to_string(bytes));
  if (!ws || bytes < L.bytes) return fail(ctx, TADMM_ERR_WORKSPACE, "workspace missing or smaller than tadmm_workspace_size()");
  if (((uintptr_t)ws) % kAlign) return fail(ctx, TADMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  ctx->solved = false;
  ctx->polished = false;
  if (L.S == 0) return TADMM_OK;
  if (!b->x0 || !b->xref || !b->q_diag || !b->r_diag) return fail(ctx, TADMM_ERR_INVALID_ARG, "batch input pointer is NULL");
  if (!out->status || !out->iters) return fail(ctx, TADMM_ERR_INVALID_ARG, "out.status and out.iters are required");
  if (!b->agent_lo != !b->agent_hi) return fail(ctx, TADMM_ERR_INVALID_ARG, "agent_lo and agent_hi: both or neither");
  if (!b->agent_A != !b->agent_B) return fail(ctx, TADMM_ERR_INVALID_ARG, "agent_A and agent_B: both or neither");
  char *w8 = (char *)ws;
  tadmm_status st = stage_tables(ctx, L, b->n_agents, b->horizon, w8, noalloc);
  if (st != TADMM_OK) return st;
  const Prob pb = to_prob(ctx->prm);
  WS w = make_ws(L, w8, b);
  w.hist = out->hist;
  int *d_flags = (int *)(w8 + L.o_flags);
  if (ctx->prm.check_inputs) {
    st = run_checks<NX, NU>(ctx, pb, w, L.S, d_flags);
    if (st != TADMM_OK) return st;
  }
  if (mode == TADMM_MODE_PLAIN) st = run_plain<NX, NU, DI>(ctx, pb, w, L, b->n_agents, b->horizon, d_flags, *out);
  else if (mode == TADMM_MODE_BATCHED) st = run_batched<NX, NU, DI>(ctx, pb, w, L, b, *out, ws, bytes, 0, noalloc);
  else if (mode == TADMM_MODE_WIDE) st = run_wide<NX, NU, DI>(ctx, pb, w, L, b, *out, ws, bytes);
  else return fail(ctx, TADMM_ERR_INVALID_ARG, "unknown mode");
  if (st != TADMM_OK) return st;
  if (noalloc) return TADMM_OK;   // the derivative needs a caller-owned workspace
  ctx->solved = true;
  ctx->solved_ws = ws;
  ctx->solved_bytes = bytes;
  ctx->solved_batch = *b;
  ctx->solved_N.assign(b->n_agents, b->n_agents + L.S);
  ctx->solved_T.assign(b->horizon, b->horizon + L.S);
  return TADMM_OK;
}

// The SQP loop (k_sqp_*): rounds of frozen-normal solves in the given mode.
// Round 0 takes the batch's normals (or the references'); each later round
// re-linearizes about the previous solution and continues from the
// workspace's state (iterate, duals, working sets, factors) for the
// scenarios still in the loop.
template <int NX, int NU, bool DI>
tadmm_status sqp_impl(tadmm_ctx *ctx, const tadmm_batch *b, const tadmm_out *out, void *ws, size_t bytes, int mode,
                      int max_rounds, float rtol, float sep_tol, float *stats) {
  if (ctx->prm.momentum) return fail(ctx, TADMM_ERR_INVALID_ARG, "tadmm_sqp takes solves without momentum");
  if (max_rounds < 1) return fail(ctx, TADMM_ERR_INVALID_ARG, "max_rounds must be >= 1");
  if (!(std::isfinite(rtol) && rtol >= 0.f && std::isfinite(sep_tol) && sep_tol >= 0.f))
    return fail(ctx, TADMM_ERR_INVALID_ARG, "rtol and sep_tol must be finite and >= 0");
  if (mode != TADMM_MODE_PLAIN && mode != TADMM_MODE_BATCHED && mode != TADMM_MODE_WIDE)
    return fail(ctx, TADMM_ERR_INVALID_ARG, "unknown mode");
  Layout L;
  if (!make_layout(&ctx->prm, b->n_scen, b->n_agents, b->horizon, L, ctx->err)) return TADMM_ERR_SHAPE;
  if (!ws || bytes < L.bytes) return fail(ctx, TADMM_ERR_WORKSPACE, "workspace missing or smaller than tadmm_workspace_size()");
  if (((uintptr_t)ws) % kAlign) return fail(ctx, TADMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  ctx->solved = false;   // the derivative is defined for tadmm_solve results only
  ctx->polished = false;
  if (L.S == 0) return TADMM_OK;
  if (!b->x0 || !b->xref || !b->q_diag || !b->r_diag) return fail(ctx, TADMM_ERR_INVALID_ARG, "batch input pointer is NULL");
  if (!out->status || !out->iters) return fail(ctx, TADMM_ERR_INVALID_ARG, "out.status and out.iters are required");
  if (!b->agent_lo != !b->agent_hi) return fail(ctx, TADMM_ERR_INVALID_ARG, "agent_lo and agent_hi: both or neither");
  if (!b->agent_A != !b->agent_B) return fail(ctx, TADMM_ERR_INVALID_ARG, "agent_A and agent_B: both or neither");
  char *w8 = (char *)ws;
  tadmm_status st = stage_tables(ctx, L, b->n_agents, b->horizon, w8);
  if (st != TADMM_OK) return st;
  Prob pb = to_prob(ctx->prm);
  pb.normal_mode = TADMM_NORMAL_FROZEN;
  WS w = make_ws(L, w8, b);
  w.hist = out->hist;
  int *d_flags = (int *)(w8 + L.o_flags);
  if (ctx->prm.check_inputs) {
    st = run_checks<NX, NU>(ctx, pb, w, L.S, d_flags);
    if (st != TADMM_OK) return st;
  }
  double *jprev = (double *)(w8 + L.o_sqpj);
  int *rounds = w.skip + L.S;
  float *minsep = (float *)(w8 + L.o_sqpf);
  float *nrm = (float *)(w8 + L.o_nrm);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((2 * L.S + 255) / 256)), dim3(256), 0, ctx->stream, w.skip, 2 * L.S, 0);
  HIPCHK(hipGetLastError());
  std::vector<int> hskip(L.S, 0);
  const int grid = std::min(L.S, 65535);
  float total_ms = 0.f;
  for (int r = 0; r < max_rounds; ++r) {
    Prob pr = pb;
    pr.cont = r > 0 ? 1 : 0;
    WS wr = w;
    if (r > 0) {
      wr.normals = nrm;
      hipLaunchKernelGGL((k_sqp_relin<NX, NU>), dim3(grid), dim3(256), 0, ctx->stream, wr, nrm, L.S);
      HIPCHK(hipGetLastError());
    }
    const int variant = 2 + pr.cont;
    if (mode == TADMM_MODE_PLAIN)
      st = run_plain<NX, NU, DI>(ctx, pr, wr, L, b->n_agents, b->horizon, d_flags, *out, hskip.data());
    else if (mode == TADMM_MODE_BATCHED)
      st = run_batched<NX, NU, DI>(ctx, pr, wr, L, b, *out, ws, bytes, variant);
    else
      st = run_wide<NX, NU, DI>(ctx, pr, wr, L, b, *out, ws, bytes, variant, hskip.data());
    if (st != TADMM_OK) return st;
    total_ms += ctx->last_ms;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, ctx->stream, d_flags + 3, 1, 0);
    hipLaunchKernelGGL((k_sqp_eval<NX, NU>), dim3(grid), dim3(256), 0, ctx->stream, pr, wr, jprev, rounds, minsep, L.S,
                       r, rtol, sep_tol, d_flags + 3);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ctx->h_flags + 3, d_flags + 3, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(hskip.data(), w.skip, sizeof(int) * L.S, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->h_flags[3] == 0) break;
  }
  if (stats) {
    hipLaunchKernelGGL(k_sqp_stats, dim3((unsigned)((L.S + 255) / 256)), dim3(256), 0, ctx->stream, w, jprev, rounds,
                       minsep, L.S, stats);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  ctx->last_ms = total_ms;
  return TADMM_OK;
}

tadmm_status sqp_dispatch(tadmm_ctx *ctx, const tadmm_batch *b, const tadmm_out *out, void *ws, size_t bytes, int mode,
                          int max_rounds, float rtol, float sep_tol, float *stats) {
  const bool di = is_double_integrator(ctx->prm, b);
  if (ctx->prm.nx == 4)
    return di ? sqp_impl<4, 2, true>(ctx, b, out, ws, bytes, mode, max_rounds, rtol, sep_tol, stats)
              : sqp_impl<4, 2, false>(ctx, b, out, ws, bytes, mode, max_rounds, rtol, sep_tol, stats);
  return di ? sqp_impl<6, 3, true>(ctx, b, out, ws, bytes, mode, max_rounds, rtol, sep_tol, stats)
            : sqp_impl<6, 3, false>(ctx, b, out, ws, bytes, mode, max_rounds, rtol, sep_tol, stats);
}

EWS make_ews(const Layout &L, char *ws) {
  EWS e;
  e.er = (void *)(ws + L.o_er);
  e.nrm = (float *)(ws + L.o_nrm);
  e.cidx = (int *)(ws + L.o_cidx);
  e.clist = (int2 *)(ws + L.o_clist);
  e.coff = (int *)(ws + L.o_coff);
  e.cent = (int2 *)(ws + L.o_cent);
  e.cg = (double *)(ws + L.o_cg);
  e.m = (int *)(ws + L.o_m);
  return e;
}

// Polish (mode EQ_POLISH) or adjoint (EQ_ADJOINT) of the last solve.
template <int NX, int NU, bool DI>
tadmm_status eqp_impl(tadmm_ctx *ctx, const tadmm_batch *b, const tadmm_out *out, void *ws, size_t bytes, int mode,
                      const EqpIO &io) {
  if (!ctx->solved || ctx->solved_ws != ws || ctx->solved_bytes != bytes)
    return fail(ctx, TADMM_ERR_STATE, "needs a successful tadmm_solve with this workspace first");
  const tadmm_batch &sb = ctx->solved_batch;
  if (b->agent_q || b->agent_r || b->agent_lo || b->agent_hi || b->agent_A || b->agent_B)
    return fail(ctx, TADMM_ERR_INVALID_ARG, "the derivative takes per-scenario weights (no agent_* arrays)");
  if (ctx->prm.state_box)
    return fail(ctx, TADMM_ERR_INVALID_ARG, "the derivative covers input bounds only (no state_box)");
  if (b->n_scen != sb.n_scen || b->x0 != sb.x0 || b->xref != sb.xref || b->q_diag != sb.q_diag ||
      b->r_diag != sb.r_diag || b->normals != sb.normals)
    return fail(ctx, TADMM_ERR_STATE, "batch differs from the one of the last tadmm_solve");
  for (int s = 0; s < b->n_scen; ++s)
    if (b->n_agents[s] != ctx->solved_N[s] || b->horizon[s] != ctx->solved_T[s])
      return fail(ctx, TADMM_ERR_STATE, "batch shape differs from the one of the last tadmm_solve");
  if (mode == EQ_POLISH && ctx->polished) return fail(ctx, TADMM_ERR_STATE, "this solve is already polished");
  if (mode == EQ_ADJOINT && !ctx->polished) return fail(ctx, TADMM_ERR_STATE, "call tadmm_polish before tadmm_adjoint");
  Layout L;
  if (!make_layout(&ctx->prm, b->n_scen, b->n_agents, b->horizon, L, ctx->err)) return TADMM_ERR_SHAPE;
  if (L.S == 0) {
    if (mode == EQ_POLISH) ctx->polished = true;
    return TADMM_OK;
  }
  char *w8 = (char *)ws;
  const Prob pb = to_prob(ctx->prm);
  const WS w = make_ws(L, w8, b);
  const EWS ew = make_ews(L, w8);
  const int grid = std::min(L.S, 65535);
  const int max_cg = 4000;
  int max_lanes = 0;
  for (int s = 0; s < L.S; ++s) max_lanes = std::max(max_lanes, xupdate_lanes<NX, NU, DI>(b->n_agents[s]));
  HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
  if (ctx->prm.eqp_fp64 && max_lanes > 256)
    hipLaunchKernelGGL((k_eqp<NX, NU, DI, double, 512>), dim3(grid), dim3(512), 0, ctx->stream, pb, w, ew, io, L.S,
                       mode, max_cg, 1e-12);
  else if (ctx->prm.eqp_fp64)
    hipLaunchKernelGGL((k_eqp<NX, NU, DI, double>), dim3(grid), dim3(256), 0, ctx->stream, pb, w, ew, io, L.S, mode,
                       max_cg, 1e-12);
  else if (max_lanes > 256)
    hipLaunchKernelGGL((k_eqp<NX, NU, DI, float, 512>), dim3(grid), dim3(512), 0, ctx->stream, pb, w, ew, io, L.S,
                       mode, max_cg, 1e-7);
  else
    hipLaunchKernelGGL((k_eqp<NX, NU, DI, float>), dim3(grid), dim3(256), 0, ctx->stream, pb, w, ew, io, L.S, mode,
                       max_cg, 1e-7);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipEventElapsedTime(&ctx->last_ms, ctx->ev0, ctx->ev1));
  if (mode == EQ_POLISH) ctx->polished = true;
  (void)out;
  return TADMM_OK;
}

tadmm_status eqp_dispatch(tadmm_ctx *ctx, const tadmm_batch *b, const tadmm_out *out, void *ws, size_t bytes, int mode,
                          const EqpIO &io) {
  const bool di = is_double_integrator(ctx->prm, b);
  if (ctx->prm.nx == 4)
    return di ? eqp_impl<4, 2, true>(ctx, b, out, ws, bytes, mode, io) : eqp_impl<4, 2, false>(ctx, b, out, ws, bytes, mode, io);
  return di ? eqp_impl<6, 3, true>(ctx, b, out, ws, bytes, mode, io) : eqp_impl<6, 3, false>(ctx, b, out, ws, bytes, mode, io);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *tadmm_version(void) { return "turboadmm-gfx950 0.1"; }

const char *tadmm_status_string(tadmm_status s) {
  const int k = (int)s;
  return (k >= 0 && k <= 7) ? kStatusStr[k] : "unknown status";
}

const char *tadmm_last_error(const tadmm_ctx *ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

float tadmm_last_kernel_ms(const tadmm_ctx *ctx) { return ctx ? ctx->last_ms : -1.f; }

tadmm_status tadmm_workspace_size(const tadmm_params *params, int32_t n_scen, const int32_t *n_agents,
                                  const int32_t *horizon, size_t *bytes) {
  std::string err;
  if (!bytes) return TADMM_ERR_INVALID_ARG;
  if (!params_ok(params, err)) return TADMM_ERR_INVALID_ARG;
  Layout L;
  if (!make_layout(params, n_scen, n_agents, horizon, L, err)) return TADMM_ERR_SHAPE;
  *bytes = L.bytes;
  return TADMM_OK;
}

tadmm_status tadmm_create(tadmm_ctx **pctx, const tadmm_params *params, void *stream) {
  if (!pctx) return TADMM_ERR_INVALID_ARG;
  *pctx = nullptr;
  std::string err;
  if (!params_ok(params, err)) return TADMM_ERR_INVALID_ARG;
  tadmm_ctx *ctx = new tadmm_ctx();
  ctx->prm = *params;
  ctx->stream = (hipStream_t)stream;
  hipError_t e = hipGetDevice(&ctx->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device);
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->h_flags, 64 * sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreate(&ctx->ev0);
  if (e == hipSuccess) e = hipEventCreate(&ctx->ev1);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = scratch_address(ctx->device, &ctx->scratch);
  if (e != hipSuccess) {
    (void)tadmm_destroy(ctx);
    return TADMM_ERR_HIP;
  }
  *pctx = ctx;
  return TADMM_OK;
}

tadmm_status tadmm_destroy(tadmm_ctx *ctx) {
  if (!ctx) return TADMM_ERR_INVALID_ARG;
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  for (int q = 0; q < 2; ++q) {
    if (ctx->wexec[q]) (void)hipGraphExecDestroy(ctx->wexec[q]);
    if (ctx->wgraph[q]) (void)hipGraphDestroy(ctx->wgraph[q]);
  }
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
  return TADMM_OK;
}

tadmm_status tadmm_solve(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                         size_t workspace_bytes, int32_t mode) {
  if (!ctx) return TADMM_ERR_INVALID_ARG;
  if (!batch || !out) return fail(ctx, TADMM_ERR_INVALID_ARG, "batch / out is NULL");
  ctx->err.clear();
  const bool di = is_double_integrator(ctx->prm, batch);
  if (ctx->prm.nx == 4)
    return di ? solve_impl<4, 2, true>(ctx, batch, out, workspace, workspace_bytes, mode)
              : solve_impl<4, 2, false>(ctx, batch, out, workspace, workspace_bytes, mode);
  return di ? solve_impl<6, 3, true>(ctx, batch, out, workspace, workspace_bytes, mode)
            : solve_impl<6, 3, false>(ctx, batch, out, workspace, workspace_bytes, mode);
}

tadmm_status tadmm_solve_noalloc(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, int32_t mode) {
  if (!ctx) return TADMM_ERR_INVALID_ARG;
  if (!batch || !out) return fail(ctx, TADMM_ERR_INVALID_ARG, "batch / out is NULL");
  ctx->err.clear();
  ctx->solved = false;
  ctx->polished = false;
  const bool di = is_double_integrator(ctx->prm, batch);
  void *ws = ctx->scratch;
  const size_t bytes = kStaticScratchBytes;
  if (ctx->prm.nx == 4)
    return di ? solve_impl<4, 2, true>(ctx, batch, out, ws, bytes, mode, true)
              : solve_impl<4, 2, false>(ctx, batch, out, ws, bytes, mode, true);
  return di ? solve_impl<6, 3, true>(ctx, batch, out, ws, bytes, mode, true)
            : solve_impl<6, 3, false>(ctx, batch, out, ws, bytes, mode, true);
}

tadmm_status tadmm_sqp(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                       size_t workspace_bytes, int32_t mode, int32_t max_rounds, float rtol, float sep_tol,
                       float *stats) {
  if (!ctx) return TADMM_ERR_INVALID_ARG;
  if (!batch || !out) return fail(ctx, TADMM_ERR_INVALID_ARG, "batch / out is NULL");
  ctx->err.clear();
  return sqp_dispatch(ctx, batch, out, workspace, workspace_bytes, mode, max_rounds, rtol, sep_tol, stats);
}

tadmm_status tadmm_autotune(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                            size_t workspace_bytes, int32_t *best_threads) {
  if (!ctx) return TADMM_ERR_INVALID_ARG;
  const int saved = ctx->prm.block_threads;
  const int cands[] = {64, 128, 192, 256};
  float best = 1e30f;
  int best_t = ctx->tuned_threads;
  for (int c : cands) {
    ctx->prm.block_threads = c;
    tadmm_status st = tadmm_solve(ctx, batch, out, workspace, workspace_bytes, TADMM_MODE_BATCHED);
    if (st != TADMM_OK) { ctx->prm.block_threads = saved; return st; }
    st = tadmm_solve(ctx, batch, out, workspace, workspace_bytes, TADMM_MODE_BATCHED);
    if (st != TADMM_OK) { ctx->prm.block_threads = saved; return st; }
    if (ctx->last_ms < best) { best = ctx->last_ms; best_t = c; }
  }
  ctx->prm.block_threads = saved;
  ctx->tuned_threads = best_t;
  if (best_threads) *best_threads = best_t;
  return TADMM_OK;
}

tadmm_status tadmm_polish(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                          size_t workspace_bytes, float *stats) {
  if (!ctx) return TADMM_ERR_INVALID_ARG;
  if (!batch || !out) return fail(ctx, TADMM_ERR_INVALID_ARG, "batch / out is NULL");
  if (!out->x || !out->u) return fail(ctx, TADMM_ERR_INVALID_ARG, "out.x and out.u are required");
  ctx->err.clear();
  EqpIO io{};
  io.x = out->x;
  io.u = out->u;
  io.stats = stats;
  return eqp_dispatch(ctx, batch, out, workspace, workspace_bytes, EQ_POLISH, io);
}

tadmm_status tadmm_adjoint(tadmm_ctx *ctx, const tadmm_batch *batch, const tadmm_out *out, void *workspace,
                           size_t workspace_bytes, const float *dL_dx, const float *dL_du, float *dL_dx0,
                           float *dL_dxref, float *dL_dlogq, float *dL_dlogr, float *stats) {
  if (!ctx) return TADMM_ERR_INVALID_ARG;
  if (!batch) return fail(ctx, TADMM_ERR_INVALID_ARG, "batch is NULL");
  if (!dL_dx) return fail(ctx, TADMM_ERR_INVALID_ARG, "dL_dx is required");
  ctx->err.clear();
  EqpIO io{};
  io.gx = dL_dx;
  io.gu = dL_du;
  io.dx0 = dL_dx0;
  io.dxref = dL_dxref;
  io.dlogq = dL_dlogq;
  io.dlogr = dL_dlogr;
  io.stats = stats;
  return eqp_dispatch(ctx, batch, out, workspace, workspace_bytes, EQ_ADJOINT, io);
}

}  // extern "C"
