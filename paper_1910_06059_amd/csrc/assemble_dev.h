// Device-side pieces of the residual and Jacobian assembly, shared by the
// one-launch-per-step kernels (assemble.hip) and the persistent ensemble
// kernel (ensemble.hip): dual numbers, cell properties, face flux and the
// work of one block row.  Paper sec. 2.1.1 (eqs. materialbalance, flux1,
// head), sec. 2.1.5 (eq. gwseg), sec. 2.1.6 (PVT), sec. 2.2.1 (eq.
// wellinflow), sec. 2.4.1 (forward-mode AD).
//
// Floating-point contraction is disabled for everything in this header: a
// face flux is evaluated by both of its cells, in the same orientation, and
// the two evaluations must round identically (u_ij = -u_ji exactly).
#pragma once
#pragma clang fp contract(off)

#include "common.h"

namespace opm {
namespace asmdev {

// ---------------------------------------------------------- dual numbers
template <int N>
struct Dual {
  double v;
  double d[N];
};

template <int N>
__device__ __forceinline__ Dual<N> cst(double v) {
  Dual<N> r;
  r.v = v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = 0.0;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, double s) {
  Dual<N> r;
  r.v = a.v * s;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * s;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, double s) {
  Dual<N> r;
  r.v = a.v / s;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / s;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> quot(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v / b.v;
  const double b2 = b.v * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / b2;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> dexp(const Dual<N>& a) {
  Dual<N> r;
  r.v = exp(a.v);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = r.v * a.d[k];
  return r;
}
// x^n for x >= 0, n >= 1 (Corey curves)
template <int N>
__device__ __forceinline__ Dual<N> dpow(const Dual<N>& a, double n) {
  Dual<N> r;
  double dv;
  if (n == 2.0) {
    r.v = a.v * a.v;
    dv = 2.0 * a.v;
  } else {
    r.v = pow(a.v, n);
    dv = n * pow(a.v, n - 1.0);
  }
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = dv * a.d[k];
  return r;
}
// clamp to [0, 1]; the argument passes through on the bounds themselves
template <int N>
__device__ __forceinline__ Dual<N> clamp01(const Dual<N>& a) {
  if (a.v < 0.0) return cst<N>(0.0);
  if (a.v > 1.0) return cst<N>(1.0);
  return a;
}
// max(a, 0); the constant branch is taken at a == 0
template <int N>
__device__ __forceinline__ Dual<N> pos(const Dual<N>& a) {
  return a.v > 0.0 ? a : cst<N>(0.0);
}

using D3 = Dual<3>;
using D6 = Dual<6>;

// Lift a cell quantity (derivatives w.r.t. the cell's own (p, sw, sg)) into
// the face slots: slots 0-2 for the lower cell, 3-5 for the upper cell.
__device__ __forceinline__ D6 lift(const D3& a, int side) {
  D6 r;
  r.v = a.v;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.d[k] = side == 0 ? a.d[k] : 0.0;
    r.d[3 + k] = side == 0 ? 0.0 : a.d[k];
  }
  return r;
}

// ------------------------------------------------------ cell properties
struct FaceProps {
  double p;
  D3 rho[3];                // densities (live oil: with its dissolved gas)
  D3 mob[3];                // b_alpha * lambda_alpha
  D3 rmob;                  // r b_o lambda_o: dissolved gas carried by the oil (live oil)
  D3 vmob;                  // r_og b_g lambda_g: oil carried by the gas (wet gas)
  D3 lamt;                  // total mobility sum_alpha lambda_alpha (well injection)
};

__device__ __forceinline__ D3 sel(bool c, const D3& x, const D3& y) {
  D3 r;
  r.v = c ? x.v : y.v;
#pragma unroll
  for (int k = 0; k < 3; ++k) r.d[k] = c ? x.d[k] : y.d[k];
  return r;
}

// Element-wise select (keeps both operands in registers; a reference picked
// at run time would force them to memory).
__device__ __forceinline__ FaceProps pick(bool c, const FaceProps& x, const FaceProps& y) {
  FaceProps r;
  r.p = c ? x.p : y.p;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.rho[a] = sel(c, x.rho[a], y.rho[a]);
    r.mob[a] = sel(c, x.mob[a], y.mob[a]);
  }
  r.rmob = sel(c, x.rmob, y.rmob);
  r.vmob = sel(c, x.vmob, y.vmob);
  r.lamt = sel(c, x.lamt, y.lamt);
  return r;
}

struct CellAcc {
  D3 A[3];                  // b_alpha s_alpha (+ r b_o s_o for gas, live oil)
  double b[3];
};

// b = exp(c (p - p_ref)); rho = rho_S b; Corey curves with the segregation
// model for three-phase oil; mob = b k_r / mu.  The third variable x is s_g,
// or, for live oil in a cell without free gas (mean = 1), r_go with s_g = 0,
// or, with wet gas in a cell without oil (mean = 2), r_og with s_g = 1 - s_w
// (eq. primaryVariableMeaning).  Wet gas (sec. 2.1.6): r_og = r_v(p) =
// rv_c p where oil is present, rho_g = b_g (rho_gS + r_og rho_oS), and the
// oil component adds r_og b_g s_g (accumulation) and r_og b_g lambda_g
// (vmob, carried with the gas).  Live oil (sec. 2.1.6): r = r_s(p) = rs_c p
// where free gas is present, b_o /= (1 + bo_r r), mu_o /= (1 + muo_r r),
// rho_o = b_o (rho_oS + r rho_gS).
template <bool LIVE, bool WET = false>
__device__ __forceinline__ void properties(const opm_fluid& f, double p_v, double sw_v,
                                           double x_v, int mean, FaceProps& P, CellAcc* acc) {
  D3 p = cst<3>(p_v);
  p.d[0] = 1.0;
  D3 sw = cst<3>(sw_v);
  sw.d[1] = 1.0;
  D3 x = cst<3>(x_v);
  x.d[2] = 1.0;
  const bool undersat = LIVE && mean == 1;
  // wet gas: meaning 2 = no oil, s_g = 1 - s_w, x = r_og
  const bool wet = LIVE && WET;   // wet gas (the caller's kernel is picked by rv_c > 0)
  const bool oilfree = wet && mean == 2;
  const D3 sg = undersat ? cst<3>(0.0) : (oilfree ? cst<3>(1.0) - sw : x);
  D3 r = cst<3>(0.0);
  if (LIVE) r = sel(undersat, x, p * f.rs_c);
  D3 rv = cst<3>(0.0);
  if (wet) rv = sel(oilfree, x, p * f.rv_c);
  D3 so = (cst<3>(1.0) - sw) - sg;
  D3 b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) b[a] = dexp((p - cst<3>(f.p_ref)) * f.c[a]);
  if (LIVE) b[1] = quot(b[1], cst<3>(1.0) + r * f.bo_r);
  const double den = 1.0 - f.swc;
  D3 krw = dpow(clamp01((sw - cst<3>(f.swc)) / den), f.n_corey);
  D3 krg = dpow(clamp01(sg / den), f.n_corey);
  D3 kr_o2 = dpow(clamp01(so / den), f.n_corey);   // k_row = k_rog (same curve)
  D3 ww = pos(sw - cst<3>(f.swc));
  D3 wg = pos(sg);
  D3 wsum = ww + wg;
  D3 kro = wsum.v > 1e-14 ? quot(ww * kr_o2 + wg * kr_o2, wsum) : kr_o2;
  P.p = p_v;
  const D3 kr[3] = {krw, kro, krg};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    P.rho[a] = b[a] * f.rho_s[a];
    P.mob[a] = b[a] * (kr[a] / f.mu[a]);
  }
  P.rmob = cst<3>(0.0);
  D3 lam_o = kro / f.mu[1];
  if (LIVE) {
    P.rho[1] = b[1] * (cst<3>(f.rho_s[1]) + r * f.rho_s[2]);
    lam_o = (kro * (cst<3>(1.0) + r * f.muo_r)) / f.mu[1];
    P.mob[1] = b[1] * lam_o;
    P.rmob = r * P.mob[1];
  }
  P.vmob = cst<3>(0.0);
  if (wet) {
    P.rho[2] = b[2] * (cst<3>(f.rho_s[2]) + rv * f.rho_s[1]);
    P.vmob = rv * P.mob[2];
  }
  P.lamt = (krw / f.mu[0] + lam_o) + krg / f.mu[2];
  if (acc) {
    const D3 s[3] = {sw, so, sg};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc->A[a] = b[a] * s[a];
      acc->b[a] = b[a].v;
    }
    if (LIVE) acc->A[2] = acc->A[2] + r * (b[1] * so);
    if (wet) acc->A[1] = acc->A[1] + rv * (b[2] * sg);
  }
}

// Potential difference of phase a from lower cell L to upper cell H:
// dPhi = p_L - p_H - g (rho_L + rho_H)/2 (z_L - z_H).
__device__ __forceinline__ D6 potential(const FaceProps& L, const FaceProps& H, int a, double dz,
                                        double g) {
  D6 pl = cst<6>(L.p);
  pl.d[0] = 1.0;
  D6 ph = cst<6>(H.p);
  ph.d[3] = 1.0;
  D6 rho_avg = (lift(L.rho[a], 0) + lift(H.rho[a], 1)) * 0.5;
  return (pl - ph) - (rho_avg * g) * dz;
}

// Flux of component a from lower cell L to upper cell H through a face of
// transmissibility T: (b lambda)_U T dPhi, U = L if dPhi >= 0 else H; for
// live oil the gas component adds the dissolved gas, (r b_o lambda_o)_Uo T
// dPhi_o with the oil phase's potential and upwind cell.
template <bool LIVE, bool WET = false>
__device__ __forceinline__ D6 face_flux(const FaceProps& L, const FaceProps& H, int a, double dz,
                                        double T, double g) {
  const D6 dphi = potential(L, H, a, dz, g);
  D6 mob = dphi.v >= 0.0 ? lift(L.mob[a], 0) : lift(H.mob[a], 1);
  D6 F = mob * (dphi * T);
  if (LIVE && a == 2) {
    const D6 dphio = potential(L, H, 1, dz, g);
    D6 rm = dphio.v >= 0.0 ? lift(L.rmob, 0) : lift(H.rmob, 1);
    F = F + rm * (dphio * T);
  }
  // wet gas: the oil component adds the vaporised oil, (r_og b_g lambda_g)_Ug
  // T dPhi_g with the gas phase's potential and upwind cell
  if (LIVE && WET && a == 1) {
    const D6 dphig = potential(L, H, 2, dz, g);
    D6 vm = dphig.v >= 0.0 ? lift(L.vmob, 0) : lift(H.vmob, 1);
    F = F + vm * (dphig * T);
  }
  return F;
}

// ------------------------------------------------- standard wells (sec. 2.2.1)
using D7 = Dual<7>;

// Weights of the weighted total rate and fractions (eq. weighted_total_rate).
constexpr double kWellG0 = 1.0, kWellG1 = 1.0, kWellG2 = 0.01;
__device__ __forceinline__ double well_g(int a) { return a == 0 ? kWellG0 : (a == 1 ? kWellG1 : kWellG2); }

// The well unknowns as duals in slots 3-6 (Q_t, F_w, F_g, p_bhp) and the
// wellbore fluid's surface volume per reservoir volume of each component,
// mix_a = (F_a / g_a) / sum_b F_b / (g_b b_b(p_bhp)), F_o = 1 - F_w - F_g.
struct WellVars {
  D7 Qt, F[3], pb, mix[3];
};

__device__ __forceinline__ WellVars well_vars(const opm_fluid& f, const double* x) {
  WellVars W;
  W.Qt = cst<7>(x[0]);
  W.Qt.d[3] = 1.0;
  W.F[0] = cst<7>(x[1]);
  W.F[0].d[4] = 1.0;
  W.F[2] = cst<7>(x[2]);
  W.F[2].d[5] = 1.0;
  W.F[1] = (cst<7>(1.0) - W.F[0]) - W.F[2];
  W.pb = cst<7>(x[3]);
  W.pb.d[6] = 1.0;
  D7 S = cst<7>(0.0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const D7 b = dexp((W.pb - cst<7>(f.p_ref)) * f.c[a]);
    S = S + quot(W.F[a] * (1.0 / well_g(a)), b);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) W.mix[a] = quot(W.F[a] * (1.0 / well_g(a)), S);
  return W;
}

// A cell dual (slots 0-2) in the connection's slots.
__device__ __forceinline__ D7 lift7(const D3& a) {
  D7 r = cst<7>(a.v);
#pragma unroll
  for (int k = 0; k < 3; ++k) r.d[k] = a.d[k];
  return r;
}

// Surface rate of each component through a standard-well connection
// (production positive; eq. wellinflow with h_w,j = 0): producing (p > p_bhp)
// the cell's phases, q_a = WI b_a lambda_a (p - p_bhp) (+ r b_o lambda_o for
// gas, live oil); injecting the wellbore fluid at the cell's total
// mobility, q_a = WI lambda_t (p - p_bhp) mix_a.  Slots 0-2: the cell's
// variables; 3-6: the well's.
template <bool LIVE, bool WET = false>
__device__ __forceinline__ void std_conn_rate(const FaceProps& P, const WellVars& W, double wi,
                                              D7 q[3]) {
  D7 pc = cst<7>(P.p);
  pc.d[0] = 1.0;
  const D7 dp = pc - W.pb;
  if (dp.v > 0.0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = (lift7(P.mob[a]) * wi) * dp;
    if (LIVE) q[2] = q[2] + (lift7(P.rmob) * wi) * dp;
    if (LIVE && WET) q[1] = q[1] + (lift7(P.vmob) * wi) * dp;
  } else {
    const D7 lt = (lift7(P.lamt) * wi) * dp;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = lt * W.mix[a];
  }
}

struct AsmArgs {
  int n;
  const double* y;
  const double* acc0;
  double dt;
  const double* trans;
  const double* pv;
  const double* depth;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* blk_face;
  const int32_t* cell_conn_ptr;
  const int32_t* cell_conn;
  const int32_t* conn_kind;
  const int32_t* conn_phase;
  const double* conn_wi;
  const double* conn_rate;
  const double* conn_bhp;
  opm_fluid fluid;
  const uint8_t* meaning;   // [n] meaning of the third variable (live oil)
  int n_wells;              // > 0: standard wells (the connection terms below)
  const int32_t* conn_well;
  const double* well_state; // [n_wells][4]
  double* Cw;               // [n_conns][3][4] out: d(cell residual)/d(well unknowns)
  double* R;
  double* J;
  double* partials;   // [gridDim.x][kNormStride] or null
};

// Residual and Jacobian block row of cell i (one lane): writes R_i, the
// blocks J_i* (if a.J) and the cell's contributions to the CNV/MB norms:
// part = (dt|R_a|/(b_a PV) for a = w,o,g; R_a; b_a; PV).  LIVE: live oil
// with the cells' variable meanings in a.meaning.
template <bool LIVE, bool WET = false>
__device__ __forceinline__ void assemble_row(const AsmArgs& a, int i, double dt,
                                             double part[kNormStride]) {
  const double yi0 = a.y[3 * i], yi1 = a.y[3 * i + 1], yi2 = a.y[3 * i + 2];
  FaceProps Pi;
  CellAcc Ai;
  properties<LIVE, WET>(a.fluid, yi0, yi1, yi2, LIVE ? a.meaning[i] : 0, Pi, &Ai);
  const double pv = a.pv[i];
  const double zi = a.depth[i];
  D3 r[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = (Ai.A[c] - cst<3>(a.acc0[3 * i + c])) * (pv / dt);
  const int q0 = a.row_ptr[i], q1 = a.row_ptr[i + 1];
  int qd = q0;
  for (int q = q0; q < q1; ++q) {
    const int j = a.col_idx[q];
    if (j == i) {
      qd = q;
      continue;
    }
    FaceProps Pj;
    properties<LIVE, WET>(a.fluid, a.y[3 * j], a.y[3 * j + 1], a.y[3 * j + 2],
                     LIVE ? a.meaning[j] : 0, Pj, nullptr);
    const double T = a.trans[a.blk_face[q]];
    const double zj = a.depth[j];
    const bool lower = i < j;
    const FaceProps L = pick(lower, Pi, Pj);
    const FaceProps H = pick(lower, Pj, Pi);
    const double dz = lower ? zi - zj : zj - zi;
    double blk[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      D6 F = face_flux<LIVE, WET>(L, H, c, dz, T, a.fluid.g);
      if (lower) {
        r[c].v += F.v;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          r[c].d[v] += F.d[v];
          blk[3 * c + v] = F.d[3 + v];
        }
      } else {
        r[c].v -= F.v;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          r[c].d[v] -= F.d[3 + v];
          blk[3 * c + v] = -F.d[v];
        }
      }
    }
    if (a.J) {
      double* Jq = a.J + 9 * (size_t)q;
#pragma unroll
      for (int e = 0; e < 9; ++e) Jq[e] = blk[e];
    }
  }
  // wells of this cell (sec. 2.2.1): fixed-rate injector source or BHP
  // producer q = b lambda WI (p - p_bhp)^+ (live oil: plus r times the oil
  // rate in the gas component)
  for (int t = a.cell_conn_ptr[i]; t < a.cell_conn_ptr[i + 1]; ++t) {
    const int k = a.cell_conn[t];
    if (a.n_wells > 0) {   // standard well: the connection rate from the well unknowns
      const WellVars W = well_vars(a.fluid, a.well_state + 4 * a.conn_well[k]);
      D7 q[3];
      std_conn_rate<LIVE, WET>(Pi, W, a.conn_wi[k], q);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        r[c].v += q[c].v;
#pragma unroll
        for (int v = 0; v < 3; ++v) r[c].d[v] += q[c].d[v];
        if (a.Cw) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) a.Cw[12 * (size_t)k + 4 * c + kk] = q[c].d[3 + kk];
        }
      }
      continue;
    }
    if (a.conn_kind[k] == OPM_WELL_RATE_INJ) {
      const int ph = a.conn_phase[k];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (c == ph) r[c].v += a.conn_rate[k];
    } else {
      D3 dp = cst<3>(yi0 - a.conn_bhp[k]);
      dp.d[0] = 1.0;
      if (dp.v > 0.0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = r[c] + (Pi.mob[c] * a.conn_wi[k]) * dp;
        if (LIVE) r[2] = r[2] + (Pi.rmob * a.conn_wi[k]) * dp;
        if (LIVE && WET) r[1] = r[1] + (Pi.vmob * a.conn_wi[k]) * dp;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) a.R[3 * i + c] = r[c].v;
  if (a.J) {
    double* Jd = a.J + 9 * (size_t)qd;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int v = 0; v < 3; ++v) Jd[3 * c + v] = r[c].d[v];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    // an exactly balanced cell contributes 0 (also when it has no pore volume)
    part[c] = r[c].v == 0.0 ? 0.0 : dt * fabs(r[c].v) / (Ai.b[c] * pv);
    part[3 + c] = r[c].v;
    part[6 + c] = Ai.b[c];
  }
  part[9] = pv;
}

}  // namespace asmdev
}  // namespace opm

#pragma clang fp contract(fast)
