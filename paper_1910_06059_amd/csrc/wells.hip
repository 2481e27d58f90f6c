// Standard well model on the device (paper sec. 2.2.1): the well equations
// and their coupling blocks, and the pieces of the Schur-complement solve
// (eq. wellequation) that the Newton step and the Krylov solver use.
//
// Each well has the unknowns x_w = (Q_t, F_w, F_g, p_bhp); its equations
// are component conservation with wellbore storage (eq. conseq-swell),
// R_a,w = (V_w mix_a - A0_a,w) / dt + Q_a - sum_j q_a,j, and its control
// (eq. well-control-bhp: p_bhp - target; eq. well-control-rate: Q_a +
// target for an injector of component a; on a well's limit: p_bhp - limit
// for an injector, Q_o - limit for a producer).  Connection rates and the
// wellbore fluid are those of the assembly (assemble_dev.h), so the cell
// rows (with their blocks C = d(cell residual)/dx_w) and the well rows
// (B = dR_w/d(cell variables), D = dR_w/dx_w) come from one definition.
//
// One workgroup of one wavefront per well: lanes take the well's
// connections in turn and the per-well sums are a fixed shuffle tree, so
// results do not depend on scheduling.  With the Schur complement the
// Krylov operator is A x - sum_w C_w D_w^{-1} B_w x: the correction
// C_q D_w^{-1} (B_w x) of every connection q is written here and subtracted
// by the SpMV in the rows of the perforated cells.
#include <algorithm>
#include <cstring>

#include "assemble_dev.h"
#include "wells_dev.h"

namespace opm {
namespace {

using namespace asmdev;

constexpr int kWellThreads = kWave;

struct WellArgs {
  int n_wells;
  const int32_t* well_conn_ptr;
  const int32_t* conn_cell;
  const double* conn_wi;
  const int32_t* well_kind;
  const int32_t* well_phase;
  const double* well_target;
  const double* well_vol;
  double* well_state;
  const double* pore_vol;
  const uint8_t* meaning;
  const double* well_limit;   // null: no limits
  int32_t* well_ctrl;
  opm_fluid fluid;
};

WellArgs well_args(const opm_problem* pb) {
  const bool lim = pb->well_limit != nullptr;
  return WellArgs{pb->n_wells,    pb->well_conn_ptr, pb->conn_cell,   pb->conn_wi,
                  pb->well_kind,  pb->well_phase,    pb->well_target, pb->well_vol,
                  pb->well_state, pb->pore_vol,      pb->meaning,
                  lim ? pb->well_limit : nullptr,    lim ? pb->well_ctrl : nullptr,
                  pb->fluid};
}

// Active control of well w: 0 its own, 1 its limit.
__device__ __forceinline__ int well_ctrl(const WellArgs& a, int w) {
  return a.well_ctrl ? a.well_ctrl[w] : 0;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Wellbore storage V_w mix_a of a well state: A0 [nw][3] (one lane per well).
__global__ void k_well_storage0(WellArgs a, const double* wx, double* A0) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= a.n_wells) return;
  const WellVars W = well_vars(a.fluid, wx + 4 * w);
#pragma unroll
  for (int c = 0; c < 3; ++c) A0[3 * w + c] = a.well_vol[w] * W.mix[c].v;
}

// Inverse of a 4x4 matrix by Gauss-Jordan elimination with partial pivoting;
// false on a zero pivot.
__device__ bool inv4(const double* Din, double* X) {
  double M[4][8];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      M[r][c] = Din[4 * r + c];
      M[r][4 + c] = r == c ? 1.0 : 0.0;
    }
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (M[piv][c] == 0.0 || !isfinite(M[piv][c])) return false;
    if (piv != c)
      for (int k = 0; k < 8; ++k) {
        const double t = M[c][k];
        M[c][k] = M[piv][k];
        M[piv][k] = t;
      }
    const double inv = 1.0 / M[c][c];
    for (int k = 0; k < 8; ++k) M[c][k] *= inv;
    for (int r = 0; r < 4; ++r)
      if (r != c) {
        const double f = M[r][c];
        for (int k = 0; k < 8; ++k) M[r][k] -= f * M[c][k];
      }
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) X[4 * r + c] = M[r][4 + c];
  return true;
}

// Well equations, B and D (and D^{-1}), and the well's convergence measure
// wn: max over components of dt |R_a| / (b_a(p_bhp) V_perf) (V_perf the pore
// volume of the perforated cells) and |R_c| / |target|.
template <bool LIVE, bool WET = false>
__global__ __launch_bounds__(kWellThreads) void k_well_system(WellArgs a, const double* y,
                                                               const double* A0, double dt,
                                                               double* Rw, double* B, double* D,
                                                               double* Dinv, double* wn,
                                                               int32_t* flags) {
  const int w = blockIdx.x, lane = threadIdx.x;
  const WellVars W = well_vars(a.fluid, a.well_state + 4 * w);
  double s[3][5] = {};   // per component: sum_j q_a,j and its 4 well derivatives
  double vref = 0.0;
  for (int q = a.well_conn_ptr[w] + lane; q < a.well_conn_ptr[w + 1]; q += kWellThreads) {
    const int c = a.conn_cell[q];
    FaceProps P;
    properties<LIVE, WET>(a.fluid, y[3 * c], y[3 * c + 1], y[3 * c + 2], LIVE ? a.meaning[c] : 0, P,
                     nullptr);
    D7 qr[3];
    std_conn_rate<LIVE, WET>(P, W, a.conn_wi[q], qr);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      s[e][0] += qr[e].v;
#pragma unroll
      for (int k = 0; k < 4; ++k) s[e][1 + k] += qr[e].d[3 + k];
#pragma unroll
      for (int v = 0; v < 3; ++v) B[12 * (size_t)q + 3 * e + v] = -qr[e].d[v];
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) B[12 * (size_t)q + 9 + v] = 0.0;   // the control row
    vref += a.pore_vol[c];
  }
#pragma unroll
  for (int e = 0; e < 3; ++e)
#pragma unroll
    for (int k = 0; k < 5; ++k) s[e][k] = wave_sum(s[e][k]);
  vref = wave_sum(vref);
  if (lane != 0) return;
  D7 R[4];
  const double vol = a.well_vol[w];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    R[e] = (W.mix[e] * vol - cst<7>(A0[3 * w + e])) / dt + W.F[e] * W.Qt * (1.0 / well_g(e));
    R[e].v -= s[e][0];
#pragma unroll
    for (int k = 0; k < 4; ++k) R[e].d[3 + k] -= s[e][1 + k];
  }
  const int ctrl = well_ctrl(a, w);
  const double target = ctrl ? a.well_limit[w] : a.well_target[w];
  if (a.well_kind[w] == OPM_WELL_BHP_PROD && ctrl == 0) {
    R[3] = W.pb - cst<7>(target);
  } else if (a.well_kind[w] == OPM_WELL_BHP_PROD) {   // oil surface rate at the limit
    R[3] = W.F[1] * W.Qt * (1.0 / well_g(1)) - cst<7>(target);
  } else if (ctrl == 0) {
    const int ph = a.well_phase[w];
    R[3] = W.F[ph] * W.Qt * (1.0 / well_g(ph)) + cst<7>(target);
  } else {   // injector at its BHP limit
    R[3] = W.pb - cst<7>(target);
  }
  double Dw[16];
  for (int e = 0; e < 4; ++e) {
    Rw[4 * w + e] = R[e].v;
    for (int k = 0; k < 4; ++k) Dw[4 * e + k] = R[e].d[3 + k];
  }
  if (D)
    for (int k = 0; k < 16; ++k) D[16 * w + k] = Dw[k];
  if (!inv4(Dw, Dinv + 16 * w)) flags[0] = OPM_ESINGULAR;
  double m = fabs(R[3].v) / fabs(target);
  for (int e = 0; e < 3; ++e) {
    const double b = exp(a.fluid.c[e] * (W.pb.v - a.fluid.p_ref));
    m = nan_max(m, dt * fabs(R[e].v) / (b * vref));
  }
  wn[w] = m;
}

// u = Dinv_w t (4 x 4 times 4).
__device__ __forceinline__ void apply_dinv(const double* Dinv, const double t[4], double u[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) v += Dinv[4 * e + k] * t[k];
    u[e] = v;
  }
}

// t = sum_q B_q x_cell(q) over the well's connections, in every lane.
__device__ __forceinline__ void sum_bx(const int32_t* well_conn_ptr, const int32_t* conn_cell,
                                      const double* B, const double* x, int w, double t[4]) {
  double p[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q = well_conn_ptr[w] + (int)threadIdx.x; q < well_conn_ptr[w + 1]; q += kWellThreads) {
    const double* xc = x + 3 * (size_t)conn_cell[q];
    const double* Bq = B + 12 * (size_t)q;
#pragma unroll
    for (int e = 0; e < 4; ++e) p[e] += Bq[3 * e] * xc[0] + Bq[3 * e + 1] * xc[1] + Bq[3 * e + 2] * xc[2];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) t[e] = wave_sum(p[e]);
}

// corr_q = C_q u for the well's connections.
__device__ __forceinline__ void write_corr(const int32_t* well_conn_ptr, const double* C,
                                           const double u[4], int w, double* corr) {
  for (int q = well_conn_ptr[w] + (int)threadIdx.x; q < well_conn_ptr[w + 1]; q += kWellThreads) {
    const double* Cq = C + 12 * (size_t)q;
#pragma unroll
    for (int e = 0; e < 3; ++e)
      corr[3 * (size_t)q + e] =
          Cq[4 * e] * u[0] + Cq[4 * e + 1] * u[1] + Cq[4 * e + 2] * u[2] + Cq[4 * e + 3] * u[3];
  }
}

// corr = C D^{-1} B x (the operator's correction); nothing while *skip != 0.
__global__ __launch_bounds__(kWellThreads) void k_well_op(WellSchur ws, const double* x,
                                                           const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int w = blockIdx.x;
  double t[4], u[4];
  sum_bx(ws.well_conn_ptr, ws.conn_cell, ws.B, x, w, t);
  apply_dinv(ws.Dinv + 16 * w, t, u);
  write_corr(ws.well_conn_ptr, ws.C, u, w, ws.corr);
}

// corr = C D^{-1} R_w (the right-hand side's correction).
__global__ __launch_bounds__(kWellThreads) void k_well_rhs(WellSchur ws, const double* Rw) {
  const int w = blockIdx.x;
  double t[4], u[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) t[e] = Rw[4 * w + e];
  apply_dinv(ws.Dinv + 16 * w, t, u);
  write_corr(ws.well_conn_ptr, ws.C, u, w, ws.corr);
}

// R_i -= sum of the corrections of cell i's connections.
__global__ __launch_bounds__(kBlock) void k_sub_corr(int n, const int32_t* ccp, const int32_t* cc,
                                                      const double* corr, double* R) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int t = ccp[i]; t < ccp[i + 1]; ++t)
#pragma unroll
    for (int e = 0; e < 3; ++e) R[3 * (size_t)i + e] -= corr[3 * (size_t)cc[t] + e];
}

// Well unknowns after the reservoir solve: d_w = D^{-1} (R_w - B d_r), and
// x_w -= d_w with |d p_bhp| <= dp_max_rel |p_bhp|, the fraction pair
// scaled to at most ds_max, fractions kept in [0, 1] with F_w + F_g <= 1.
// Then the control switch of a well with a limit (sec. 2.2.1 names BHP and
// rate controls; the rule is a reading): on its own control it moves to
// the limit when the limit is exceeded (a producer's oil surface rate, an
// injector's BHP above it), on the limit back to its own control when that
// binds again (the producer's BHP below its target, the injector's rate
// above its target).
__global__ __launch_bounds__(kWellThreads) void k_well_update(WellSchur ws, WellArgs a,
                                                               const double* Rw, const double* d,
                                                               double* wx, double ds_max,
                                                               double dp_max_rel, int32_t* flags) {
  const int w = blockIdx.x;
  double t[4], u[4];
  sum_bx(ws.well_conn_ptr, ws.conn_cell, ws.B, d, w, t);
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) t[e] = Rw[4 * w + e] - t[e];
  apply_dinv(ws.Dinv + 16 * w, t, u);
  double* x = wx + 4 * w;
  double dpb = -u[3];
  const double lim = dp_max_rel * fabs(x[3]);
  dpb = fmin(fmax(dpb, -lim), lim);
  double dfw = -u[1], dfg = -u[2];
  const double mx = fmax(fabs(dfw), fabs(dfg));
  if (mx > ds_max) {
    dfw *= ds_max / mx;
    dfg *= ds_max / mx;
  }
  x[0] -= u[0];
  x[1] = fmin(fmax(x[1] + dfw, 0.0), 1.0);
  x[2] = fmin(fmax(x[2] + dfg, 0.0), 1.0);
  if (x[1] + x[2] > 1.0) {
    const double sc = 1.0 / (x[1] + x[2]);
    x[1] *= sc;
    x[2] *= sc;
  }
  x[3] += dpb;
  if (!isfinite(x[0]) || !isfinite(x[1]) || !isfinite(x[2]) || !isfinite(x[3])) flags[1] = 1;
  if (a.well_ctrl && a.well_limit[w] > 0.0) {
    const int c = a.well_ctrl[w];
    const double limit = a.well_limit[w], target = a.well_target[w];
    int next = c;
    if (a.well_kind[w] == OPM_WELL_BHP_PROD) {
      const double qo = (1.0 - x[1] - x[2]) * x[0] / well_g(1);
      if (c == 0 && qo > limit) next = 1;
      else if (c == 1 && x[3] < target) next = 0;
    } else {
      const int ph = a.well_phase[w];
      const double f = ph == 0 ? x[1] : ph == 2 ? x[2] : 1.0 - x[1] - x[2];
      const double inj = -f * x[0] / well_g(ph);
      if (c == 0 && x[3] > limit) next = 1;
      else if (c == 1 && inj > target) next = 0;
    }
    a.well_ctrl[w] = next;
  }
}

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t wells_bytes(const opm_problem* pb) {
  if (pb->n_wells <= 0) return 0;
  const size_t nw = pb->n_wells, nc = pb->n_conns;
  return al256(8 * 4 * nw) + 2 * al256(8 * 12 * nc) + 2 * al256(8 * 16 * nw) +
         al256(8 * 3 * nc) + al256(8 * 3 * nw) + al256(8 * nw) + al256(8 * 4 * nw) +
         al256(4 * nw);
}

WellWork wells_carve(const opm_problem* pb, void* p) {
  const size_t nw = pb->n_wells, nc = pb->n_conns;
  char* c = (char*)p;
  WellWork w;
  w.Rw = (double*)c;
  c += al256(8 * 4 * nw);
  w.B = (double*)c;
  c += al256(8 * 12 * nc);
  w.C = (double*)c;
  c += al256(8 * 12 * nc);
  w.D = (double*)c;
  c += al256(8 * 16 * nw);
  w.Dinv = (double*)c;
  c += al256(8 * 16 * nw);
  w.corr = (double*)c;
  c += al256(8 * 3 * nc);
  w.A0 = (double*)c;
  c += al256(8 * 3 * nw);
  w.wn = (double*)c;
  c += al256(8 * nw);
  w.save = (double*)c;
  c += al256(8 * 4 * nw);
  w.save_ctrl = (int32_t*)c;
  return w;
}

WellSchur well_schur(const opm_problem* pb, const WellWork& ww) {
  WellSchur s;
  std::memset(&s, 0, sizeof s);   // zero padding: the struct is part of a graph key
  s.n_wells = pb->n_wells;
  s.well_conn_ptr = pb->well_conn_ptr;
  s.conn_cell = pb->conn_cell;
  s.B = ww.B;
  s.C = ww.C;
  s.Dinv = ww.Dinv;
  s.corr = ww.corr;
  s.ccp = pb->cell_conn_ptr;
  s.cc = pb->cell_conn;
  return s;
}

int well_storage0(const opm_problem* pb, const double* wx, double* A0, hipStream_t s) {
  hipLaunchKernelGGL(k_well_storage0, dim3(blocks_for(pb->n_wells, kWave)), dim3(kWave), 0, s,
                     well_args(pb), wx, A0);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int well_system(const opm_problem* pb, const double* y, double dt, const WellWork& ww,
                int32_t* flags, hipStream_t s) {
  if (pb->fluid.live && pb->fluid.rv_c > 0.0)   // wet gas
    hipLaunchKernelGGL((k_well_system<true, true>), dim3(pb->n_wells), dim3(kWellThreads), 0, s,
                       well_args(pb), y, ww.A0, dt, ww.Rw, ww.B, ww.D, ww.Dinv, ww.wn, flags);
  else if (pb->fluid.live)
    hipLaunchKernelGGL(k_well_system<true>, dim3(pb->n_wells), dim3(kWellThreads), 0, s,
                       well_args(pb), y, ww.A0, dt, ww.Rw, ww.B, ww.D, ww.Dinv, ww.wn, flags);
  else
    hipLaunchKernelGGL(k_well_system<false>, dim3(pb->n_wells), dim3(kWellThreads), 0, s,
                       well_args(pb), y, ww.A0, dt, ww.Rw, ww.B, ww.D, ww.Dinv, ww.wn, flags);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int well_rhs(const opm_problem* pb, const WellWork& ww, double* R, hipStream_t s) {
  const WellSchur ws = well_schur(pb, ww);
  hipLaunchKernelGGL(k_well_rhs, dim3(pb->n_wells), dim3(kWellThreads), 0, s, ws, ww.Rw);
  hipLaunchKernelGGL(k_sub_corr, dim3(blocks_for(pb->n_cells, kBlock)), dim3(kBlock), 0, s,
                     pb->n_cells, pb->cell_conn_ptr, pb->cell_conn, ww.corr, R);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int well_op(const WellSchur& ws, const double* x, const int32_t* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_well_op, dim3(ws.n_wells), dim3(kWellThreads), 0, s, ws, x, skip);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int well_update(const opm_problem* pb, const WellWork& ww, const double* d, double ds_max,
                double dp_max_rel, int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_well_update, dim3(pb->n_wells), dim3(kWellThreads), 0, s,
                     well_schur(pb, ww), well_args(pb), ww.Rw, d, pb->well_state, ds_max,
                     dp_max_rel, flags);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

}  // namespace opm
