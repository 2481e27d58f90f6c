// Residual and 3x3-block Jacobian of the discrete black-oil mass balance by
// forward-mode AD (paper sec. 2.1.1 eq. materialbalance, eqs. flux1 and head,
// sec. 2.1.5 eq. gwseg, sec. 2.1.6 PVT, sec. 2.2.1 eq. wellinflow; AD as in
// sec. 2.4.1, localisation as in sec. 2.4.2).
//
// One lane owns one block row (cell i): it evaluates the AD properties of
// its cell and of each neighbour, the TPFA flux of each of its faces, the
// accumulation and well terms, and writes R_i and the blocks J_i* with plain
// stores (no atomics, deterministic).  Each face flux is evaluated in the
// canonical orientation (lower cell -> upper cell) by both of its cells with
// the same instruction sequence, and floating-point contraction is disabled
// in this file, so the two evaluations are bitwise equal and u_ij = -u_ji
// holds exactly.  The CNV / MB norms are reduced in the same pass.
#pragma clang fp contract(off)

#include "common.h"

namespace opm {
namespace {

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
  double rho[3], drho[3];   // density and d rho / dp (rho depends on p only)
  D3 mob[3];                // b_alpha * lambda_alpha
};

// Element-wise select (keeps both operands in registers; a reference picked
// at run time would force them to memory).
__device__ __forceinline__ FaceProps pick(bool c, const FaceProps& x, const FaceProps& y) {
  FaceProps r;
  r.p = c ? x.p : y.p;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.rho[a] = c ? x.rho[a] : y.rho[a];
    r.drho[a] = c ? x.drho[a] : y.drho[a];
    r.mob[a].v = c ? x.mob[a].v : y.mob[a].v;
#pragma unroll
    for (int k = 0; k < 3; ++k) r.mob[a].d[k] = c ? x.mob[a].d[k] : y.mob[a].d[k];
  }
  return r;
}

struct CellAcc {
  D3 A[3];                  // b_alpha s_alpha
  double b[3];
};

// b = exp(c (p - p_ref)); rho = rho_S b; Corey curves with the segregation
// model for three-phase oil; mob = b k_r / mu.
__device__ __forceinline__ void properties(const opm_fluid& f, double p_v, double sw_v,
                                           double sg_v, FaceProps& P, CellAcc* acc) {
  D3 p = cst<3>(p_v);
  p.d[0] = 1.0;
  D3 sw = cst<3>(sw_v);
  sw.d[1] = 1.0;
  D3 sg = cst<3>(sg_v);
  sg.d[2] = 1.0;
  D3 so = (cst<3>(1.0) - sw) - sg;
  D3 b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) b[a] = dexp((p - cst<3>(f.p_ref)) * f.c[a]);
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
    P.rho[a] = f.rho_s[a] * b[a].v;
    P.drho[a] = f.rho_s[a] * b[a].d[0];
    P.mob[a] = b[a] * (kr[a] / f.mu[a]);
  }
  if (acc) {
    const D3 s[3] = {sw, so, sg};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc->A[a] = b[a] * s[a];
      acc->b[a] = b[a].v;
    }
  }
}

// Flux of component a from lower cell L to upper cell H through a face of
// transmissibility T: (b lambda)_U T dPhi with dPhi = p_L - p_H -
// g (rho_L + rho_H)/2 (z_L - z_H), U = L if dPhi >= 0 else H.
__device__ __forceinline__ D6 face_flux(const FaceProps& L, const FaceProps& H, int a, double dz,
                                        double T, double g) {
  D6 pl = cst<6>(L.p);
  pl.d[0] = 1.0;
  D6 ph = cst<6>(H.p);
  ph.d[3] = 1.0;
  D6 rl = cst<6>(L.rho[a]);
  rl.d[0] = L.drho[a];
  D6 rh = cst<6>(H.rho[a]);
  rh.d[3] = H.drho[a];
  D6 rho_avg = (rl + rh) * 0.5;
  D6 dphi = (pl - ph) - (rho_avg * g) * dz;
  D6 mob = dphi.v >= 0.0 ? lift(L.mob[a], 0) : lift(H.mob[a], 1);
  return mob * (dphi * T);
}

struct Args {
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
  double* R;
  double* J;
  double* partials;   // [gridDim.x][kNormStride] or null
};

__global__ __launch_bounds__(kBlock) void k_assemble(Args a) {
  __shared__ double sh[kBlock / kWave];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < a.n;
  double part[kNormStride];
#pragma unroll
  for (int k = 0; k < kNormStride; ++k) part[k] = 0.0;
  if (valid) {
    const double yi0 = a.y[3 * i], yi1 = a.y[3 * i + 1], yi2 = a.y[3 * i + 2];
    FaceProps Pi;
    CellAcc Ai;
    properties(a.fluid, yi0, yi1, yi2, Pi, &Ai);
    const double pv = a.pv[i];
    const double zi = a.depth[i];
    D3 r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = (Ai.A[c] - cst<3>(a.acc0[3 * i + c])) * (pv / a.dt);
    const int q0 = a.row_ptr[i], q1 = a.row_ptr[i + 1];
    int qd = q0;
    for (int q = q0; q < q1; ++q) {
      const int j = a.col_idx[q];
      if (j == i) {
        qd = q;
        continue;
      }
      FaceProps Pj;
      properties(a.fluid, a.y[3 * j], a.y[3 * j + 1], a.y[3 * j + 2], Pj, nullptr);
      const double T = a.trans[a.blk_face[q]];
      const double zj = a.depth[j];
      const bool lower = i < j;
      const FaceProps L = pick(lower, Pi, Pj);
      const FaceProps H = pick(lower, Pj, Pi);
      const double dz = lower ? zi - zj : zj - zi;
      double blk[9];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        D6 F = face_flux(L, H, c, dz, T, a.fluid.g);
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
    // producer q = b lambda WI (p - p_bhp)^+
    for (int t = a.cell_conn_ptr[i]; t < a.cell_conn_ptr[i + 1]; ++t) {
      const int k = a.cell_conn[t];
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
      part[c] = r[c].v == 0.0 ? 0.0 : a.dt * fabs(r[c].v) / (Ai.b[c] * pv);
      part[3 + c] = r[c].v;
      part[6 + c] = Ai.b[c];
    }
    part[9] = pv;
  }
  if (a.partials) {
    double out[kNormStride];
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = block_max<kBlock>(part[c], sh);
#pragma unroll
    for (int k = 3; k < kNormStride; ++k) out[k] = block_sum<kBlock>(part[k], sh);
    if (threadIdx.x < kNormStride) {
      double v = out[0];
#pragma unroll
      for (int k = 1; k < kNormStride; ++k)
        if ((int)threadIdx.x == k) v = out[k];
      a.partials[(size_t)blockIdx.x * kNormStride + threadIdx.x] = v;
    }
  }
}

// Final, fixed-order reduction of the per-block partials into
// (CNV_w, CNV_o, CNV_g, MB_w, MB_o, MB_g, max CNV, max MB).
__global__ __launch_bounds__(kBlock) void k_norms_final(const double* partials, int nblk, int n,
                                                         double dt, double* norms) {
  __shared__ double sh[kBlock / kWave];
  double part[kNormStride];
#pragma unroll
  for (int k = 0; k < kNormStride; ++k) part[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
    const double* pb = partials + (size_t)b * kNormStride;
#pragma unroll
    for (int c = 0; c < 3; ++c) part[c] = nan_max(part[c], pb[c]);
#pragma unroll
    for (int k = 3; k < kNormStride; ++k) part[k] += pb[k];
  }
  double out[kNormStride];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = block_max<kBlock>(part[c], sh);
#pragma unroll
  for (int k = 3; k < kNormStride; ++k) out[k] = block_sum<kBlock>(part[k], sh);
  if (threadIdx.x == 0) {
    double cmax = 0.0, mmax = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double bbar = out[6 + c] / n;
      const double mb = dt * fabs(out[3 + c]) / (bbar * out[9]);
      norms[c] = out[c];
      norms[3 + c] = mb;
      cmax = nan_max(cmax, out[c]);
      mmax = nan_max(mmax, mb);
    }
    norms[6] = cmax;
    norms[7] = mmax;
  }
}

__global__ __launch_bounds__(kBlock) void k_accumulation(int n, opm_fluid f, const double* y,
                                                          double* acc) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  FaceProps P;
  CellAcc A;
  properties(f, y[3 * i], y[3 * i + 1], y[3 * i + 2], P, &A);
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[3 * i + c] = A.A[c].v;
}

}  // namespace

int launch_assemble(const opm_problem* pb, const double* y, const double* acc0, double dt,
                    double* R, double* J, double* norms, hipStream_t s) {
  const int nblk = blocks_for(pb->n_cells, kBlock);
  Args a;
  a.n = pb->n_cells;
  a.y = y;
  a.acc0 = acc0;
  a.dt = dt;
  a.trans = pb->trans;
  a.pv = pb->pore_vol;
  a.depth = pb->depth;
  a.row_ptr = pb->row_ptr;
  a.col_idx = pb->col_idx;
  a.blk_face = pb->blk_face;
  a.cell_conn_ptr = pb->cell_conn_ptr;
  a.cell_conn = pb->cell_conn;
  a.conn_kind = pb->conn_kind;
  a.conn_phase = pb->conn_phase;
  a.conn_wi = pb->conn_wi;
  a.conn_rate = pb->conn_rate;
  a.conn_bhp = pb->conn_bhp;
  a.fluid = pb->fluid;
  a.R = R;
  a.J = J;
  a.partials = norms ? norms + 8 : nullptr;
  hipLaunchKernelGGL(k_assemble, dim3(nblk), dim3(kBlock), 0, s, a);
  OPM_TRY_HIP(hipGetLastError());
  if (norms) {
    hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(kBlock), 0, s, norms + 8, nblk, pb->n_cells,
                       dt, norms);
    OPM_TRY_HIP(hipGetLastError());
  }
  return OPM_OK;
}

int launch_accumulation(const opm_problem* pb, const double* y, double* acc0, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulation, dim3(blocks_for(pb->n_cells, kBlock)), dim3(kBlock), 0, s,
                     pb->n_cells, pb->fluid, y, acc0);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

}  // namespace opm
