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
// for that code (assemble_dev.h), so the two evaluations are bitwise equal
// and u_ij = -u_ji holds exactly.  The CNV / MB norms are reduced in the same
// pass.
#include <mutex>

#include "assemble_dev.h"

namespace opm {

// Scratch of the allocation-free assembly (opm_assemble_noalloc): the
// per-workgroup partials of the CNV/MB norms, kNormStride doubles for each
// of at most kScratchBlocks workgroups (5 MiB; every GPU the library runs
// on holds one copy until the process ends).  Host code never names the
// array: it uses the device address resolved once per device below.
constexpr int kScratchBlocks = 65536;
static __device__ __align__(256) double scratch[(size_t)kScratchBlocks * kNormStride];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kScratchDevices] = {};

using namespace asmdev;

template <bool LIVE, bool WET = false>
__global__ __launch_bounds__(kBlock) void k_assemble(AsmArgs a) {
  __shared__ double sh[kBlock / kWave];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double part[kNormStride];
#pragma unroll
  for (int k = 0; k < kNormStride; ++k) part[k] = 0.0;
  if (i < a.n) assemble_row<LIVE, WET>(a, i, a.dt, part);
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

// ------------------------------------------------ LDS-tiled assembly
// Dead oil with fixed-source wells (paper sec. 2.4.2 localisation; eqs.
// materialbalance, flux1, head, gwseg, wellinflow).  A workgroup owns an
// 8x8x4 tile of the lattice, one lane per cell.  Phase 1: every lane
// evaluates the properties of its own cell and of one cell of the tile's
// one-cell halo (the 256 face neighbours of the tile) once, and stages what
// the face fluxes need in LDS.  Phase 2, one component at a time: the lane of
// each cell computes the flux of its three faces towards its lower
// neighbours (-x, -y, -z) once, from LDS, keeps -F and its derivatives for
// its own row, and hands F, dF/dy_L and dF/dy_H to the lane of the lower
// cell through LDS; faces towards the halo above the tile are computed by
// the tile's own cells (the neighbouring tile computes the same face from
// the same staged inputs with the same instructions, so the two copies are
// bitwise equal and u_ij = -u_ji holds exactly).  Phase 3: accumulation and
// well terms, then the residual and the block row, written contiguously.
//
// With one Corey curve for k_row and k_rog (opm_fluid.n_corey for every
// curve), eq. gwseg's weighted mean of the two is the curve itself, so the
// oil relative permeability is k_row(s_o) with its own derivatives.
// Floating-point contraction is off for this part: a face on a tile
// boundary is computed by both tiles, whose two copies must round alike.
#pragma clang fp contract(off)
constexpr int kTX = 8, kTY = 8, kTZ = 4;
constexpr int kTile = kTX * kTY * kTZ;                               // 256 lanes
constexpr int kHalo = 2 * (kTY * kTZ + kTX * kTZ + kTX * kTY);       // 256 halo cells
constexpr int kSlots = kTile + kHalo;
static_assert(kTile == kBlock, "one lane per tile cell");

struct TileProps {          // what the faces and the cell terms need of a cell
  double p, sw, sg;
  double b[3];              // b_a(p); d b_a/dp = c_a b_a
  double mv[3];             // b_a k_ra / mu_a; d/dp = c_a mv_a
  double mw1, mo1, mo2, mg2;  // d mv_w/ds_w, d mv_o/ds_w (= d mv_o/ds_g), d mv_g/ds_g
};

struct ClampD {
  double v, d;
};
// clamp to [0, 1]; the argument passes through on the bounds themselves
__device__ __forceinline__ ClampD clamp01d(double v, double d) {
  if (v < 0.0) return {0.0, 0.0};
  if (v > 1.0) return {1.0, 0.0};
  return {v, d};
}
// Corey curve x^n and its derivative with respect to the saturation
__device__ __forceinline__ ClampD corey(ClampD x, double n) {
  if (n == 2.0) return {x.v * x.v, (2.0 * x.v) * x.d};
  return {pow(x.v, n), (n * pow(x.v, n - 1.0)) * x.d};
}

__device__ __forceinline__ void tile_props(const opm_fluid& f, double p, double sw, double sg,
                                           TileProps& P) {
  P.p = p;
  P.sw = sw;
  P.sg = sg;
#pragma unroll
  for (int a = 0; a < 3; ++a) P.b[a] = exp((p - f.p_ref) * f.c[a]);
  const double den = 1.0 - f.swc, rden = 1.0 / den;
  const ClampD krw = corey(clamp01d((sw - f.swc) / den, rden), f.n_corey);
  const ClampD krg = corey(clamp01d(sg / den, rden), f.n_corey);
  const ClampD kro = corey(clamp01d(((1.0 - sw) - sg) / den, -rden), f.n_corey);
  P.mv[0] = P.b[0] * (krw.v / f.mu[0]);
  P.mv[1] = P.b[1] * (kro.v / f.mu[1]);
  P.mv[2] = P.b[2] * (krg.v / f.mu[2]);
  P.mw1 = P.b[0] * (krw.d / f.mu[0]);
  P.mo1 = P.b[1] * (kro.d / f.mu[1]);
  P.mo2 = P.mo1;
  P.mg2 = P.b[2] * (krg.d / f.mu[2]);
}

// Staged per slot for the current component a: b_a, mv_a and its two
// saturation derivatives (p and depth are staged once).  Once the fluxes are
// done the same LDS stages the block rows for the write-out: per wavefront
// (one z-layer of the tile, eight x-runs of eight cells), four x-runs at a
// time, each run's rows contiguous as they are in J.
constexpr int kRunStage = kTX * 7 * 9;   // doubles of the block rows of one x-run
struct TileFaceLds {
  double p[kSlots], z[kSlots];
  double b[kSlots], mv[kSlots], m1[kSlots], m2[kSlots];
  double ex[3][7][kTile];   // face (L, own) of each lane's -x, -y, -z face
  int32_t cell[kSlots];
};
constexpr int kWaveStage = (int)(sizeof(TileFaceLds) / sizeof(double)) / (kTile / kWave);
static_assert(kWaveStage >= 4 * kRunStage, "four x-runs of block rows per wavefront");
struct TileLds {
  union {
    TileFaceLds f;
    double rows[kTile / kWave][kWaveStage];
  } u;
  double red[kBlock / kWave];
};

// Flux of component a from the lower cell L to the upper cell H (eqs. flux1,
// head): F = (b_a lambda_a)_U T dPhi, dPhi = p_L - p_H - g (rho_L + rho_H)/2
// (z_L - z_H), U = L if dPhi >= 0.  out: F, dF/dy_L (3), dF/dy_H (3).
__device__ __forceinline__ void tile_flux(const TileFaceLds& S, int sL, int sH, double T, double rho_s,
                                          double c, double g, double out[7]) {
  const double pL = S.p[sL], pH = S.p[sH];
  const double dz = S.z[sL] - S.z[sH];
  const double rL = rho_s * S.b[sL], rH = rho_s * S.b[sH];
  const double drL = rL * c, drH = rH * c;
  const double dphi = (pL - pH) - (((rL + rH) * 0.5) * g) * dz;
  const double dphi_pL = 1.0 - ((drL * 0.5) * g) * dz;
  const double dphi_pH = -1.0 - ((drH * 0.5) * g) * dz;
  const bool up_L = dphi >= 0.0;
  const int sU = up_L ? sL : sH;
  const double mv = S.mv[sU], m1 = S.m1[sU], m2 = S.m2[sU];
  const double phiT = dphi * T;
  const double mp = (c * mv) * phiT;   // d mob/dp of the upwind cell times dPhi T
  out[0] = mv * phiT;
  out[1] = mv * (dphi_pL * T) + (up_L ? mp : 0.0);
  out[2] = up_L ? m1 * phiT : 0.0;
  out[3] = up_L ? m2 * phiT : 0.0;
  out[4] = mv * (dphi_pH * T) + (up_L ? 0.0 : mp);
  out[5] = up_L ? 0.0 : m1 * phiT;
  out[6] = up_L ? 0.0 : m2 * phiT;
}

struct TileArgs {
  int n, nx, ny, nz, tiles_x, tiles_y;
  const int32_t* box_cell;
  const double* y;
  const double* acc0;
  double dt;
  const double* trans;
  const double* pv;
  const double* depth;
  const int32_t* row_ptr;
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
  double* partials;
};

// Halo slot h (0..255) of a tile: its lattice coordinates relative to the
// tile origin.  Faces -x, +x (8 x 4 each), -y, +y (8 x 4), -z, +z (8 x 8).
__device__ __forceinline__ void halo_coord(int h, int& x, int& y, int& z) {
  if (h < 64) {
    const int q = h & 31;
    x = h < 32 ? -1 : kTX;
    y = q % kTY;
    z = q / kTY;
  } else if (h < 128) {
    const int q = (h - 64) & 31;
    y = h < 96 ? -1 : kTY;
    x = q % kTX;
    z = q / kTX;
  } else {
    const int q = (h - 128) & 63;
    z = h < 192 ? -1 : kTZ;
    x = q % kTX;
    y = q / kTX;
  }
}

__global__ __launch_bounds__(kBlock, 2) void k_assemble_tiled(TileArgs a) {
  __shared__ TileLds S;
  const opm_fluid& f = a.fluid;
  const int l = threadIdx.x;
  const int lx = l % kTX, ly = (l / kTX) % kTY, lz = l / (kTX * kTY);
  const int t = blockIdx.x;
  const int x0 = (t % a.tiles_x) * kTX, y0 = ((t / a.tiles_x) % a.tiles_y) * kTY,
            z0 = (t / (a.tiles_x * a.tiles_y)) * kTZ;
  auto cell_at = [&](int x, int y, int z) -> int {
    if (x < 0 || y < 0 || z < 0 || x >= a.nx || y >= a.ny || z >= a.nz) return -1;
    return a.box_cell[x + a.nx * (y + a.ny * z)];
  };
  // ---- phase 1: properties of the own cell and of one halo cell
  const int c = cell_at(x0 + lx, y0 + ly, z0 + lz);
  int hx, hy, hz;
  halo_coord(l, hx, hy, hz);
  const int ch = cell_at(x0 + hx, y0 + hy, z0 + hz);
  TileProps P, Ph;
  const int cs = c >= 0 ? c : 0, chs = ch >= 0 ? ch : 0;
  tile_props(f, a.y[3 * cs], a.y[3 * cs + 1], a.y[3 * cs + 2], P);
  tile_props(f, a.y[3 * chs], a.y[3 * chs + 1], a.y[3 * chs + 2], Ph);
  S.u.f.p[l] = P.p;
  S.u.f.p[kTile + l] = Ph.p;
  S.u.f.z[l] = a.depth[cs];
  S.u.f.z[kTile + l] = a.depth[chs];
  // slots of the six neighbours: -x, +x, -y, +y, -z, +z
  int nb[6];
  nb[0] = lx > 0 ? l - 1 : kTile + (ly + kTY * lz);
  nb[1] = lx < kTX - 1 ? l + 1 : kTile + 32 + (ly + kTY * lz);
  nb[2] = ly > 0 ? l - kTX : kTile + 64 + (lx + kTX * lz);
  nb[3] = ly < kTY - 1 ? l + kTX : kTile + 96 + (lx + kTX * lz);
  nb[4] = lz > 0 ? l - kTX * kTY : kTile + 128 + (lx + kTX * ly);
  nb[5] = lz < kTZ - 1 ? l + kTX * kTY : kTile + 192 + (lx + kTX * ly);
  S.u.f.cell[l] = c;
  S.u.f.cell[kTile + l] = ch;
  __syncthreads();
  bool has[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) has[d] = c >= 0 && S.u.f.cell[nb[d]] >= 0;
  // block positions in the row: (-z, -y, -x, diag, +x, +y, +z) by column
  const int q0 = c >= 0 ? a.row_ptr[c] : 0;
  int qn[6];
  qn[4] = q0;
  qn[2] = qn[4] + (has[4] ? 1 : 0);
  qn[0] = qn[2] + (has[2] ? 1 : 0);
  const int qd = qn[0] + (has[0] ? 1 : 0);
  qn[1] = qd + 1;
  qn[3] = qn[1] + (has[1] ? 1 : 0);
  qn[5] = qn[3] + (has[3] ? 1 : 0);
  double T[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) T[d] = has[d] ? a.trans[a.blk_face[qn[d]]] : 0.0;
  // a lane computes its lower faces, and its upper faces whose cell is in
  // the halo; the other upper faces arrive from the neighbour's lane
  const bool up_halo[3] = {lx == kTX - 1, ly == kTY - 1, lz == kTZ - 1};

  double blk[6][9];
  double diag[9];
  double r[3];
#pragma unroll
  for (int d = 0; d < 6; ++d)
#pragma unroll
    for (int e = 0; e < 9; ++e) blk[d][e] = 0.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) diag[e] = 0.0;
  // ---- phase 2: face fluxes, one component at a time
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    const double m1 = al == 0 ? P.mw1 : P.mo1, m2 = al == 1 ? P.mo2 : (al == 2 ? P.mg2 : 0.0);
    const double m1h = al == 0 ? Ph.mw1 : Ph.mo1,
                 m2h = al == 1 ? Ph.mo2 : (al == 2 ? Ph.mg2 : 0.0);
    S.u.f.b[l] = P.b[al];
    S.u.f.mv[l] = P.mv[al];
    S.u.f.m1[l] = al == 2 ? 0.0 : m1;
    S.u.f.m2[l] = m2;
    S.u.f.b[kTile + l] = Ph.b[al];
    S.u.f.mv[kTile + l] = Ph.mv[al];
    S.u.f.m1[kTile + l] = al == 2 ? 0.0 : m1h;
    S.u.f.m2[kTile + l] = m2h;
    __syncthreads();
    double ra = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      // lower face in direction k: L = neighbour, H = own
      double F[7];
      tile_flux(S.u.f, nb[2 * k], l, T[2 * k], f.rho_s[al], f.c[al], f.g, F);
      const bool on = has[2 * k];
      if (on) {
        ra -= F[0];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          diag[3 * al + v] -= F[4 + v];
          blk[2 * k][3 * al + v] = -F[1 + v];
        }
      }
      if (nb[2 * k] < kTile) {   // the lower cell is in the tile: hand the face over
#pragma unroll
        for (int e = 0; e < 7; ++e) S.u.f.ex[k][e][nb[2 * k]] = on ? F[e] : 0.0;
      }
      // upper face into the halo: L = own, H = neighbour
      if (up_halo[k]) {
        tile_flux(S.u.f, l, nb[2 * k + 1], T[2 * k + 1], f.rho_s[al], f.c[al], f.g, F);
        if (has[2 * k + 1]) {
          ra += F[0];
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            diag[3 * al + v] += F[1 + v];
            blk[2 * k + 1][3 * al + v] = F[4 + v];
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (!up_halo[k] && has[2 * k + 1]) {   // face (own, upper neighbour) from its lane
        ra += S.u.f.ex[k][0][l];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          diag[3 * al + v] += S.u.f.ex[k][1 + v][l];
          blk[2 * k + 1][3 * al + v] = S.u.f.ex[k][4 + v][l];
        }
      }
    }
    r[al] = ra;
  }
  // ---- phase 3: accumulation, wells, outputs
  double dg[9];   // the diagonal block
#pragma unroll
  for (int e = 0; e < 9; ++e) dg[e] = 0.0;
  double part[kNormStride];
#pragma unroll
  for (int k = 0; k < kNormStride; ++k) part[k] = 0.0;
  if (c >= 0) {
    const double pv = a.pv[c];
    const double w = pv / a.dt;
    const double so = (1.0 - P.sw) - P.sg;
    const double s[3] = {P.sw, so, P.sg};
    // accumulation b_a s_a and its derivatives
    double acc[3][4];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      acc[al][0] = P.b[al] * s[al];
      acc[al][1] = (P.b[al] * f.c[al]) * s[al];
    }
    acc[0][2] = P.b[0];
    acc[0][3] = 0.0;
    acc[1][2] = -P.b[1];
    acc[1][3] = -P.b[1];
    acc[2][2] = 0.0;
    acc[2][3] = P.b[2];
    // residual = accumulation + fluxes (+ wells): the flux sums are added last
    double rr[3], dd[9];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      rr[al] = (acc[al][0] - a.acc0[3 * c + al]) * w;
#pragma unroll
      for (int v = 0; v < 3; ++v) dd[3 * al + v] = acc[al][1 + v] * w;
    }
    for (int tq = a.cell_conn_ptr[c]; tq < a.cell_conn_ptr[c + 1]; ++tq) {
      const int k = a.cell_conn[tq];
      if (a.conn_kind[k] == OPM_WELL_RATE_INJ) {
        const int ph = a.conn_phase[k];
#pragma unroll
        for (int al = 0; al < 3; ++al)
          if (al == ph) rr[al] += a.conn_rate[k];
      } else {
        const double dp = P.p - a.conn_bhp[k];
        if (dp > 0.0) {
          const double wi = a.conn_wi[k];
          const double m1[3] = {P.mw1, P.mo1, 0.0}, m2[3] = {0.0, P.mo2, P.mg2};
#pragma unroll
          for (int al = 0; al < 3; ++al) {
            const double mw = P.mv[al] * wi;
            rr[al] += mw * dp;
            dd[3 * al] += ((f.c[al] * P.mv[al]) * wi) * dp + mw;
            dd[3 * al + 1] += (m1[al] * wi) * dp;
            dd[3 * al + 2] += (m2[al] * wi) * dp;
          }
        }
      }
    }
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      rr[al] += r[al];
#pragma unroll
      for (int v = 0; v < 3; ++v) dg[3 * al + v] = dd[3 * al + v] + diag[3 * al + v];
      a.R[3 * c + al] = rr[al];
    }
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      part[al] = rr[al] == 0.0 ? 0.0 : a.dt * fabs(rr[al]) / (P.b[al] * pv);
      part[3 + al] = rr[al];
      part[6 + al] = P.b[al];
    }
    part[9] = pv;
  }
  if (a.partials) {
    double out[kNormStride];
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = block_max<kBlock>(part[k], S.red);
#pragma unroll
    for (int k = 3; k < kNormStride; ++k) out[k] = block_sum<kBlock>(part[k], S.red);
    if (l < kNormStride) {
      double v = out[0];
#pragma unroll
      for (int k = 1; k < kNormStride; ++k)
        if (l == k) v = out[k];
      a.partials[(size_t)blockIdx.x * kNormStride + l] = v;
    }
  }
  // ---- phase 4: the block rows.  The rows of an x-run of the tile are
  // consecutive in J; each run's rows are staged in LDS in J's order and the
  // wavefront writes the run out as one contiguous range (streaming stores:
  // no block of J is read again by this kernel).
  if (!a.J) return;
  const int wave = l / kWave, lane = l % kWave, run = lane / kTX;
  int nbk = 1;
#pragma unroll
  for (int d = 0; d < 6; ++d) nbk += has[d] ? 1 : 0;
  int qb = c >= 0 ? q0 : 0x7fffffff, qe = c >= 0 ? q0 + nbk : -1;
#pragma unroll
  for (int off = 1; off < kTX; off <<= 1) {
    qb = min(qb, __shfl_xor(qb, off, kWave));
    qe = max(qe, __shfl_xor(qe, off, kWave));
  }
  double* stage = S.u.rows[wave];
  constexpr int order[6] = {4, 2, 0, 1, 3, 5};   // (-z, -y, -x | +x, +y, +z)
#pragma unroll
  for (int pass = 0; pass < kTY / 4; ++pass) {
    __syncthreads();   // LDS free: the fluxes' reads, or the last pass's copy, are done
    if (c >= 0 && run / 4 == pass) {
      double* row = stage + (run % 4) * kRunStage + 9 * (q0 - qb);
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        const int d = order[o];
        if (has[d]) {
#pragma unroll
          for (int e = 0; e < 9; ++e) row[9 * (qn[d] - q0) + e] = blk[d][e];
        }
      }
#pragma unroll
      for (int e = 0; e < 9; ++e) row[9 * (qd - q0) + e] = dg[e];
#pragma unroll
      for (int o = 3; o < 6; ++o) {
        const int d = order[o];
        if (has[d]) {
#pragma unroll
          for (int e = 0; e < 9; ++e) row[9 * (qn[d] - q0) + e] = blk[d][e];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int src = (pass * 4 + r) * kTX;
      const int rb = __shfl(qb, src, kWave), re = __shfl(qe, src, kWave);
      if (rb >= re) continue;   // no active cell in the run (uniform over the wavefront)
      const int len = 9 * (re - rb);
      const double* from = stage + r * kRunStage;
      double* to = a.J + 9 * (size_t)rb;
      // 16-byte stores from the first 16-byte boundary of the range (h: one
      // leading value before it), a trailing value after the last pair
      const int h = (int)(((uintptr_t)to >> 3) & 1u), np = (len - h) / 2;
      if (lane == 0 && h) __builtin_nontemporal_store(from[0], to);
      typedef double Pair __attribute__((ext_vector_type(2)));
      for (int e = lane; e < np; e += kWave) {
        const Pair v = {from[h + 2 * e], from[h + 2 * e + 1]};
        __builtin_nontemporal_store(v, reinterpret_cast<Pair*>(to + h + 2 * e));
      }
      if (lane == 0 && h + 2 * np < len)
        __builtin_nontemporal_store(from[len - 1], to + len - 1);
    }
  }
}

#pragma clang fp contract(fast)

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

template <bool LIVE, bool WET = false>
__global__ __launch_bounds__(kBlock) void k_accumulation(int n, opm_fluid f, const double* y,
                                                          const uint8_t* meaning, double* acc) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  FaceProps P;
  CellAcc A;
  properties<LIVE, WET>(f, y[3 * i], y[3 * i + 1], y[3 * i + 2], LIVE ? meaning[i] : 0, P, &A);
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[3 * i + c] = A.A[c].v;
}

}  // namespace

// Resolve the device address of the scratch array on `device` (which must
// be current); called by opm_init, and by the allocation-free entry point
// on its first call on a device.
int assemble_scratch_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return OPM_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return OPM_OK;
  void* ptr = nullptr;
  OPM_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return OPM_EHIP;
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return OPM_OK;
}

long assemble_noalloc_max_cells() { return (long)kScratchBlocks * kBlock; }

// Assembly kernel selection (OPM_OPT_ASSEMBLY): 1 the LDS-tiled kernel where
// the problem allows it, 0 the row-per-lane kernel.
int g_assembly_kernel = 1;

namespace {
bool use_tiled(const opm_problem* pb, const double* Cw) {
  return g_assembly_kernel == 1 && pb->box_cell && !pb->fluid.live && pb->n_wells == 0 && !Cw &&
         pb->nx > 0 && pb->ny > 0 && pb->nz > 0;
}
long tiles_of(const opm_problem* pb) {
  return (long)((pb->nx + kTX - 1) / kTX) * ((pb->ny + kTY - 1) / kTY) * ((pb->nz + kTZ - 1) / kTZ);
}
}  // namespace

// Workgroups of the assembly (one partial of the norms each).
long assemble_workgroups(const opm_problem* pb, const double* Cw) {
  return use_tiled(pb, Cw) ? tiles_of(pb) : (long)blocks_for(pb->n_cells, kBlock);
}

// The most workgroups either assembly kernel may launch for pb.
long assemble_max_workgroups(const opm_problem* pb) {
  const long rows = blocks_for(pb->n_cells, kBlock);
  const bool tileable = pb->box_cell && pb->nx > 0 && pb->ny > 0 && pb->nz > 0;
  return tileable && tiles_of(pb) > rows ? tiles_of(pb) : rows;
}

int launch_assemble_parts(const opm_problem* pb, const double* y, const double* acc0, double dt,
                          double* R, double* J, double* norms, double* partials, hipStream_t s,
                          double* Cw);

// Assembly with the norms' partials in the library's scratch array: norms
// receives only the 8 results.  The array is shared by every call on the
// device, so calls that overlap on one GPU race.
int launch_assemble_noalloc(const opm_problem* pb, const double* y, const double* acc0, double dt,
                            double* R, double* J, double* norms, hipStream_t s) {
  if (assemble_workgroups(pb, nullptr) > kScratchBlocks) return OPM_EINVAL;
  int dev = 0;
  OPM_TRY_HIP(hipGetDevice(&dev));
  OPM_TRY(assemble_scratch_setup(dev));
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    part = g_scratch_ptr[dev];
  }
  return launch_assemble_parts(pb, y, acc0, dt, R, J, norms, norms ? part : nullptr, s, nullptr);
}

// Cw (standard wells, with J): [n_conns][3][4] derivatives of the cell
// residuals w.r.t. the well unknowns.
int launch_assemble(const opm_problem* pb, const double* y, const double* acc0, double dt,
                    double* R, double* J, double* norms, hipStream_t s, double* Cw) {
  return launch_assemble_parts(pb, y, acc0, dt, R, J, norms, norms ? norms + 8 : nullptr, s, Cw);
}

// norms: the 8 results (or null); partials: kNormStride doubles per
// workgroup of the assembly (null without norms).
int launch_assemble_parts(const opm_problem* pb, const double* y, const double* acc0, double dt,
                          double* R, double* J, double* norms, double* partials, hipStream_t s,
                          double* Cw) {
  if (use_tiled(pb, Cw)) {
    const int nt = (int)tiles_of(pb);
    TileArgs t;
    t.n = pb->n_cells;
    t.nx = pb->nx;
    t.ny = pb->ny;
    t.nz = pb->nz;
    t.tiles_x = (pb->nx + kTX - 1) / kTX;
    t.tiles_y = (pb->ny + kTY - 1) / kTY;
    t.box_cell = pb->box_cell;
    t.y = y;
    t.acc0 = acc0;
    t.dt = dt;
    t.trans = pb->trans;
    t.pv = pb->pore_vol;
    t.depth = pb->depth;
    t.row_ptr = pb->row_ptr;
    t.blk_face = pb->blk_face;
    t.cell_conn_ptr = pb->cell_conn_ptr;
    t.cell_conn = pb->cell_conn;
    t.conn_kind = pb->conn_kind;
    t.conn_phase = pb->conn_phase;
    t.conn_wi = pb->conn_wi;
    t.conn_rate = pb->conn_rate;
    t.conn_bhp = pb->conn_bhp;
    t.fluid = pb->fluid;
    t.R = R;
    t.J = J;
    t.partials = norms ? partials : nullptr;
    hipLaunchKernelGGL(k_assemble_tiled, dim3(nt), dim3(kBlock), 0, s, t);
    OPM_TRY_HIP(hipGetLastError());
    if (norms) {
      hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(kBlock), 0, s, t.partials, nt,
                         pb->n_cells, dt, norms);
      OPM_TRY_HIP(hipGetLastError());
    }
    return OPM_OK;
  }
  const int nblk = blocks_for(pb->n_cells, kBlock);
  AsmArgs a;
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
  a.meaning = pb->meaning;
  a.n_wells = pb->n_wells;
  a.conn_well = pb->conn_well;
  a.well_state = pb->well_state;
  a.Cw = Cw;
  a.R = R;
  a.J = J;
  a.partials = norms ? partials : nullptr;
  if (pb->fluid.live && pb->fluid.rv_c > 0.0)   // wet gas
    hipLaunchKernelGGL((k_assemble<true, true>), dim3(nblk), dim3(kBlock), 0, s, a);
  else if (pb->fluid.live)
    hipLaunchKernelGGL(k_assemble<true>, dim3(nblk), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_assemble<false>, dim3(nblk), dim3(kBlock), 0, s, a);
  OPM_TRY_HIP(hipGetLastError());
  if (norms) {
    hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(kBlock), 0, s, a.partials, nblk, pb->n_cells,
                       dt, norms);
    OPM_TRY_HIP(hipGetLastError());
  }
  return OPM_OK;
}

int launch_accumulation(const opm_problem* pb, const double* y, double* acc0, hipStream_t s) {
  const dim3 grid(blocks_for(pb->n_cells, kBlock));
  if (pb->fluid.live && pb->fluid.rv_c > 0.0)
    hipLaunchKernelGGL((k_accumulation<true, true>), grid, dim3(kBlock), 0, s, pb->n_cells, pb->fluid, y,
                       pb->meaning, acc0);
  else if (pb->fluid.live)
    hipLaunchKernelGGL(k_accumulation<true>, grid, dim3(kBlock), 0, s, pb->n_cells, pb->fluid, y,
                       pb->meaning, acc0);
  else
    hipLaunchKernelGGL(k_accumulation<false>, grid, dim3(kBlock), 0, s, pb->n_cells, pb->fluid, y,
                       pb->meaning, acc0);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

}  // namespace opm
