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

int launch_assemble_parts(const opm_problem* pb, const double* y, const double* acc0, double dt,
                          double* R, double* J, double* norms, double* partials, hipStream_t s,
                          double* Cw);

// Assembly with the norms' partials in the library's scratch array: norms
// receives only the 8 results.  The array is shared by every call on the
// device, so calls that overlap on one GPU race.
int launch_assemble_noalloc(const opm_problem* pb, const double* y, const double* acc0, double dt,
                            double* R, double* J, double* norms, hipStream_t s) {
  if ((long)pb->n_cells > assemble_noalloc_max_cells()) return OPM_EINVAL;
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
