// Case set-up on the device, once per case: transmissibilities (paper
// appendix B), pore volumes and depths (sec. 2.1.4), Peaceman well indices
// and fixed injection sources of the well connections (sec. 2.2.1).
#include <cmath>

#include "common.h"

namespace opm {
namespace {

__device__ __forceinline__ double layer_top(const double* dz, int k) {
  double z = 0.0;
  for (int q = 0; q < k; ++q) z += dz[q];
  return z;
}

// For axis-aligned cells the half-transmissibility of appendix B reduces to
// t = |F| k / (d/2): the cell-centre-to-face vector is parallel to the face
// normal and has length d/2.
__global__ __launch_bounds__(kBlock) void k_trans(int nx, int ny, double dx, double dy,
                                                   const double* dz, const double* perm,
                                                   double kv_kh, int nf, const int32_t* cell_box,
                                                   const int32_t* face_cells,
                                                   const int32_t* face_dir, double* trans) {
  const int f = blockIdx.x * kBlock + threadIdx.x;
  if (f >= nf) return;
  const int lo = face_cells[2 * f], hi = face_cells[2 * f + 1];
  const int k = cell_box[lo] / (nx * ny);
  const int dir = face_dir[f];
  double area, dl, dh, kl = perm[lo], kh = perm[hi];
  if (dir == 0) {
    area = dy * dz[k];
    dl = dh = dx;
  } else if (dir == 1) {
    area = dx * dz[k];
    dl = dh = dy;
  } else {
    area = dx * dy;
    dl = dz[k];
    dh = dz[k + 1];
    kl *= kv_kh;
    kh *= kv_kh;
  }
  const double tl = area * kl / (0.5 * dl);
  const double th = area * kh / (0.5 * dh);
  trans[f] = (tl + th > 0.0) ? tl * th / (tl + th) : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_cells(int nx, int ny, double dx, double dy,
                                                   const double* dz, const double* poro, int n,
                                                   const int32_t* cell_box, double* pv,
                                                   double* depth) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  const int k = cell_box[c] / (nx * ny);
  pv[c] = poro[c] * (dx * dy * dz[k]);
  depth[c] = layer_top(dz, k) + 0.5 * dz[k];
}

__global__ __launch_bounds__(kBlock) void k_well_index(
    int nx, int ny, double dx, double dy, const double* dz, const double* perm,
    const int32_t* cell_box, const int32_t* well_kind, const int32_t* well_phase,
    const double* well_target, const double* well_rw, int nc, const int32_t* conn_cell,
    const int32_t* conn_well, double* conn_wi, double* conn_rate, int32_t* conn_kind,
    int32_t* conn_phase, double* conn_bhp) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= nc) return;
  const double ro = 0.14 * sqrt(dx * dx + dy * dy);
  auto wi_of = [&](int t) {
    const int c = conn_cell[t];
    const int k = cell_box[c] / (nx * ny);
    return 2.0 * M_PI * perm[c] * dz[k] / log(ro / well_rw[conn_well[t]]);
  };
  const int w = conn_well[q];
  const double wi = wi_of(q);
  double wsum = 0.0;   // connections of one well, in connection order
  for (int t = 0; t < nc; ++t)
    if (conn_well[t] == w) wsum += wi_of(t);
  conn_wi[q] = wi;
  conn_kind[q] = well_kind[w];
  conn_phase[q] = well_phase[w];
  const bool inj = well_kind[w] == OPM_WELL_RATE_INJ;
  conn_rate[q] = inj ? -well_target[w] * wi / wsum : 0.0;
  conn_bhp[q] = inj ? 0.0 : well_target[w];
}

}  // namespace
}  // namespace opm

using namespace opm;

extern "C" int opm_geometry(int32_t nx, int32_t ny, int32_t nz, double dx, double dy,
                            const double* dz, const double* perm_h, double kv_kh,
                            const double* poro, int32_t n_cells, int32_t n_faces,
                            const int32_t* cell_box, const int32_t* face_cells,
                            const int32_t* face_dir, double* trans, double* pore_vol,
                            double* depth, void* stream) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || n_cells < 0 || n_faces < 0 || !dz || !perm_h || !poro ||
      !cell_box || !pore_vol || !depth || (n_faces > 0 && (!face_cells || !face_dir || !trans)))
    return OPM_EINVAL;
  hipStream_t s = as_stream(stream);
  if (n_faces > 0) {
    hipLaunchKernelGGL(k_trans, dim3(blocks_for(n_faces, kBlock)), dim3(kBlock), 0, s, nx, ny, dx,
                       dy, dz, perm_h, kv_kh, n_faces, cell_box, face_cells, face_dir, trans);
    OPM_TRY_HIP(hipGetLastError());
  }
  if (n_cells > 0) {
    hipLaunchKernelGGL(k_cells, dim3(blocks_for(n_cells, kBlock)), dim3(kBlock), 0, s, nx, ny, dx,
                       dy, dz, poro, n_cells, cell_box, pore_vol, depth);
    OPM_TRY_HIP(hipGetLastError());
  }
  return OPM_OK;
}

extern "C" int opm_well_index(int32_t nx, int32_t ny, double dx, double dy, const double* dz,
                              const double* perm_h, const int32_t* cell_box, int32_t n_wells,
                              const int32_t* well_kind, const int32_t* well_phase,
                              const double* well_target, const double* well_rw, int32_t n_conns,
                              const int32_t* conn_cell, const int32_t* conn_well,
                              double* conn_wi, double* conn_rate, int32_t* conn_kind,
                              int32_t* conn_phase, double* conn_bhp, void* stream) {
  if (n_conns < 0 || n_wells < 0) return OPM_EINVAL;
  if (n_conns == 0) return OPM_OK;
  if (!dz || !perm_h || !cell_box || !well_kind || !well_phase || !well_target || !well_rw ||
      !conn_cell || !conn_well || !conn_wi || !conn_rate || !conn_kind || !conn_phase || !conn_bhp)
    return OPM_EINVAL;
  hipLaunchKernelGGL(k_well_index, dim3(blocks_for(n_conns, kBlock)), dim3(kBlock), 0,
                     as_stream(stream), nx, ny, dx, dy, dz, perm_h, cell_box, well_kind,
                     well_phase, well_target, well_rw, n_conns, conn_cell, conn_well, conn_wi,
                     conn_rate, conn_kind, conn_phase, conn_bhp);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}
