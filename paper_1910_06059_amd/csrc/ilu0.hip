// Block ILU(0) preconditioner (paper sec. 2.3.1: the default ILU0 with
// BiCGStab, on block-CSR storage).
//
// For a pattern whose graph has no triangles (the 7-point TPFA stencil of a
// Cartesian grid: two neighbours of a cell are never neighbours of each
// other), ILU(0) creates no update of any off-diagonal block, so the factors
// are L_ik = A_ik D_k^{-1} (k < i), U_ij = A_ij (j > i) and the pivot blocks
//   D_i = A_ii - sum_{k<i, k in C(i)} A_ik D_k^{-1} A_ki .
// Only D_i^{-1} has to be computed.  Rows are processed by dependency level
// (all lower neighbours of a row sit on earlier levels), which gives the same
// factors as the natural order.  The triangular solves of M = LU become
//   forward:  y_i = D_i^{-1} (r_i - sum_{k<i} A_ik y_k)        (y = D^{-1} w)
//   backward: x_i = y_i - D_i^{-1} sum_{j>i} A_ij x_j .
// The factor step also copies the off-diagonal blocks of each row into
// level-ordered, structure-of-arrays storage so that the sweeps read them with
// fully coalesced loads; in mixed precision these copies and D^{-1} are FP32.
//
// Two launch shapes: one workgroup that walks all levels with workgroup
// barriers (small systems: no kernel launch per level), or one launch per
// level over many workgroups (large systems).
#include "common.h"

namespace opm {
namespace {

constexpr int kSweepBlock = 1024;

inline size_t padded(int n) { return ((size_t)n + 63) / 64 * 64; }

template <typename T>
struct IluView {
  int ns;          // SoA stride (n padded to 64)
  double* dinv64;  // [9][ns] FP64 pivots' inverses (factor recursion)
  T* dinv;         // [9][ns] sweep copy (aliases dinv64 for FP64)
  T* lov;          // [27][ns] A_ik of the lower neighbours, slot-major
  T* upv;          // [27][ns] A_ij of the upper neighbours
};

template <typename T>
IluView<T> view(const opm_problem* pb, void* ilu) {
  IluView<T> v;
  v.ns = (int)padded(pb->n_cells);
  char* base = (char*)ilu;
  v.dinv64 = (double*)base;
  base += sizeof(double) * 9 * v.ns;
  if (sizeof(T) == sizeof(double)) {
    v.dinv = (T*)v.dinv64;
  } else {
    v.dinv = (T*)base;
    base += sizeof(T) * 9 * v.ns;
  }
  v.lov = (T*)base;
  base += sizeof(T) * 27 * v.ns;
  v.upv = (T*)base;
  return v;
}

struct Topo {
  const int32_t* perm;
  const int32_t* diag_pos;
  const int32_t* lo_blk;
  const int32_t* lo_tblk;
  const int32_t* lo_pos;
  const int32_t* up_blk;
  const int32_t* up_pos;
  const int32_t* level_ptr;
};

Topo topo_of(const opm_problem* pb) {
  return Topo{pb->perm, pb->diag_pos, pb->lo_blk, pb->lo_tblk, pb->lo_pos, pb->up_blk, pb->up_pos,
              pb->level_ptr};
}

// Inverse of a 3x3 block by cofactors; false on a zero or non-finite
// determinant.
__device__ __forceinline__ bool inverse3(const double* a, double* inv) {
  const double c0 = a[4] * a[8] - a[5] * a[7];
  const double c1 = a[5] * a[6] - a[3] * a[8];
  const double c2 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c0 + a[1] * c1 + a[2] * c2;
  if (det == 0.0 || !isfinite(det)) return false;
  const double r = 1.0 / det;
  inv[0] = c0 * r;
  inv[1] = (a[2] * a[7] - a[1] * a[8]) * r;
  inv[2] = (a[1] * a[5] - a[2] * a[4]) * r;
  inv[3] = c1 * r;
  inv[4] = (a[0] * a[8] - a[2] * a[6]) * r;
  inv[5] = (a[2] * a[3] - a[0] * a[5]) * r;
  inv[6] = c2 * r;
  inv[7] = (a[1] * a[6] - a[0] * a[7]) * r;
  inv[8] = (a[0] * a[4] - a[1] * a[3]) * r;
  return true;
}

__device__ __forceinline__ void mat3_mul(const double* A, const double* B, double* C) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

template <typename T>
__device__ __forceinline__ void factor_row(const Topo& t, const double* J, IluView<T> v, int pos,
                                           int32_t* status) {
  const int i = t.perm[pos];
  double D[9];
  const double* Aii = J + 9 * (size_t)t.diag_pos[i];
#pragma unroll
  for (int e = 0; e < 9; ++e) D[e] = Aii[e];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int b = t.lo_blk[3 * pos + s];
    T* dst = v.lov + (size_t)(9 * s) * v.ns + pos;
    if (b < 0) {
#pragma unroll
      for (int e = 0; e < 9; ++e) dst[(size_t)e * v.ns] = (T)0;
      continue;
    }
    const int kpos = t.lo_pos[3 * pos + s];
    const double* Aik = J + 9 * (size_t)b;
    const double* Aki = J + 9 * (size_t)t.lo_tblk[3 * pos + s];
    double Dk[9], tmp[9], upd[9], aik[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      Dk[e] = v.dinv64[(size_t)e * v.ns + kpos];
      aik[e] = Aik[e];
      dst[(size_t)e * v.ns] = (T)aik[e];
    }
    mat3_mul(aik, Dk, tmp);   // L_ik = A_ik D_k^{-1}
    double aki[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) aki[e] = Aki[e];
    mat3_mul(tmp, aki, upd);
#pragma unroll
    for (int e = 0; e < 9; ++e) D[e] -= upd[e];
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int b = t.up_blk[3 * pos + s];
    T* dst = v.upv + (size_t)(9 * s) * v.ns + pos;
    const double* Aij = J + 9 * (size_t)(b < 0 ? 0 : b);
#pragma unroll
    for (int e = 0; e < 9; ++e) dst[(size_t)e * v.ns] = b < 0 ? (T)0 : (T)Aij[e];
  }
  double inv[9];
  if (!inverse3(D, inv)) {
    if (status) *status = OPM_ESINGULAR;
#pragma unroll
    for (int e = 0; e < 9; ++e) inv[e] = 0.0;
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    v.dinv64[(size_t)e * v.ns + pos] = inv[e];
    if (sizeof(T) != sizeof(double)) v.dinv[(size_t)e * v.ns + pos] = (T)inv[e];
  }
}

template <typename T>
__device__ __forceinline__ void fwd_row(const Topo& t, IluView<T> v, int pos, const double* r,
                                        double* x) {
  const int i = t.perm[pos];
  T acc[3] = {(T)r[3 * i], (T)r[3 * i + 1], (T)r[3 * i + 2]};
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int kpos = t.lo_pos[3 * pos + s];
    if (kpos < 0) continue;
    const int k = t.perm[kpos];
    const T yk[3] = {(T)x[3 * k], (T)x[3 * k + 1], (T)x[3 * k + 2]};
    const T* L = v.lov + (size_t)(9 * s) * v.ns + pos;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[a] -= L[(size_t)(3 * a + c) * v.ns] * yk[c];
  }
  const T* Di = v.dinv + pos;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T s = Di[(size_t)(3 * a) * v.ns] * acc[0] + Di[(size_t)(3 * a + 1) * v.ns] * acc[1] +
          Di[(size_t)(3 * a + 2) * v.ns] * acc[2];
    x[3 * i + a] = (double)s;
  }
}

template <typename T>
__device__ __forceinline__ void bwd_row(const Topo& t, IluView<T> v, int pos, double* x) {
  const int i = t.perm[pos];
  T acc[3] = {(T)0, (T)0, (T)0};
  bool any = false;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int jpos = t.up_pos[3 * pos + s];
    if (jpos < 0) continue;
    any = true;
    const int j = t.perm[jpos];
    const T xj[3] = {(T)x[3 * j], (T)x[3 * j + 1], (T)x[3 * j + 2]};
    const T* U = v.upv + (size_t)(9 * s) * v.ns + pos;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[a] += U[(size_t)(3 * a + c) * v.ns] * xj[c];
  }
  if (!any) return;
  const T* Di = v.dinv + pos;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T s = Di[(size_t)(3 * a) * v.ns] * acc[0] + Di[(size_t)(3 * a + 1) * v.ns] * acc[1] +
          Di[(size_t)(3 * a + 2) * v.ns] * acc[2];
    x[3 * i + a] -= (double)s;
  }
}

// ---- one launch per level -------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_factor_level(Topo t, const double* J, IluView<T> v,
                                                          int p0, int p1, int32_t* status) {
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos < p1) factor_row<T>(t, J, v, pos, status);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd_level(Topo t, IluView<T> v, int p0, int p1,
                                                       const double* r, double* x,
                                                       const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos < p1) fwd_row<T>(t, v, pos, r, x);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bwd_level(Topo t, IluView<T> v, int p0, int p1,
                                                       double* x, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos < p1) bwd_row<T>(t, v, pos, x);
}

// ---- one workgroup walks every level --------------------------------------
template <typename T>
__global__ __launch_bounds__(kSweepBlock) void k_factor_wg(Topo t, const double* J, IluView<T> v,
                                                            int nlev, int32_t* status) {
  for (int l = 0; l < nlev; ++l) {
    const int p1 = t.level_ptr[l + 1];
    for (int pos = t.level_ptr[l] + threadIdx.x; pos < p1; pos += kSweepBlock)
      factor_row<T>(t, J, v, pos, status);
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kSweepBlock) void k_apply_wg(Topo t, IluView<T> v, int nlev,
                                                           const double* r, double* x,
                                                           const int32_t* skip) {
  if (skip && *skip != 0) return;
  for (int l = 0; l < nlev; ++l) {
    const int p1 = t.level_ptr[l + 1];
    for (int pos = t.level_ptr[l] + threadIdx.x; pos < p1; pos += kSweepBlock)
      fwd_row<T>(t, v, pos, r, x);
    __syncthreads();
  }
  for (int l = nlev - 1; l >= 0; --l) {
    const int p1 = t.level_ptr[l + 1];
    for (int pos = t.level_ptr[l] + threadIdx.x; pos < p1; pos += kSweepBlock)
      bwd_row<T>(t, v, pos, x);
    __syncthreads();
  }
}

template <typename T>
int factor_impl(const opm_problem* pb, const double* J, void* ilu, int32_t* status, int mode,
                hipStream_t s) {
  IluView<T> v = view<T>(pb, ilu);
  Topo t = topo_of(pb);
  if (mode == 0) {
    hipLaunchKernelGGL(k_factor_wg<T>, dim3(1), dim3(kSweepBlock), 0, s, t, J, v, pb->n_levels,
                       status);
    OPM_TRY_HIP(hipGetLastError());
    return OPM_OK;
  }
  for (int l = 0; l < pb->n_levels; ++l) {
    const int p0 = pb->level_ptr_h[l], p1 = pb->level_ptr_h[l + 1];
    hipLaunchKernelGGL(k_factor_level<T>, dim3(blocks_for(p1 - p0, kBlock)), dim3(kBlock), 0, s,
                       t, J, v, p0, p1, status);
  }
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

template <typename T>
int apply_impl(const opm_problem* pb, void* ilu, const double* r, double* x, int mode,
               hipStream_t s, const int32_t* skip) {
  IluView<T> v = view<T>(pb, ilu);
  Topo t = topo_of(pb);
  if (mode == 0) {
    hipLaunchKernelGGL(k_apply_wg<T>, dim3(1), dim3(kSweepBlock), 0, s, t, v, pb->n_levels, r, x,
                       skip);
    OPM_TRY_HIP(hipGetLastError());
    return OPM_OK;
  }
  for (int l = 0; l < pb->n_levels; ++l) {
    const int p0 = pb->level_ptr_h[l], p1 = pb->level_ptr_h[l + 1];
    hipLaunchKernelGGL(k_fwd_level<T>, dim3(blocks_for(p1 - p0, kBlock)), dim3(kBlock), 0, s, t,
                       v, p0, p1, r, x, skip);
  }
  for (int l = pb->n_levels - 1; l >= 0; --l) {
    const int p0 = pb->level_ptr_h[l], p1 = pb->level_ptr_h[l + 1];
    hipLaunchKernelGGL(k_bwd_level<T>, dim3(blocks_for(p1 - p0, kBlock)), dim3(kBlock), 0, s, t,
                       v, p0, p1, x, skip);
  }
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

}  // namespace

size_t ilu_bytes(const opm_problem* pb, int precision) {
  const size_t ns = padded(pb->n_cells);
  if (precision == OPM_PREC_MIXED) return ns * (9 * sizeof(double) + 63 * sizeof(float));
  return ns * 63 * sizeof(double);
}

// Sweep shape: one workgroup for systems whose widest level fits in a few
// passes of one workgroup, else one launch per level; g_sweep_mode (set by
// opm_set_option) forces one of them.
int g_sweep_mode = -1;

int sweep_mode(const opm_problem* pb) {
  if (g_sweep_mode == 0 || g_sweep_mode == 1) return g_sweep_mode;
  return pb->max_level <= 4 * kSweepBlock && pb->n_cells <= 200000 ? 0 : 1;
}

int ilu_factor(const opm_problem* pb, const double* J, void* ilu, int precision, int32_t* status,
               hipStream_t s) {
  const int mode = sweep_mode(pb);
  if (precision == OPM_PREC_MIXED) return factor_impl<float>(pb, J, ilu, status, mode, s);
  return factor_impl<double>(pb, J, ilu, status, mode, s);
}

// skip (device, may be null): the sweeps return at once while *skip != 0.
int ilu_apply(const opm_problem* pb, void* ilu, int precision, const double* r, double* x,
              hipStream_t s, const int32_t* skip) {
  const int mode = sweep_mode(pb);
  if (precision == OPM_PREC_MIXED) return apply_impl<float>(pb, ilu, r, x, mode, s, skip);
  return apply_impl<double>(pb, ilu, r, x, mode, s, skip);
}

}  // namespace opm
