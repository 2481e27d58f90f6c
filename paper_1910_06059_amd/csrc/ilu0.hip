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
//
// Data layout: everything the sweeps read is in level order (position p of
// the schedule, rows of one level contiguous) and structure-of-arrays
// (element e of row p at [e * ns + p]), so a wavefront reads consecutive
// addresses: the three lower and three upper off-diagonal blocks of each row,
// D^{-1}, and a level-ordered scratch vector z that holds y after the
// forward sweep and x after the backward sweep.  In mixed precision these
// arrays are FP32 while D^{-1} is still computed in FP64.
//
// Launch shapes:
//  - one workgroup walks all levels with workgroup barriers (systems whose
//    widest level is small): the results of the previous level stay in an
//    LDS window, and the matrix data of the next level is loaded before the
//    barrier so that its latency overlaps the current level;
//  - one launch per level over many workgroups (large systems).
// Packing the off-diagonal blocks into level order does not depend on the
// levels and runs as one wide kernel over all rows.
#include "common.h"

namespace opm {
namespace {

constexpr int kWgThreads = 512;        // threads of the one-workgroup sweep
constexpr int kFacThreads = 256;       // threads of the one-workgroup factorisation
constexpr int kMaxWindowRows = 2048;   // widest level served by the one-workgroup sweep
constexpr int kMaxFactorWindowRows = 640;

inline size_t padded(int n) { return ((size_t)n + 63) / 64 * 64; }

template <typename T>
struct IluView {
  int ns;          // SoA stride (n padded to 64)
  double* dinv64;  // [9][ns] FP64 inverse pivots (factor recursion)
  T* dinv;         // [9][ns] sweep copy (aliases dinv64 for FP64)
  T* lov;          // [27][ns] A_ik of the lower neighbours, slot-major
  T* upv;          // [27][ns] A_ij of the upper neighbours
  T* z;            // [3][ns] level-ordered sweep scratch
};

template <typename T>
size_t view_bytes(int n) {
  const size_t ns = padded(n);
  size_t b = sizeof(double) * 9 * ns;
  if (sizeof(T) != sizeof(double)) b += sizeof(T) * 9 * ns;
  return b + sizeof(T) * (27 + 27 + 3) * ns;
}

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
  base += sizeof(T) * 27 * v.ns;
  v.z = (T*)base;
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
  int n, nlev, max_level;
};

Topo topo_of(const opm_problem* pb) {
  return Topo{pb->perm,   pb->diag_pos,  pb->lo_blk,   pb->lo_tblk, pb->lo_pos,
              pb->up_blk, pb->up_pos,    pb->level_ptr, pb->n_cells, pb->n_levels,
              pb->max_level};
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

// ---------------------------------------------------------------- packing
// Level-ordered SoA copies of the off-diagonal blocks (no level dependence).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack(Topo t, const double* J, IluView<T> v) {
  const int pos = blockIdx.x * kBlock + threadIdx.x;
  if (pos >= t.n) return;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int bl = t.lo_blk[3 * pos + s];
    const int bu = t.up_blk[3 * pos + s];
    const double* Al = J + 9 * (size_t)(bl < 0 ? 0 : bl);
    const double* Au = J + 9 * (size_t)(bu < 0 ? 0 : bu);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      v.lov[(size_t)(9 * s + e) * v.ns + pos] = bl < 0 ? (T)0 : (T)Al[e];
      v.upv[(size_t)(9 * s + e) * v.ns + pos] = bu < 0 ? (T)0 : (T)Au[e];
    }
  }
}

// ---------------------------------------------------------- pivot recursion
struct FacJob {
  double D[9];       // A_ii
  double Aik[3][9];  // lower blocks
  double Aki[3][9];  // transposed blocks
  int kp[3];         // level positions of the lower neighbours
};

__device__ __forceinline__ void load_fac(const Topo& t, const double* J, int pos, FacJob& j) {
  const int i = t.perm[pos];
  const double* Aii = J + 9 * (size_t)t.diag_pos[i];
#pragma unroll
  for (int e = 0; e < 9; ++e) j.D[e] = Aii[e];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int b = t.lo_blk[3 * pos + s];
    j.kp[s] = b < 0 ? -1 : t.lo_pos[3 * pos + s];
    const double* A = J + 9 * (size_t)(b < 0 ? 0 : b);
    const double* B = J + 9 * (size_t)(b < 0 ? 0 : t.lo_tblk[3 * pos + s]);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      j.Aik[s][e] = A[e];
      j.Aki[s][e] = B[e];
    }
  }
}

// D = A_ii - sum_k A_ik D_k^{-1} A_ki, then D^{-1}; `dk` fetches D_k^{-1}.
template <typename T, typename DkFn>
__device__ __forceinline__ void finish_fac(const FacJob& j, int pos, IluView<T> v, DkFn dk,
                                           int32_t* status, double* inv) {
  double D[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) D[e] = j.D[e];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    if (j.kp[s] < 0) continue;
    double Dk[9], tmp[9], upd[9];
    dk(j.kp[s], Dk);
    mat3_mul(j.Aik[s], Dk, tmp);   // L_ik = A_ik D_k^{-1}
    mat3_mul(tmp, j.Aki[s], upd);
#pragma unroll
    for (int e = 0; e < 9; ++e) D[e] -= upd[e];
  }
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
__global__ __launch_bounds__(kBlock) void k_factor_level(Topo t, const double* J, IluView<T> v,
                                                          int p0, int p1, int32_t* status) {
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos >= p1) return;
  FacJob j;
  load_fac(t, J, pos, j);
  double inv[9];
  finish_fac<T>(j, pos, v,
                [&](int kp, double* Dk) {
#pragma unroll
                  for (int e = 0; e < 9; ++e) Dk[e] = v.dinv64[(size_t)e * v.ns + kp];
                },
                status, inv);
}

// One workgroup walks all levels.  With WINDOW the inverse pivots of the
// previous level are also kept in LDS (2 buffers of max_level x 9 doubles).
template <typename T, bool WINDOW>
__global__ __launch_bounds__(kFacThreads) void k_factor_wg(Topo t, const double* J, IluView<T> v,
                                                           int32_t* status) {
  extern __shared__ double win[];
  const int L = t.max_level;
  FacJob next;
  int npos = t.level_ptr[0] + threadIdx.x;
  if (npos < t.level_ptr[1]) load_fac(t, J, npos, next);
  int prev0 = 0, prev1 = 0, buf = 0;
  for (int l = 0; l < t.nlev; ++l) {
    const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
    for (int pos = p0 + threadIdx.x; pos < p1; pos += kFacThreads) {
      FacJob cur;
      if (pos == p0 + (int)threadIdx.x)
        cur = next;
      else
        load_fac(t, J, pos, cur);
      double inv[9];
      finish_fac<T>(cur, pos, v,
                    [&](int kp, double* Dk) {
                      if (WINDOW && kp >= prev0 && kp < prev1) {
                        const double* w = win + (size_t)((buf ^ 1) * L + (kp - prev0)) * 9;
#pragma unroll
                        for (int e = 0; e < 9; ++e) Dk[e] = w[e];
                      } else {
#pragma unroll
                        for (int e = 0; e < 9; ++e) Dk[e] = v.dinv64[(size_t)e * v.ns + kp];
                      }
                    },
                    status, inv);
      if (WINDOW) {
        double* w = win + (size_t)(buf * L + (pos - p0)) * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) w[e] = inv[e];
      }
    }
    if (l + 1 < t.nlev) {
      npos = p1 + threadIdx.x;
      if (npos < t.level_ptr[l + 2]) load_fac(t, J, npos, next);
    }
    __syncthreads();
    prev0 = p0;
    prev1 = p1;
    buf ^= 1;
  }
}

// -------------------------------------------------------------- sweeps
template <typename T>
struct SweepJob {
  T a[27];    // three neighbour blocks
  T D[9];     // D^{-1}
  T rhs[3];   // r_i (forward) or y_i (backward)
  int kp[3];  // neighbour positions (-1 if absent)
  int cell;
};

// lower: forward-sweep data of row pos (r gathered from natural order)
template <typename T>
__device__ __forceinline__ void load_fwd(const Topo& t, IluView<T> v, const double* r, int pos,
                                         SweepJob<T>& j) {
  j.cell = t.perm[pos];
#pragma unroll
  for (int c = 0; c < 3; ++c) j.rhs[c] = (T)r[3 * j.cell + c];
#pragma unroll
  for (int s = 0; s < 3; ++s) j.kp[s] = t.lo_pos[3 * pos + s];
#pragma unroll
  for (int e = 0; e < 27; ++e) j.a[e] = v.lov[(size_t)e * v.ns + pos];
#pragma unroll
  for (int e = 0; e < 9; ++e) j.D[e] = v.dinv[(size_t)e * v.ns + pos];
}

template <typename T>
__device__ __forceinline__ void load_bwd(const Topo& t, IluView<T> v, int pos, SweepJob<T>& j) {
  j.cell = t.perm[pos];
#pragma unroll
  for (int c = 0; c < 3; ++c) j.rhs[c] = v.z[(size_t)c * v.ns + pos];
#pragma unroll
  for (int s = 0; s < 3; ++s) j.kp[s] = t.up_pos[3 * pos + s];
#pragma unroll
  for (int e = 0; e < 27; ++e) j.a[e] = v.upv[(size_t)e * v.ns + pos];
#pragma unroll
  for (int e = 0; e < 9; ++e) j.D[e] = v.dinv[(size_t)e * v.ns + pos];
}

// forward: y = D^{-1} (r - sum_s A_s y_{k_s});  backward: x = y - D^{-1} sum_s A_s x_{k_s}
template <typename T, bool FWD, typename NbrFn>
__device__ __forceinline__ void solve_row(const SweepJob<T>& j, NbrFn nbr, T* out) {
  T acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = FWD ? j.rhs[c] : (T)0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    if (j.kp[s] < 0) continue;
    T xv[3];
    nbr(j.kp[s], xv);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T t = j.a[9 * s + 3 * a] * xv[0] + j.a[9 * s + 3 * a + 1] * xv[1] +
                  j.a[9 * s + 3 * a + 2] * xv[2];
      acc[a] = FWD ? acc[a] - t : acc[a] + t;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T d = j.D[3 * a] * acc[0] + j.D[3 * a + 1] * acc[1] + j.D[3 * a + 2] * acc[2];
    out[a] = FWD ? d : j.rhs[a] - d;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd_level(Topo t, IluView<T> v, int p0, int p1,
                                                       const double* r, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos >= p1) return;
  SweepJob<T> j;
  load_fwd(t, v, r, pos, j);
  T y[3];
  solve_row<T, true>(j, [&](int kp, T* xv) {
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[c] = v.z[(size_t)c * v.ns + kp];
  }, y);
#pragma unroll
  for (int c = 0; c < 3; ++c) v.z[(size_t)c * v.ns + pos] = y[c];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bwd_level(Topo t, IluView<T> v, int p0, int p1,
                                                       double* x, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos >= p1) return;
  SweepJob<T> j;
  load_bwd(t, v, pos, j);
  T xo[3];
  solve_row<T, false>(j, [&](int kp, T* xv) {
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[c] = v.z[(size_t)c * v.ns + kp];
  }, xo);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v.z[(size_t)c * v.ns + pos] = xo[c];
    x[3 * j.cell + c] = (double)xo[c];
  }
}

// One workgroup applies the whole preconditioner.  The window holds the
// values of the level just finished (2 buffers of max_level x 3 entries).
template <typename T>
__global__ __launch_bounds__(kWgThreads) void k_apply_wg(Topo t, IluView<T> v, const double* r,
                                                          double* x, const int32_t* skip) {
  if (skip && *skip != 0) return;
  extern __shared__ unsigned char smem[];
  T* win = reinterpret_cast<T*>(smem);
  const int L = t.max_level;
  const int tid = threadIdx.x;
  // ---- forward sweep, levels ascending
  SweepJob<T> next;
  if (t.level_ptr[0] + tid < t.level_ptr[1]) load_fwd(t, v, r, t.level_ptr[0] + tid, next);
  int prev0 = 0, prev1 = 0, buf = 0;
  for (int l = 0; l < t.nlev; ++l) {
    const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
    for (int pos = p0 + tid; pos < p1; pos += kWgThreads) {
      SweepJob<T> cur;
      if (pos == p0 + tid)
        cur = next;
      else
        load_fwd(t, v, r, pos, cur);
      T y[3];
      solve_row<T, true>(cur, [&](int kp, T* xv) {
        if (kp >= prev0 && kp < prev1) {
          const T* w = win + (size_t)((buf ^ 1) * L + (kp - prev0)) * 3;
          xv[0] = w[0];
          xv[1] = w[1];
          xv[2] = w[2];
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) xv[c] = v.z[(size_t)c * v.ns + kp];
        }
      }, y);
      T* w = win + (size_t)(buf * L + (pos - p0)) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[c] = y[c];
        v.z[(size_t)c * v.ns + pos] = y[c];
      }
    }
    if (l + 1 < t.nlev && p1 + tid < t.level_ptr[l + 2]) load_fwd(t, v, r, p1 + tid, next);
    __syncthreads();
    prev0 = p0;
    prev1 = p1;
    buf ^= 1;
  }
  // ---- backward sweep, levels descending; z[pos] turns from y into x
  {
    const int l = t.nlev - 1;
    if (t.level_ptr[l] + tid < t.level_ptr[l + 1]) load_bwd(t, v, t.level_ptr[l] + tid, next);
  }
  prev0 = prev1 = 0;
  for (int l = t.nlev - 1; l >= 0; --l) {
    const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
    for (int pos = p0 + tid; pos < p1; pos += kWgThreads) {
      SweepJob<T> cur;
      if (pos == p0 + tid)
        cur = next;
      else
        load_bwd(t, v, pos, cur);
      T xo[3];
      solve_row<T, false>(cur, [&](int kp, T* xv) {
        if (kp >= prev0 && kp < prev1) {
          const T* w = win + (size_t)((buf ^ 1) * L + (kp - prev0)) * 3;
          xv[0] = w[0];
          xv[1] = w[1];
          xv[2] = w[2];
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) xv[c] = v.z[(size_t)c * v.ns + kp];
        }
      }, xo);
      T* w = win + (size_t)(buf * L + (pos - p0)) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        w[c] = xo[c];
        v.z[(size_t)c * v.ns + pos] = xo[c];
        x[3 * cur.cell + c] = (double)xo[c];
      }
    }
    if (l > 0 && t.level_ptr[l - 1] + tid < p0) load_bwd(t, v, t.level_ptr[l - 1] + tid, next);
    __syncthreads();
    prev0 = p0;
    prev1 = p1;
    buf ^= 1;
  }
}

template <typename T>
size_t apply_lds(const opm_problem* pb) {
  return sizeof(T) * 2 * 3 * (size_t)pb->max_level;
}

size_t factor_lds(const opm_problem* pb) { return sizeof(double) * 2 * 9 * (size_t)pb->max_level; }

bool g_lds_attr_set[4] = {false, false, false, false};

template <typename K>
int allow_lds(K kernel, int slot) {
  if (!g_lds_attr_set[slot]) {
    OPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    g_lds_attr_set[slot] = true;
  }
  return OPM_OK;
}

template <typename T>
int factor_impl(const opm_problem* pb, const double* J, void* ilu, int32_t* status, int mode,
                hipStream_t s) {
  IluView<T> v = view<T>(pb, ilu);
  Topo t = topo_of(pb);
  hipLaunchKernelGGL(k_pack<T>, dim3(blocks_for(pb->n_cells, kBlock)), dim3(kBlock), 0, s, t, J,
                     v);
  if (mode == 0) {
    if (pb->max_level <= kMaxFactorWindowRows) {
      OPM_TRY(allow_lds(k_factor_wg<T, true>, sizeof(T) == 8 ? 0 : 1));
      hipLaunchKernelGGL((k_factor_wg<T, true>), dim3(1), dim3(kFacThreads), factor_lds(pb), s, t,
                         J, v, status);
    } else {
      hipLaunchKernelGGL((k_factor_wg<T, false>), dim3(1), dim3(kFacThreads), 0, s, t, J, v,
                         status);
    }
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
    OPM_TRY(allow_lds(k_apply_wg<T>, sizeof(T) == 8 ? 2 : 3));
    hipLaunchKernelGGL(k_apply_wg<T>, dim3(1), dim3(kWgThreads), apply_lds<T>(pb), s, t, v, r, x,
                       skip);
    OPM_TRY_HIP(hipGetLastError());
    return OPM_OK;
  }
  for (int l = 0; l < pb->n_levels; ++l) {
    const int p0 = pb->level_ptr_h[l], p1 = pb->level_ptr_h[l + 1];
    hipLaunchKernelGGL(k_fwd_level<T>, dim3(blocks_for(p1 - p0, kBlock)), dim3(kBlock), 0, s, t,
                       v, p0, p1, r, skip);
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
  return precision == OPM_PREC_MIXED ? view_bytes<float>(pb->n_cells)
                                     : view_bytes<double>(pb->n_cells);
}

// Sweep shape: one workgroup when the widest level fits the LDS window and
// the system is small enough for one compute unit, else one launch per
// level; g_sweep_mode (set by opm_set_option) forces one of them.
int g_sweep_mode = -1;

int sweep_mode(const opm_problem* pb) {
  if (g_sweep_mode == 0 || g_sweep_mode == 1) {
    if (g_sweep_mode == 0 && pb->max_level > kMaxWindowRows) return 1;
    return g_sweep_mode;
  }
  return pb->max_level <= kMaxWindowRows && pb->n_cells <= 200000 ? 0 : 1;
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
