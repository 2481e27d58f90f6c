// Device-side pieces of the block ILU(0) preconditioner and the block-CSR
// product, shared by the single-system kernels (ilu0.hip, krylov.hip) and
// the persistent ensemble kernel (ensemble.hip).  Paper sec. 2.3.1.
//
// Level-ordered structure-of-arrays storage of the factors: element e of row
// position p at [e * ns + p]; see ilu0.hip for the algorithm.
#pragma once

#include "common.h"

namespace opm {
namespace ilu {

__host__ __device__ inline size_t ilu_padded(int n) { return ((size_t)n + 63) / 64 * 64; }

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
__host__ __device__ inline size_t view_bytes(int n) {
  const size_t ns = ilu_padded(n);
  size_t b = sizeof(double) * 9 * ns;
  if (sizeof(T) != sizeof(double)) b += sizeof(T) * 9 * ns;
  return b + sizeof(T) * (27 + 27 + 3) * ns;
}

template <typename T>
__host__ __device__ inline IluView<T> view(const opm_problem* pb, void* ilu) {
  IluView<T> v;
  v.ns = (int)ilu_padded(pb->n_cells);
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

__host__ __device__ inline Topo topo_of(const opm_problem* pb) {
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

// Level-ordered SoA copy of the off-diagonal blocks of one row position.
template <typename T>
__device__ __forceinline__ void pack_row(const Topo& t, const double* J, IluView<T> v, int pos) {
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

// Pivot recursion of all levels by one workgroup of NT threads.  With WINDOW
// the inverse pivots of the previous level are also kept in LDS (`win`: 2
// buffers of max_level x 9 doubles); with PREFETCH the next level's blocks
// are loaded before the barrier (it needs registers for two rows).
template <typename T, bool WINDOW, int NT, bool PREFETCH = true>
__device__ __forceinline__ void factor_levels_wg(const Topo& t, const double* J, IluView<T> v,
                                                 int32_t* status, double* win) {
  const int L = t.max_level;
  FacJob next;
  int npos = t.level_ptr[0] + threadIdx.x;
  if (PREFETCH && npos < t.level_ptr[1]) load_fac(t, J, npos, next);
  int prev0 = 0, prev1 = 0, buf = 0;
  for (int l = 0; l < t.nlev; ++l) {
    const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
    for (int pos = p0 + threadIdx.x; pos < p1; pos += NT) {
      FacJob cur;
      if (PREFETCH && pos == p0 + (int)threadIdx.x)
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
    if (PREFETCH && l + 1 < t.nlev) {
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

// x = (LU)^{-1} r by one workgroup of NT threads: forward sweep over the
// levels ascending, backward sweep descending; the values of the level just
// finished stay in the LDS window `win` (2 buffers of max_level x 3 entries),
// the next level's data is loaded before the barrier.
template <typename T, int NT>
__device__ __forceinline__ void apply_levels_wg(const Topo& t, IluView<T> v, const double* r,
                                                double* x, T* win) {
  const int L = t.max_level;
  const int tid = threadIdx.x;
  SweepJob<T> next;
  if (t.level_ptr[0] + tid < t.level_ptr[1]) load_fwd(t, v, r, t.level_ptr[0] + tid, next);
  int prev0 = 0, prev1 = 0, buf = 0;
  for (int l = 0; l < t.nlev; ++l) {
    const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
    for (int pos = p0 + tid; pos < p1; pos += NT) {
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
  {
    const int l = t.nlev - 1;
    if (t.level_ptr[l] + tid < t.level_ptr[l + 1]) load_bwd(t, v, t.level_ptr[l] + tid, next);
  }
  prev0 = prev1 = 0;
  for (int l = t.nlev - 1; l >= 0; --l) {
    const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
    for (int pos = p0 + tid; pos < p1; pos += NT) {
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

// One block row of y = J x (3 outputs).
__device__ __forceinline__ void spmv_row(const int32_t* row_ptr, const int32_t* col,
                                         const double* J, const double* x, int i, double* y3) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
    const int j = col[q];
    const double* B = J + 9 * (size_t)q;
    const double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
    a0 += B[0] * x0 + B[1] * x1 + B[2] * x2;
    a1 += B[3] * x0 + B[4] * x1 + B[5] * x2;
    a2 += B[6] * x0 + B[7] * x1 + B[8] * x2;
  }
  y3[0] = a0;
  y3[1] = a1;
  y3[2] = a2;
}

}  // namespace ilu
}  // namespace opm
