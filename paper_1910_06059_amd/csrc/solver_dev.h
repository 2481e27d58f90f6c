// Device-side pieces of the block ILU(0) preconditioner and the block-CSR
// product, shared by the single-system kernels (ilu0.hip, krylov.hip) and
// the persistent ensemble kernel (ensemble.hip).  Paper sec. 2.3.1.
//
// Level-ordered structure-of-arrays storage of the factors: element e of row
// position p at [e * ns + p]; see ilu0.hip for the algorithm.
#pragma once

#include "common.h"
#include "wells_dev.h"

namespace opm {
namespace ilu {

__host__ __device__ inline size_t ilu_padded(int n) { return ((size_t)n + 63) / 64 * 64; }

// Sweep records: the 36 values a sweep row needs (its three neighbour
// blocks, then D^{-1}) as 16-byte chunks, chunk-major: value e of position p
// at [((e / kV) * ns + p) * kV + e % kV] with kV = 16 / sizeof(T), so one
// 16-byte load per chunk and lane reads consecutive chunks across lanes.
constexpr int kRecValues = 36;
template <typename T>
struct Vec16 {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
typedef int int4v __attribute__((ext_vector_type(4)));

template <typename T>
struct IluView {
  int ns;          // SoA stride (n padded to 64)
  double* dinv64;  // [9][ns] FP64 inverse pivots (factor recursion)
  T* dinv;         // [9][ns] sweep copy (aliases dinv64 for FP64)
  T* lov;          // [27][ns] A_ik of the lower neighbours, slot-major
  T* upv;          // [27][ns] A_ij of the upper neighbours
  T* z;            // [3][ns] level-ordered sweep scratch
  T* rec_f;        // forward sweep records (lower blocks, D^{-1})
  T* rec_b;        // backward sweep records (upper blocks, D^{-1})
  int4v* idx_f;    // [ns] (lower neighbour positions, row)
  int4v* idx_b;    // [ns] (upper neighbour positions, row)
  T* z4;           // [ns][4] level-ordered sweep scratch of the record sweep
};

template <typename T>
__host__ __device__ inline size_t view_bytes(int n) {
  const size_t ns = ilu_padded(n);
  size_t b = sizeof(double) * 9 * ns;
  if (sizeof(T) != sizeof(double)) b += sizeof(T) * 9 * ns;
  return b + sizeof(T) * (27 + 27 + 3) * ns + sizeof(T) * (2 * kRecValues + 4) * ns +
         2 * sizeof(int4v) * ns;
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
  base += sizeof(T) * 3 * v.ns;
  v.rec_f = (T*)base;
  base += sizeof(T) * kRecValues * v.ns;
  v.rec_b = (T*)base;
  base += sizeof(T) * kRecValues * v.ns;
  v.idx_f = (int4v*)base;
  base += sizeof(int4v) * v.ns;
  v.idx_b = (int4v*)base;
  base += sizeof(int4v) * v.ns;
  v.z4 = (T*)base;
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
  // The rows of level l that a walk takes: [level_ptr[l lstride + s0],
  // level_ptr[l lstride + s1]).  The whole level: lstride 1, s0 0, s1 1; the
  // subdomains [s0, s1) of a block ILU0: level_ptr = sub_level_ptr,
  // lstride = n_sub + 1.
  int lstride, s0, s1;
};

__host__ __device__ inline Topo topo_of(const opm_problem* pb) {
  return Topo{pb->perm,   pb->diag_pos,  pb->lo_blk,   pb->lo_tblk, pb->lo_pos,
              pb->up_blk, pb->up_pos,    pb->level_ptr, pb->n_cells, pb->n_levels,
              pb->max_level, 1, 0, 1};
}

__host__ __device__ inline int lvl_begin(const Topo& t, int l) {
  return t.level_ptr[l * t.lstride + t.s0];
}
__host__ __device__ inline int lvl_end(const Topo& t, int l) {
  return t.level_ptr[l * t.lstride + t.s1];
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
  int npos = lvl_begin(t, 0) + threadIdx.x;
  if (PREFETCH && npos < lvl_end(t, 0)) load_fac(t, J, npos, next);
  int prev0 = 0, prev1 = 0, buf = 0;
  for (int l = 0; l < t.nlev; ++l) {
    const int p0 = lvl_begin(t, l), p1 = lvl_end(t, l);
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
      npos = lvl_begin(t, l + 1) + threadIdx.x;
      if (npos < lvl_end(t, l + 1)) load_fac(t, J, npos, next);
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

// lower: forward-sweep data of row pos (r gathered from natural order).
// Offsets are 32-bit so that addresses stay (uniform base, lane offset).
template <typename T>
__device__ __forceinline__ void load_fwd(const Topo& t, IluView<T> v, const double* r, int pos,
                                         SweepJob<T>& j) {
  const unsigned ns = (unsigned)v.ns, up = (unsigned)pos;
  j.cell = t.perm[up];
#pragma unroll
  for (unsigned c = 0; c < 3; ++c) j.rhs[c] = (T)r[3u * (unsigned)j.cell + c];
#pragma unroll
  for (unsigned s = 0; s < 3; ++s) j.kp[s] = t.lo_pos[3u * up + s];
#pragma unroll
  for (unsigned e = 0; e < 27; ++e) j.a[e] = v.lov[e * ns + up];
#pragma unroll
  for (unsigned e = 0; e < 9; ++e) j.D[e] = v.dinv[e * ns + up];
}

template <typename T>
__device__ __forceinline__ void load_bwd(const Topo& t, IluView<T> v, int pos, SweepJob<T>& j) {
  const unsigned ns = (unsigned)v.ns, up = (unsigned)pos;
  j.cell = t.perm[up];
#pragma unroll
  for (unsigned c = 0; c < 3; ++c) j.rhs[c] = v.z[c * ns + up];
#pragma unroll
  for (unsigned s = 0; s < 3; ++s) j.kp[s] = t.up_pos[3u * up + s];
#pragma unroll
  for (unsigned e = 0; e < 27; ++e) j.a[e] = v.upv[e * ns + up];
#pragma unroll
  for (unsigned e = 0; e < 9; ++e) j.D[e] = v.dinv[e * ns + up];
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
template <typename T, bool FWD>
__device__ __forceinline__ void wg_row(const SweepJob<T>& j, IluView<T> v, double* x, T* win,
                                       int L, int buf, int prev0, int prev1, int p0, int pos) {
  T out[3];
  solve_row<T, FWD>(j, [&](int kp, T* xv) {
    if (kp >= prev0 && kp < prev1) {
      const T* w = win + (unsigned)((buf ^ 1) * L + (kp - prev0)) * 3u;
      xv[0] = w[0];
      xv[1] = w[1];
      xv[2] = w[2];
    } else {
#pragma unroll
      for (unsigned c = 0; c < 3; ++c) xv[c] = v.z[c * (unsigned)v.ns + (unsigned)kp];
    }
  }, out);
  T* w = win + (unsigned)(buf * L + (pos - p0)) * 3u;
#pragma unroll
  for (unsigned c = 0; c < 3; ++c) {
    w[c] = out[c];
    v.z[c * (unsigned)v.ns + (unsigned)pos] = out[c];
    if (!FWD) x[3u * (unsigned)j.cell + c] = (double)out[c];
  }
}

// One sweep (forward: levels ascending; backward: descending) by one
// workgroup; the data of the next level is requested before the current
// level is computed.
template <typename T, int NT, bool FWD>
__device__ __forceinline__ void wg_sweep(const Topo& t, IluView<T> v, const double* r, double* x,
                                         T* win) {
  const int L = t.max_level;
  const int tid = threadIdx.x;
  auto load = [&](int pos, SweepJob<T>& j) {
    if (FWD)
      load_fwd(t, v, r, pos, j);
    else
      load_bwd(t, v, pos, j);
  };
  SweepJob<T> next, cur;
  {
    const int l0 = FWD ? 0 : t.nlev - 1;
    if (lvl_begin(t, l0) + tid < lvl_end(t, l0)) load(lvl_begin(t, l0) + tid, next);
  }
  int prev0 = 0, prev1 = 0, buf = 0;
  for (int k = 0; k < t.nlev; ++k) {
    const int l = FWD ? k : t.nlev - 1 - k;
    const int p0 = lvl_begin(t, l), p1 = lvl_end(t, l);
    cur = next;
    if (k + 1 < t.nlev) {
      const int ln = FWD ? l + 1 : l - 1;
      const int q0 = lvl_begin(t, ln);
      if (q0 + tid < lvl_end(t, ln)) load(q0 + tid, next);
    }
    if (p0 + tid < p1) wg_row<T, FWD>(cur, v, x, win, L, buf, prev0, prev1, p0, p0 + tid);
    for (int pos = p0 + tid + NT; pos < p1; pos += NT) {   // levels wider than the workgroup
      SweepJob<T> j;
      load(pos, j);
      wg_row<T, FWD>(j, v, x, win, L, buf, prev0, prev1, p0, pos);
    }
    __syncthreads();
    prev0 = p0;
    prev1 = p1;
    buf ^= 1;
  }
}

template <typename T, int NT>
__device__ __forceinline__ void apply_levels_wg(const Topo& t, IluView<T> v, const double* r,
                                                double* x, T* win) {
  wg_sweep<T, NT, true>(t, v, r, x, win);
  wg_sweep<T, NT, false>(t, v, r, x, win);
}

// Block SpMV with three block rows per wavefront.  Lane l serves row l / 21
// of the group, block (l % 21) / 3 of that row (and every 7th block after
// it) and output component l % 3, so the 21 lanes of a row read its blocks
// (at most 7 on the 7-point stencil) as one contiguous run of doubles and a
// wavefront reads one contiguous span of the matrix.  The per-block partial
// sums of an output component sit in lanes l, l+3, ..., l+18 and are added in
// block order by the lane of block 0, which returns true and the row and
// component it owns.  Lane 63 and rows past n contribute nothing.  Every lane
// of the wavefront must call it (cross-lane reads).  With standard wells
// (wc.corr non-null) the owning lane subtracts the well corrections of its
// cell's connections: the Schur-complement operator.
constexpr int kSpmvRowsPerWave = 3;

__device__ __forceinline__ bool spmv_group(int n, const int32_t* row_ptr, const int32_t* col,
                                           const double* J, const double* x, int group,
                                           int lane, int& row, int& comp, double& yv,
                                           const WellCorr& wc = WellCorr{nullptr, nullptr,
                                                                         nullptr}) {
  const int rl = lane / 21, rem = lane - 21 * rl;
  const int q = rem / 3;
  comp = rem - 3 * q;
  row = group * kSpmvRowsPerWave + rl;
  double v = 0.0;
  const bool live = lane < 21 * kSpmvRowsPerWave && row < n;
  if (live) {
    const int q1 = row_ptr[row + 1];
    for (int qb = row_ptr[row] + q; qb < q1; qb += 7) {
      const double* B = J + 9 * (size_t)qb + 3 * comp;
      const double* xj = x + 3 * (size_t)col[qb];
      v += B[0] * xj[0] + B[1] * xj[1] + B[2] * xj[2];
    }
  }
  double sum = v;
#pragma unroll
  for (int k = 1; k < 7; ++k) sum += __shfl(v, lane + 3 * k, kWave);
  if (wc.corr && live && q == 0)
    for (int t = wc.ccp[row]; t < wc.ccp[row + 1]; ++t) sum -= wc.corr[3 * (size_t)wc.cc[t] + comp];
  yv = sum;
  return live && q == 0;
}

__host__ __device__ inline int spmv_groups(int n) { return (n + kSpmvRowsPerWave - 1) / kSpmvRowsPerWave; }
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

namespace opm {
namespace ilu {

// ---------------------------------------------------------------------------
// Quad sweep: x = (LU)^{-1} r by one workgroup of NT threads where four lanes
// share one row (NT/4 rows per pass).  Lane q < 3 owns equation q of the row:
// it holds row q of each neighbour block and of D^{-1} (13 values), so a
// row's data is spread over three lanes and each lane can keep the data of
// the next three levels in registers: the loads for level l+3 are issued
// while level l is computed, which hides the memory latency of one level
// behind three levels of work.  The three partial results of a row are
// exchanged inside the quad.  Lane 3 of a quad only takes part in the
// exchange.
template <typename T>
struct QuadJob {
  T a[9];     // row q of the three neighbour blocks: a[3*s + c]
  T d[3];     // row q of D^{-1}
  T rhs;      // r_q (forward) or y_q (backward)
  int kp[3];  // neighbour positions
  int cell;
};

template <typename T, bool FWD>
__device__ __forceinline__ void quad_load(const Topo& t, IluView<T> v, const double* r, int pos,
                                          int q, QuadJob<T>& j) {
  // 32-bit element offsets keep the addresses as (uniform base, lane offset)
  const unsigned qq = q < 3 ? (unsigned)q : 0u;
  const unsigned ns = (unsigned)v.ns, up = (unsigned)pos;
  j.cell = t.perm[up];
  const T* blk = FWD ? v.lov : v.upv;
  const int32_t* kp = FWD ? t.lo_pos : t.up_pos;
#pragma unroll
  for (unsigned s = 0; s < 3; ++s) {
    j.kp[s] = kp[3u * up + s];
#pragma unroll
    for (unsigned c = 0; c < 3; ++c) j.a[3 * s + c] = blk[(9u * s + 3u * qq + c) * ns + up];
  }
#pragma unroll
  for (unsigned c = 0; c < 3; ++c) j.d[c] = v.dinv[(3u * qq + c) * ns + up];
  j.rhs = FWD ? (T)r[3u * (unsigned)j.cell + qq] : v.z[qq * ns + up];
}

// One row by its quad: neighbour values come from the LDS window (previous
// level) or from z; returns this lane's component.  The arithmetic is that of
// solve_row, term by term, so both launch shapes give bitwise equal results.
template <typename T, bool FWD>
__device__ __forceinline__ T quad_row(const QuadJob<T>& j, IluView<T> v, const T* win_prev,
                                      int prev0, int prev1) {
  T acc = FWD ? j.rhs : (T)0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int kp = j.kp[s];
    if (kp < 0) continue;
    T xv[3];
    if (kp >= prev0 && kp < prev1) {
      const T* w = win_prev + (unsigned)(kp - prev0) * 3u;
      xv[0] = w[0];
      xv[1] = w[1];
      xv[2] = w[2];
    } else {
#pragma unroll
      for (unsigned c = 0; c < 3; ++c) xv[c] = v.z[c * (unsigned)v.ns + (unsigned)kp];
    }
    const T t = j.a[3 * s] * xv[0] + j.a[3 * s + 1] * xv[1] + j.a[3 * s + 2] * xv[2];
    acc = FWD ? acc - t : acc + t;
  }
  // exchange the three components of the row inside the quad
  const int base = (threadIdx.x & (kWave - 1)) & ~3;
  const T t0 = __shfl(acc, base + 0, kWave);
  const T t1 = __shfl(acc, base + 1, kWave);
  const T t2 = __shfl(acc, base + 2, kWave);
  const T d = j.d[0] * t0 + j.d[1] * t1 + j.d[2] * t2;
  return FWD ? d : j.rhs - d;
}

template <typename T, bool FWD>
__device__ __forceinline__ void quad_store(IluView<T> v, double* x, T* wcur, int p0, int pos,
                                           int q, int cell, T val) {
  if (q < 3) {
    wcur[(unsigned)(pos - p0) * 3u + (unsigned)q] = val;
    v.z[(unsigned)q * (unsigned)v.ns + (unsigned)pos] = val;
    if (!FWD) x[3u * (unsigned)cell + (unsigned)q] = (double)val;
  }
}

template <typename T, int NT, bool FWD>
__device__ __forceinline__ void quad_level(const Topo& t, IluView<T> v, const double* r, double* x,
                                           T* win, int L, int l, int& prev0, int& prev1, int& buf,
                                           const QuadJob<T>& first) {
  const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
  const int q = threadIdx.x & 3, row0 = threadIdx.x >> 2;
  const T* wprev = win + (size_t)((buf ^ 1) * L) * 3;
  T* wcur = win + (size_t)(buf * L) * 3;
  if (p0 + row0 < p1) {   // first pass: data loaded levels ago
    const T val = quad_row<T, FWD>(first, v, wprev, prev0, prev1);
    quad_store<T, FWD>(v, x, wcur, p0, p0 + row0, q, first.cell, val);
  }
  for (int pos = p0 + row0 + NT / 4; pos < p1; pos += NT / 4) {   // wide levels
    QuadJob<T> j;
    quad_load<T, FWD>(t, v, r, pos, q, j);
    const T val = quad_row<T, FWD>(j, v, wprev, prev0, prev1);
    quad_store<T, FWD>(v, x, wcur, p0, pos, q, j.cell, val);
  }
  __syncthreads();
  prev0 = p0;
  prev1 = p1;
  buf ^= 1;
}

// level index of the k-th step of a sweep (ascending forward, descending backward)
template <bool FWD>
__device__ __forceinline__ int sweep_level(const Topo& t, int k) {
  return FWD ? k : t.nlev - 1 - k;
}

template <typename T, int NT, bool FWD>
__device__ __forceinline__ void quad_prefetch(const Topo& t, IluView<T> v, const double* r, int k,
                                              QuadJob<T>& j) {
  if (k >= t.nlev) return;
  const int l = sweep_level<FWD>(t, k);
  const int pos = t.level_ptr[l] + (threadIdx.x >> 2);
  if (pos < t.level_ptr[l + 1]) quad_load<T, FWD>(t, v, r, pos, threadIdx.x & 3, j);
}

// Three levels in flight (FP32 data fits the register budget of 1024 threads).
template <typename T, int NT, bool FWD>
__device__ __forceinline__ void quad_sweep3(const Topo& t, IluView<T> v, const double* r,
                                            double* x, T* win) {
  const int L = t.max_level;
  int prev0 = 0, prev1 = 0, buf = 0;
  QuadJob<T> ja, jb, jc;
  quad_prefetch<T, NT, FWD>(t, v, r, 0, ja);
  quad_prefetch<T, NT, FWD>(t, v, r, 1, jb);
  quad_prefetch<T, NT, FWD>(t, v, r, 2, jc);
  for (int k = 0; k < t.nlev; k += 3) {
    quad_level<T, NT, FWD>(t, v, r, x, win, L, sweep_level<FWD>(t, k), prev0, prev1, buf, ja);
    quad_prefetch<T, NT, FWD>(t, v, r, k + 3, ja);
    if (k + 1 >= t.nlev) break;
    quad_level<T, NT, FWD>(t, v, r, x, win, L, sweep_level<FWD>(t, k + 1), prev0, prev1, buf, jb);
    quad_prefetch<T, NT, FWD>(t, v, r, k + 4, jb);
    if (k + 2 >= t.nlev) break;
    quad_level<T, NT, FWD>(t, v, r, x, win, L, sweep_level<FWD>(t, k + 2), prev0, prev1, buf, jc);
    quad_prefetch<T, NT, FWD>(t, v, r, k + 5, jc);
  }
}

// Two levels in flight (FP64).
template <typename T, int NT, bool FWD>
__device__ __forceinline__ void quad_sweep2(const Topo& t, IluView<T> v, const double* r,
                                            double* x, T* win) {
  const int L = t.max_level;
  int prev0 = 0, prev1 = 0, buf = 0;
  QuadJob<T> ja, jb;
  quad_prefetch<T, NT, FWD>(t, v, r, 0, ja);
  quad_prefetch<T, NT, FWD>(t, v, r, 1, jb);
  for (int k = 0; k < t.nlev; k += 2) {
    quad_level<T, NT, FWD>(t, v, r, x, win, L, sweep_level<FWD>(t, k), prev0, prev1, buf, ja);
    quad_prefetch<T, NT, FWD>(t, v, r, k + 2, ja);
    if (k + 1 >= t.nlev) break;
    quad_level<T, NT, FWD>(t, v, r, x, win, L, sweep_level<FWD>(t, k + 1), prev0, prev1, buf, jb);
    quad_prefetch<T, NT, FWD>(t, v, r, k + 3, jb);
  }
}

template <typename T, int NT>
__device__ __forceinline__ void apply_levels_quad(const Topo& t, IluView<T> v, const double* r,
                                                  double* x, T* win) {
  if (sizeof(T) == sizeof(double)) {
    quad_sweep2<T, NT, true>(t, v, r, x, win);
    quad_sweep2<T, NT, false>(t, v, r, x, win);
  } else {
    quad_sweep3<T, NT, true>(t, v, r, x, win);
    quad_sweep3<T, NT, false>(t, v, r, x, win);
  }
}

}  // namespace ilu
}  // namespace opm

namespace opm {
namespace ilu {

// Ring capacity (rows, a power of two) that holds every value a sweep can
// still need: a row reads neighbours at most `span` positions away, and the
// rows of one level (at most max_level) write concurrently.
__host__ __device__ inline int ring_rows(int span, int max_level) {
  int c = 1;
  while (c < span + max_level + 1) c <<= 1;
  return c;
}

// One row of a sweep with every neighbour value read from the LDS ring.
template <typename T, bool FWD>
__device__ __forceinline__ void ring_row(const SweepJob<T>& j, IluView<T> v, double* x, T* ring,
                                         unsigned mask, int pos) {
  T out[3];
  solve_row<T, FWD>(j, [&](int kp, T* xv) {
    const T* w = ring + ((unsigned)kp & mask) * 3u;
    xv[0] = w[0];
    xv[1] = w[1];
    xv[2] = w[2];
  }, out);
  T* w = ring + ((unsigned)pos & mask) * 3u;
#pragma unroll
  for (unsigned c = 0; c < 3; ++c) {
    w[c] = out[c];
    if (FWD)
      v.z[c * (unsigned)v.ns + (unsigned)pos] = out[c];
    else
      x[3u * (unsigned)j.cell + c] = (double)out[c];
  }
}

// Rows of level l by the workgroup: the first row of each thread comes from
// registers loaded earlier (`first`), further rows of a wide level are loaded
// here.
template <typename T, int NT, bool FWD, typename LoadFn>
__device__ __forceinline__ void ring_level(const Topo& t, IluView<T> v, double* x, T* ring,
                                           unsigned mask, int l, const SweepJob<T>& first,
                                           LoadFn load) {
  const int tid = threadIdx.x;
  const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
  if (p0 + tid < p1) ring_row<T, FWD>(first, v, x, ring, mask, p0 + tid);
  for (int pos = p0 + tid + NT; pos < p1; pos += NT) {
    SweepJob<T> j;
    load(pos, j);
    ring_row<T, FWD>(j, v, x, ring, mask, pos);
  }
  __syncthreads();
}

// One sweep by one workgroup with the LDS ring: no neighbour value is read
// from global memory, so the only global loads are the row data.  Two
// register sets alternate between levels, and the next level's row data is
// requested before the current level is computed (no register copy, which
// would force the loads to complete).
template <typename T, int NT, bool FWD>
__device__ __forceinline__ void ring_sweep(const Topo& t, IluView<T> v, const double* r, double* x,
                                           T* ring, unsigned mask) {
  const int tid = threadIdx.x;
  auto load = [&](int pos, SweepJob<T>& j) {
    if (FWD)
      load_fwd(t, v, r, pos, j);
    else
      load_bwd(t, v, pos, j);
  };
  auto level_of = [&](int k) { return FWD ? k : t.nlev - 1 - k; };
  auto prefetch = [&](int k, SweepJob<T>& j) {
    if (k >= t.nlev) return;
    const int l = level_of(k);
    const int pos = t.level_ptr[l] + tid;
    if (pos < t.level_ptr[l + 1]) load(pos, j);
  };
  SweepJob<T> ja, jb;
  prefetch(0, ja);
  for (int k = 0; k < t.nlev; k += 2) {
    prefetch(k + 1, jb);
    ring_level<T, NT, FWD>(t, v, x, ring, mask, level_of(k), ja, load);
    if (k + 1 >= t.nlev) break;
    prefetch(k + 2, ja);
    ring_level<T, NT, FWD>(t, v, x, ring, mask, level_of(k + 1), jb, load);
  }
}

template <typename T, int NT>
__device__ __forceinline__ void apply_levels_ring(const Topo& t, IluView<T> v, const double* r,
                                                  double* x, T* ring, unsigned mask) {
  ring_sweep<T, NT, true>(t, v, r, x, ring, mask);
  ring_sweep<T, NT, false>(t, v, r, x, ring, mask);
}

}  // namespace ilu
}  // namespace opm

namespace opm {
namespace ilu {

// ---------------------------------------------------------------------------
// Ring sweep with branch-free prefetch.  The forward sweep takes its
// right-hand side from z4 in level order (gathered there before the sweep),
// so the data of a row are loads at its own level position only and the
// next level's loads never wait for an index; the row's blocks, D^{-1},
// neighbour positions and right-hand side come from the sweep records in
// 16-byte loads (21 per row in FP64, 12 in FP32).  A prefetch clamps the level
// (past the last level: the last level) and the row (lanes past a level's
// end: its last row), so every lane issues the same loads on every path and
// the compiler can wait for exactly the loads a level needs while the next
// level's loads stay in flight; lanes past a level's end recompute its last
// row but store nothing (their early load of that row's z may return the
// owner's later forward result).  Missing neighbours have zero blocks and
// read a zero value, which leaves every sum bitwise unchanged.
template <typename T>
struct RingJob {
  T a[27];    // three neighbour blocks
  T D[9];     // D^{-1}
  T rhs[3];   // level-ordered r (forward) or y (backward)
  int kp[3];  // neighbour positions (-1 if absent)
  int pos;
  int cell;   // backward: output row of x
  bool live;  // the lane owns row pos
};

template <typename T, bool FWD>
__device__ __forceinline__ void ring2_load(const Topo& t, IluView<T> v, int pos, RingJob<T>& j) {
  typedef typename Vec16<T>::type V;
  constexpr unsigned kV = 16 / sizeof(T);
  const unsigned ns = (unsigned)v.ns, up = (unsigned)pos;
  const V* rec = reinterpret_cast<const V*>(FWD ? v.rec_f : v.rec_b);
  const int4v ix = (FWD ? v.idx_f : v.idx_b)[up];
  j.pos = pos;
  j.live = true;
  j.kp[0] = ix.x;
  j.kp[1] = ix.y;
  j.kp[2] = ix.z;
  j.cell = ix.w;
  const V* zr = reinterpret_cast<const V*>(v.z4) + up * (4u / kV);
#pragma unroll
  for (unsigned q = 0; q < 4u / kV; ++q) {
    const V r = zr[q];
#pragma unroll
    for (unsigned l = 0; l < kV; ++l)
      if (q * kV + l < 3u) j.rhs[q * kV + l] = r[l];
  }
#pragma unroll
  for (unsigned c = 0; c < (unsigned)kRecValues / kV; ++c) {
    const V w = rec[c * ns + up];
#pragma unroll
    for (unsigned l = 0; l < kV; ++l) {
      const unsigned e = c * kV + l;
      if (e < 27u)
        j.a[e] = w[l];
      else
        j.D[e - 27u] = w[l];
    }
  }
}

// SKIP: a wavefront with no row in the level issues no load (a branch that
// is uniform over the wavefront).
template <typename T, bool FWD, bool SKIP>
__device__ __forceinline__ void ring2_fetch(const Topo& t, IluView<T> v, int k, RingJob<T>& j) {
  const int kk = k < t.nlev ? k : t.nlev - 1;
  const int l = FWD ? kk : t.nlev - 1 - kk;
  const int p0 = t.level_ptr[l], p1 = t.level_ptr[l + 1];
  j.live = k < t.nlev && p0 + (int)threadIdx.x < p1;
  if (SKIP && __builtin_amdgcn_readfirstlane(p0 + (int)(threadIdx.x & ~63u)) >= p1) return;
  const int pos = min(p0 + (int)threadIdx.x, p1 - 1);
  ring2_load<T, FWD>(t, v, pos, j);
  j.live = k < t.nlev && p0 + (int)threadIdx.x < p1;
}

template <typename T, bool FWD, bool SKIP = false>
__device__ __forceinline__ void ring2_row(const RingJob<T>& j, IluView<T> v, double* x, T* ring,
                                          unsigned mask) {
  if (SKIP && !j.live) return;
  T acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = FWD ? j.rhs[c] : (T)0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int kp = j.kp[s];
    const T* w = ring + ((unsigned)kp & mask) * 3u;
    const bool has = kp >= 0;
    const T x0 = has ? w[0] : (T)0, x1 = has ? w[1] : (T)0, x2 = has ? w[2] : (T)0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T t = j.a[9 * s + 3 * a] * x0 + j.a[9 * s + 3 * a + 1] * x1 +
                  j.a[9 * s + 3 * a + 2] * x2;
      acc[a] = FWD ? acc[a] - t : acc[a] + t;
    }
  }
  T out[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T d = j.D[3 * a] * acc[0] + j.D[3 * a + 1] * acc[1] + j.D[3 * a + 2] * acc[2];
    out[a] = FWD ? d : j.rhs[a] - d;
  }
  if (!j.live) return;
  T* w = ring + ((unsigned)j.pos & mask) * 3u;
#pragma unroll
  for (unsigned c = 0; c < 3; ++c) w[c] = out[c];
  if (FWD) {
    typedef typename Vec16<T>::type V;
    constexpr unsigned kV = 16 / sizeof(T);
    const T o4[4] = {out[0], out[1], out[2], (T)0};
    V* zr = reinterpret_cast<V*>(v.z4) + (unsigned)j.pos * (4u / kV);
#pragma unroll
    for (unsigned q = 0; q < 4u / kV; ++q) {
      V r;
#pragma unroll
      for (unsigned l = 0; l < kV; ++l) r[l] = o4[q * kV + l];
      zr[q] = r;
    }
  } else {
#pragma unroll
    for (unsigned c = 0; c < 3; ++c) x[3u * (unsigned)j.cell + c] = (double)out[c];
  }
}

// Rows of level index k beyond the first NT (levels wider than the workgroup).
template <typename T, int NT, bool FWD>
__device__ __forceinline__ void ring2_extra(const Topo& t, IluView<T> v, double* x, T* ring,
                                            unsigned mask, int k) {
  const int l = FWD ? k : t.nlev - 1 - k;
  const int p1 = t.level_ptr[l + 1];
  for (int pos = t.level_ptr[l] + NT + (int)threadIdx.x; pos < p1; pos += NT) {
    RingJob<T> j;
    ring2_load<T, FWD>(t, v, pos, j);
    ring2_row<T, FWD>(j, v, x, ring, mask);
  }
}

// WIDE: some level has more rows than the workgroup has threads.
template <typename T, int NT, bool FWD, bool WIDE, bool SKIP>
__device__ __forceinline__ void ring2_sweep(const Topo& t, IluView<T> v, double* x, T* ring,
                                            unsigned mask) {
  RingJob<T> ja, jb;
  ring2_fetch<T, FWD, SKIP>(t, v, 0, ja);
  for (int k = 0; k < t.nlev; k += 2) {
    ring2_fetch<T, FWD, SKIP>(t, v, k + 1, jb);
    ring2_row<T, FWD, SKIP>(ja, v, x, ring, mask);
    if (WIDE) ring2_extra<T, NT, FWD>(t, v, x, ring, mask, k);
    __syncthreads();
    if (k + 1 >= t.nlev) break;
    ring2_fetch<T, FWD, SKIP>(t, v, k + 2, ja);
    ring2_row<T, FWD, SKIP>(jb, v, x, ring, mask);
    if (WIDE) ring2_extra<T, NT, FWD>(t, v, x, ring, mask, k + 1);
    __syncthreads();
  }
}

}  // namespace ilu
}  // namespace opm
