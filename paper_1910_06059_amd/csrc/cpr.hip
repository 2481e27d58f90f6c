// CPR-AMG on the device (paper sec. 2.3.1: the two-stage constrained-
// pressure-residual preconditioner with an AMG for the pressure system).
//
// Setup, once per Jacobian: quasi-IMPES weights w_i with D_i^T w_i = e_p
// (D_i the diagonal block of row i), the pressure matrix (A_p)_ij =
// w_i^T A_ij e_p on the block pattern, the Galerkin coarse matrices of the
// aggregation hierarchy (each coarse entry the sum of its gather list of
// fine entries, in a fixed order) and the inverse of the coarsest matrix
// (Gauss-Jordan with partial pivoting, at most 64 unknowns).
// Application, z = CPR(r): b_0 = w^T r; one V(1,1) cycle (damped Jacobi,
// omega = 2/3, before and after the coarse correction; the coarsest level
// by its inverse) gives x_p; x1 = e_p x_p; z = x1 + M_ILU^{-1} (r - A x1)
// with the (block-)ILU(0) factors of A.
//
// Every kernel is a gather (no atomics), so results are the same on every
// run.  Contraction is off in this file: the 3x3 weight solves and the
// sparse products round like plain multiply-then-add code.
#include <cstring>

#include "cpr_dev.h"

#pragma clang fp contract(off)

namespace opm {

int ilu_apply(const opm_problem* pb, void* ilu, int precision, const double* r, double* x,
              hipStream_t s, const int32_t* skip);

namespace {

constexpr double kOmega = 2.0 / 3.0;

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Gaussian elimination with partial pivoting on a 3x3 system (A row-major,
// b overwritten by the solution); false on a zero pivot.
__device__ bool solve3(double* A, double* b) {
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(A[r * 3 + col]) > fabs(A[piv * 3 + col])) piv = r;
    if (A[piv * 3 + col] == 0.0) return false;
    if (piv != col) {
      for (int c = 0; c < 3; ++c) {
        const double t = A[col * 3 + c];
        A[col * 3 + c] = A[piv * 3 + c];
        A[piv * 3 + c] = t;
      }
      const double t = b[col];
      b[col] = b[piv];
      b[piv] = t;
    }
    for (int r = col + 1; r < 3; ++r) {
      const double f = A[r * 3 + col] / A[col * 3 + col];
      if (f == 0.0) continue;
      for (int c = col; c < 3; ++c) A[r * 3 + c] -= f * A[col * 3 + c];
      b[r] -= f * b[col];
    }
  }
  for (int r = 2; r >= 0; --r) {
    double s = b[r];
    for (int c = r + 1; c < 3; ++c) s -= A[r * 3 + c] * b[c];
    b[r] = s / A[r * 3 + r];
  }
  return true;
}

// Weights and the level-0 pressure matrix (one lane per cell).
__global__ __launch_bounds__(kBlock) void k_cpr_weights(int n, const int32_t* row_ptr,
                                                         const int32_t* diag_pos, const double* J,
                                                         double* w, double* a0, double* d0,
                                                         int32_t* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double* D = J + 9 * (size_t)diag_pos[i];
  double T[9] = {D[0], D[3], D[6], D[1], D[4], D[7], D[2], D[5], D[8]};   // D^T
  double e[3] = {1.0, 0.0, 0.0};
  if (!solve3(T, e)) flags[0] = OPM_ESINGULAR;
  w[3 * i] = e[0];
  w[3 * i + 1] = e[1];
  w[3 * i + 2] = e[2];
  for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
    const double* B = J + 9 * (size_t)q;
    double v = 0.0;
    for (int a = 0; a < 3; ++a) v += e[a] * B[3 * a];
    a0[q] = v;
  }
  d0[i] = a0[diag_pos[i]];
}

// One coarse level's matrix by its gather lists (one lane per entry).
__global__ __launch_bounds__(kBlock) void k_cpr_galerkin(int nnz, const int32_t* gptr,
                                                          const int32_t* gmap, const double* fine,
                                                          double* coarse) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= nnz) return;
  double s = 0.0;
  for (int t = gptr[e]; t < gptr[e + 1]; ++t) s += fine[gmap[t]];
  coarse[e] = s;
}

__global__ __launch_bounds__(kBlock) void k_cpr_diag(int n, const int32_t* dpos, const double* a,
                                                      double* d) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) d[i] = a[dpos[i]];
}

// Inverse of the coarsest matrix (n <= 64) by Gauss-Jordan elimination with
// partial pivoting on [A | I] (M: n x 2n working copy), one workgroup.
constexpr int kGjThreads = 256;
__global__ __launch_bounds__(kGjThreads) void k_cpr_inverse(int n, const int32_t* row_ptr,
                                                             const int32_t* col, const double* a,
                                                             double* M, double* inv,
                                                             int32_t* flags) {
  __shared__ int piv, bad;
  const int t = threadIdx.x, w2 = 2 * n;
  for (int k = t; k < n * w2; k += kGjThreads) M[k] = 0.0;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int i = t; i < n; i += kGjThreads) {
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) M[i * w2 + col[q]] = a[q];
    M[i * w2 + n + i] = 1.0;
  }
  __syncthreads();
  for (int c0 = 0; c0 < n; ++c0) {
    if (t == 0) {
      int p = c0;
      for (int r = c0 + 1; r < n; ++r)
        if (fabs(M[r * w2 + c0]) > fabs(M[p * w2 + c0])) p = r;
      piv = p;
      if (M[p * w2 + c0] == 0.0) bad = 1;
    }
    __syncthreads();
    if (bad) break;   // uniform across the workgroup
    const int p = piv;
    if (p != c0)
      for (int c = c0 + t; c < w2; c += kGjThreads) {
        const double v = M[c0 * w2 + c];
        M[c0 * w2 + c] = M[p * w2 + c];
        M[p * w2 + c] = v;
      }
    __syncthreads();
    // every other row loses its multiple of the pivot row; column c0 itself
    // is never read again, so only the columns right of it are updated
    const int width = w2 - c0 - 1;
    for (int k = t; k < n * width; k += kGjThreads) {
      const int r = k / width, c = c0 + 1 + k % width;
      if (r == c0) continue;
      const double f = M[r * w2 + c0] / M[c0 * w2 + c0];
      M[r * w2 + c] -= f * M[c0 * w2 + c];
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) flags[0] = OPM_ESINGULAR;
    return;
  }
  for (int k = t; k < n * n; k += kGjThreads) {
    const int r = k / n, c = k % n;
    inv[k] = M[r * w2 + n + c] / M[r * w2 + r];
  }
}

// b_0 = w^T r (one lane per cell).
__global__ __launch_bounds__(kBlock) void k_cpr_rhs(int n, const double* w, const double* r,
                                                     double* b, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  b[i] = w[3 * i] * r[3 * i] + w[3 * i + 1] * r[3 * i + 1] + w[3 * i + 2] * r[3 * i + 2];
}

// Pre-smoothing from zero: x = omega D^{-1} b.
__global__ __launch_bounds__(kBlock) void k_cpr_smooth0(int n, const double* b, const double* d,
                                                         double* x, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = kOmega * b[i] / d[i];
}

__device__ __forceinline__ double row_mv(const int32_t* row_ptr, const int32_t* col,
                                         const double* a, const double* x, int i) {
  double s = 0.0;
  for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) s += a[q] * x[col[q]];
  return s;
}

// The restricted residual: b_c[I] = sum over the children i of I of
// (b - A x)_i, children ascending (one lane per coarse unknown).
__global__ __launch_bounds__(kBlock) void k_cpr_restrict(int nc, const int32_t* child_ptr,
                                                          const int32_t* child,
                                                          const int32_t* row_ptr,
                                                          const int32_t* col, const double* a,
                                                          const double* b, const double* x,
                                                          double* bc, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int I = blockIdx.x * kBlock + threadIdx.x;
  if (I >= nc) return;
  double s = 0.0;
  for (int t = child_ptr[I]; t < child_ptr[I + 1]; ++t) {
    const int i = child[t];
    s += b[i] - row_mv(row_ptr, col, a, x, i);
  }
  bc[I] = s;
}

// Coarsest level: x = A^{-1} b (one lane per row).
__global__ __launch_bounds__(64) void k_cpr_coarse(int n, const double* inv, const double* b,
                                                    double* x, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int i = threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < n; ++c) s += inv[i * n + c] * b[c];
  x[i] = s;
}

// Coarse correction: x_i += x_c[agg i].
__global__ __launch_bounds__(kBlock) void k_cpr_prolong(int n, const int32_t* agg,
                                                         const double* xc, double* x,
                                                         const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] += xc[agg[i]];
}

// Post-smoothing: y = x + omega D^{-1} (b - A x).
__global__ __launch_bounds__(kBlock) void k_cpr_smooth(int n, const int32_t* row_ptr,
                                                        const int32_t* col, const double* a,
                                                        const double* d, const double* b,
                                                        const double* x, double* y,
                                                        const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = x[i] + kOmega * (b[i] - row_mv(row_ptr, col, a, x, i)) / d[i];
}

// Second-stage residual r2 = r - A x1 with x1 = (x_p, 0, 0) per cell.
__global__ __launch_bounds__(kBlock) void k_cpr_r2(int n, const int32_t* row_ptr,
                                                    const int32_t* col, const double* J,
                                                    const double* r, const double* xp,
                                                    double* r2, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
    const double* B = J + 9 * (size_t)q;
    const double xj = xp[col[q]];
    t0 += B[0] * xj;
    t1 += B[3] * xj;
    t2 += B[6] * xj;
  }
  r2[3 * i] = r[3 * i] - t0;
  r2[3 * i + 1] = r[3 * i + 1] - t1;
  r2[3 * i + 2] = r[3 * i + 2] - t2;
}

// z += x1.
__global__ __launch_bounds__(kBlock) void k_cpr_add(int n, const double* xp, double* z,
                                                     const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) z[3 * i] += xp[i];
}

const int32_t* level_rows(const opm_problem* pb, int l) {
  return l == 0 ? pb->row_ptr : pb->amg->row_ptr[l];
}
const int32_t* level_cols(const opm_problem* pb, int l) {
  return l == 0 ? pb->col_idx : pb->amg->col[l];
}

}  // namespace

size_t cpr_bytes(const opm_problem* pb) {
  const opm_amg* g = pb->amg;
  if (!g) return 0;
  const int L = g->n_levels, nc = g->n[L - 1];
  size_t s = 2 * al256(8 * 3 * (size_t)pb->n_cells) + al256(8 * (size_t)nc * nc) +
             al256(8 * 2 * (size_t)nc * nc);
  for (int l = 0; l < L; ++l) s += al256(8 * (size_t)g->nnz[l]) + 4 * al256(8 * (size_t)g->n[l]);
  return s;
}

CprWork cpr_carve(const opm_problem* pb, void* p) {
  const opm_amg* g = pb->amg;
  CprWork w;
  std::memset(&w, 0, sizeof w);
  char* c = (char*)p;
  auto take = [&](size_t bytes) {
    char* r = c;
    c += al256(bytes);
    return (double*)r;
  };
  const int L = g->n_levels, nc = g->n[L - 1];
  w.w = take(8 * 3 * (size_t)pb->n_cells);
  for (int l = 0; l < L; ++l) {
    w.a[l] = take(8 * (size_t)g->nnz[l]);
    w.d[l] = take(8 * (size_t)g->n[l]);
    w.b[l] = take(8 * (size_t)g->n[l]);
    w.x[l] = take(8 * (size_t)g->n[l]);
    w.y[l] = take(8 * (size_t)g->n[l]);
  }
  w.inv = take(8 * (size_t)nc * nc);
  w.gj = take(8 * 2 * (size_t)nc * nc);
  w.r2 = take(8 * 3 * (size_t)pb->n_cells);
  return w;
}

int cpr_setup(const opm_problem* pb, const double* J, const CprWork& w, int32_t* flags,
              hipStream_t s) {
  const opm_amg* g = pb->amg;
  const int n = pb->n_cells, L = g->n_levels;
  hipLaunchKernelGGL(k_cpr_weights, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, n,
                     pb->row_ptr, pb->diag_pos, J, w.w, w.a[0], w.d[0], flags);
  for (int l = 1; l < L; ++l) {
    hipLaunchKernelGGL(k_cpr_galerkin, dim3(blocks_for(g->nnz[l], kBlock)), dim3(kBlock), 0, s,
                       g->nnz[l], g->gmap_ptr[l], g->gmap[l], w.a[l - 1], w.a[l]);
    hipLaunchKernelGGL(k_cpr_diag, dim3(blocks_for(g->n[l], kBlock)), dim3(kBlock), 0, s,
                       g->n[l], g->dpos[l], w.a[l], w.d[l]);
  }
  hipLaunchKernelGGL(k_cpr_inverse, dim3(1), dim3(kGjThreads), 0, s, g->n[L - 1],
                     level_rows(pb, L - 1), level_cols(pb, L - 1), w.a[L - 1], w.gj, w.inv,
                     flags);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int cpr_vcycle(const opm_problem* pb, const CprWork& w, hipStream_t s, const int32_t* skip) {
  const opm_amg* g = pb->amg;
  const int L = g->n_levels;
  for (int l = 0; l + 1 < L; ++l) {
    const int nl = g->n[l];
    hipLaunchKernelGGL(k_cpr_smooth0, dim3(blocks_for(nl, kBlock)), dim3(kBlock), 0, s, nl,
                       w.b[l], w.d[l], w.x[l], skip);
    hipLaunchKernelGGL(k_cpr_restrict, dim3(blocks_for(g->n[l + 1], kBlock)), dim3(kBlock), 0, s,
                       g->n[l + 1], g->child_ptr[l], g->child[l], level_rows(pb, l),
                       level_cols(pb, l), w.a[l], w.b[l], w.x[l], w.b[l + 1], skip);
  }
  // the coarsest level's solution is its y (the result of every level)
  hipLaunchKernelGGL(k_cpr_coarse, dim3(1), dim3(64), 0, s, g->n[L - 1], w.inv, w.b[L - 1],
                     w.y[L - 1], skip);
  for (int l = L - 2; l >= 0; --l) {
    const int nl = g->n[l];
    hipLaunchKernelGGL(k_cpr_prolong, dim3(blocks_for(nl, kBlock)), dim3(kBlock), 0, s, nl,
                       g->agg[l], w.y[l + 1], w.x[l], skip);
    hipLaunchKernelGGL(k_cpr_smooth, dim3(blocks_for(nl, kBlock)), dim3(kBlock), 0, s, nl,
                       level_rows(pb, l), level_cols(pb, l), w.a[l], w.d[l], w.b[l], w.x[l],
                       w.y[l], skip);
  }
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int cpr_apply(const opm_problem* pb, const double* J, void* ilu, int precision, const CprWork& w,
              const double* r, double* z, hipStream_t s, const int32_t* skip) {
  const int n = pb->n_cells;
  hipLaunchKernelGGL(k_cpr_rhs, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, n, w.w, r,
                     w.b[0], skip);
  OPM_TRY(cpr_vcycle(pb, w, s, skip));
  hipLaunchKernelGGL(k_cpr_r2, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, n, pb->row_ptr,
                     pb->col_idx, J, r, w.y[0], w.r2, skip);
  OPM_TRY_HIP(hipGetLastError());
  OPM_TRY(ilu_apply(pb, ilu, precision, w.r2, z, s, skip));
  hipLaunchKernelGGL(k_cpr_add, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, n, w.y[0], z,
                     skip);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

}  // namespace opm
