// CPR-AMG on the device (paper sec. 2.3.1: the two-stage constrained-
// pressure-residual preconditioner with an AMG for the pressure system).
//
// Setup, once per Jacobian: quasi-IMPES weights w_i with D_i^T w_i = e_p
// (D_i the diagonal block of row i), the pressure matrix (A_p)_ij =
// w_i^T A_ij e_p on the block pattern, the Galerkin coarse matrices of the
// aggregation hierarchy (each coarse entry the sum of its gather list of
// fine entries, in a fixed order) and the inverse of the coarsest matrix
// (in-place Gauss-Jordan with partial pivoting, at most 64 unknowns).
// Application, z = CPR(r): b_0 = w^T r; one V(1,1) cycle (damped Jacobi,
// omega = 2/3, before and after the coarse correction; the coarsest level
// by its inverse) gives x_p; x1 = e_p x_p; z = x1 + M_ILU^{-1} (r - A x1)
// with the (block-)ILU(0) factors of A.
//
// The cycle takes one kernel per level on the way down and one on the way
// up.  The pre-smoothed iterate x = omega D^{-1} b is never stored: a lane
// recomputes it for each neighbour it needs (the same expression, so the
// same bits), and likewise the right-hand side of a coarse unknown (the
// in-order sum of its children's residuals) and the prolonged iterate.
// Down at level l a lane writes b_l and the residual b_l - A_l x_l of its
// unknown; the coarsest level sums its children, applies the inverse; up
// at level l a lane writes the post-smoothed x_l + omega D^{-1} (b - A x_l)
// with x_l = omega D^{-1} b_l + P x_{l+1}.
//
// Every kernel is a gather (no atomics), so results are the same on every
// run.  Contraction is off in this file: the 3x3 weight solves and the
// sparse products round like plain multiply-then-add code.
#include <algorithm>
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

// Rows of a level are spread over a wavefront seven lanes each (nine rows
// per wavefront, one entry per lane: the 7-point stencil and its Galerkin
// coarse stencils have at most seven entries per row; longer rows are
// strided over the same lanes).  Consecutive lanes read consecutive entries.
constexpr int kRowLanes = 7;
constexpr int kWaveRows = kWave / kRowLanes;   // 9

struct RowLane {
  int row, k;
  bool live;
};

__device__ __forceinline__ RowLane row_lane(int n) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  RowLane r;
  r.row = wave * kWaveRows + lane / kRowLanes;
  r.k = lane % kRowLanes;
  r.live = lane < kWaveRows * kRowLanes && r.row < n;
  return r;
}

inline int row_blocks(int n) {
  const int waves = (n + kWaveRows - 1) / kWaveRows;
  return std::max(1, (waves + kBlock / kWave - 1) / (kBlock / kWave));
}

// Sum of p over the seven lanes of a row, in entry order (every lane of the
// wavefront takes part; the row's first lane holds the result).
__device__ __forceinline__ double row_sum(double p) {
  const int lane = threadIdx.x & (kWave - 1);
  const int base = lane - lane % kRowLanes;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kRowLanes; ++k) s += __shfl(p, base + k, kWave);
  return s;
}

// Weights and the level-0 diagonal (one lane per cell).
__global__ __launch_bounds__(kBlock) void k_cpr_weights(int n, const int32_t* diag_pos,
                                                         const double* J, double* w, double* d0,
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
  double v = 0.0;
  v += e[0] * D[0];
  v += e[1] * D[3];
  v += e[2] * D[6];
  d0[i] = v;
}

// The level-0 pressure matrix w_i^T A_ij e_p and the compact pressure
// column of J (one lane per block).
__global__ __launch_bounds__(kBlock) void k_cpr_pressure(int n, const int32_t* row_ptr,
                                                          const double* J, const double* w,
                                                          double* a0, double* jp) {
  const RowLane rl = row_lane(n);
  if (!rl.live) return;
  const int i = rl.row;
  const double w0 = w[3 * i], w1 = w[3 * i + 1], w2 = w[3 * i + 2];
  for (int q = row_ptr[i] + rl.k; q < row_ptr[i + 1]; q += kRowLanes) {
    const double* B = J + 9 * (size_t)q;
    const double c0 = B[0], c1 = B[3], c2 = B[6];
    double v = 0.0;
    v += w0 * c0;
    v += w1 * c1;
    v += w2 * c2;
    a0[q] = v;
    jp[3 * (size_t)q] = c0;
    jp[3 * (size_t)q + 1] = c1;
    jp[3 * (size_t)q + 2] = c2;
  }
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

// Inverse of the coarsest matrix (n <= 64) by in-place Gauss-Jordan
// elimination with partial pivoting in LDS (one workgroup): at step k the
// row with the largest |a_rk| (r >= k, lowest index on ties) is swapped
// into place, row k is divided by the pivot and eliminated from every other
// row, and column k becomes the corresponding column of the inverse; the
// row swaps are undone as column swaps at the end, last first.
constexpr int kGjThreads = 256;
__global__ __launch_bounds__(kGjThreads) void k_cpr_inverse(int n, const int32_t* row_ptr,
                                                             const int32_t* col, const double* a,
                                                             double* inv, int32_t* flags) {
  // rows padded to an odd stride: a column walk across lanes spreads over
  // the LDS banks
  __shared__ double A[OPM_AMG_COARSE * (OPM_AMG_COARSE + 1)];
  __shared__ int perm[OPM_AMG_COARSE];
  __shared__ int sel, bad;
  const int t = threadIdx.x, ld = n | 1;
  for (int k = t; k < n * ld; k += kGjThreads) A[k] = 0.0;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int i = t; i < n; i += kGjThreads)
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) A[i * ld + col[q]] = a[q];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (t < kWave) {   // the first wave picks the pivot row
      double v = (t >= k && t < n) ? fabs(A[t * ld + k]) : -1.0;
      int idx = t;
      for (int off = kWave / 2; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, kWave);
        const int oi = __shfl_xor(idx, off, kWave);
        if (ov > v || (ov == v && oi < idx)) {
          v = ov;
          idx = oi;
        }
      }
      if (t == 0) {
        sel = idx;
        perm[k] = idx;
        if (!(A[idx * ld + k] != 0.0)) bad = 1;
      }
    }
    __syncthreads();
    if (bad) break;   // uniform across the workgroup
    const int p = sel;
    if (p != k)
      for (int j = t; j < n; j += kGjThreads) {
        const double v = A[k * ld + j];
        A[k * ld + j] = A[p * ld + j];
        A[p * ld + j] = v;
      }
    __syncthreads();
    const double pk = 1.0 / A[k * ld + k];
    for (int j = t; j < n; j += kGjThreads)
      if (j != k) A[k * ld + j] *= pk;
    __syncthreads();
    for (int e = t; e < n * n; e += kGjThreads) {
      const int i = e / n, j = e - (e / n) * n;
      if (i != k && j != k) A[i * ld + j] -= A[i * ld + k] * A[k * ld + j];
    }
    __syncthreads();
    for (int i = t; i < n; i += kGjThreads) A[i * ld + k] = i == k ? pk : -A[i * ld + k] * pk;
    __syncthreads();
  }
  if (bad) {
    if (t == 0) flags[0] = OPM_ESINGULAR;
    return;
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = t; i < n; i += kGjThreads) {
        const double v = A[i * ld + k];
        A[i * ld + k] = A[i * ld + p];
        A[i * ld + p] = v;
      }
    __syncthreads();
  }
  for (int e = t; e < n * n; e += kGjThreads) inv[e] = A[(e / n) * ld + e % n];
}

// Where a level's right-hand side comes from.
enum BSrc { kFromR = 0, kGiven = 1, kChildren = 2 };

struct BArgs {
  const double* w;           // kFromR: weights and residual
  const double* r;
  const double* b0;          // kGiven
  const int32_t* child_ptr;  // kChildren: the finer level's aggregates and residuals
  const int32_t* child;
  const double* res;
};

template <int SRC>
__device__ __forceinline__ double bval(const BArgs& s, int i) {
  if (SRC == kFromR) {
    double v = s.w[3 * i] * s.r[3 * i];
    v += s.w[3 * i + 1] * s.r[3 * i + 1];
    v += s.w[3 * i + 2] * s.r[3 * i + 2];
    return v;
  } else if (SRC == kGiven) {
    return s.b0[i];
  } else {
    double v = 0.0;
    for (int t = s.child_ptr[i]; t < s.child_ptr[i + 1]; ++t) v += s.res[s.child[t]];
    return v;
  }
}

// Down at one level: b and the residual b - A x with x = omega D^{-1} b.
template <int SRC>
__global__ __launch_bounds__(kBlock) void k_cpr_down(int n, const int32_t* row_ptr,
                                                      const int32_t* col, const double* a,
                                                      const double* d, BArgs src, double* b,
                                                      double* res, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const RowLane rl = row_lane(n);
  double p = 0.0;
  if (rl.live)
    for (int q = row_ptr[rl.row] + rl.k; q < row_ptr[rl.row + 1]; q += kRowLanes) {
      const int j = col[q];
      p += a[q] * (kOmega * bval<SRC>(src, j) / d[j]);
    }
  const double s = row_sum(p);
  if (rl.live && rl.k == 0) {
    const double bi = bval<SRC>(src, rl.row);
    b[rl.row] = bi;
    res[rl.row] = bi - s;
  }
}

// Coarsest level: b from its source, x = A^{-1} b (one workgroup, a lane
// per row).
template <int SRC>
__global__ __launch_bounds__(OPM_AMG_COARSE) void k_cpr_coarse(int n, const double* inv,
                                                                BArgs src, double* x,
                                                                const int32_t* skip) {
  __shared__ double sb[OPM_AMG_COARSE];
  if (skip && *skip != 0) return;
  const int i = threadIdx.x;
  if (i < n) sb[i] = bval<SRC>(src, i);
  __syncthreads();
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < n; ++c) s += inv[i * n + c] * sb[c];
  x[i] = s;
}

// Up at one level: y = x + omega D^{-1} (b - A x) with the corrected
// x = omega D^{-1} b + x_c[agg].
__global__ __launch_bounds__(kBlock) void k_cpr_up(int n, const int32_t* row_ptr,
                                                    const int32_t* col, const double* a,
                                                    const double* d, const double* b,
                                                    const int32_t* agg, const double* xc,
                                                    double* y, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const RowLane rl = row_lane(n);
  double p = 0.0;
  if (rl.live)
    for (int q = row_ptr[rl.row] + rl.k; q < row_ptr[rl.row + 1]; q += kRowLanes) {
      const int j = col[q];
      p += a[q] * (kOmega * b[j] / d[j] + xc[agg[j]]);
    }
  const double s = row_sum(p);
  if (rl.live && rl.k == 0) {
    const int i = rl.row;
    const double bi = b[i], di = d[i];
    const double xi = kOmega * bi / di + xc[agg[i]];
    y[i] = xi + kOmega * (bi - s) / di;
  }
}

// Second-stage residual r2 = r - A x1 with x1 = (x_p, 0, 0) per cell, from
// the compact pressure column of J: seven lanes per row (one entry each,
// its three values in one 24-byte run), summed in entry order.
__global__ __launch_bounds__(kBlock) void k_cpr_r2(int n, const int32_t* row_ptr,
                                                    const int32_t* col, const double* jp,
                                                    const double* r, const double* xp,
                                                    double* r2, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const RowLane rl = row_lane(n);
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  if (rl.live)
    for (int q = row_ptr[rl.row] + rl.k; q < row_ptr[rl.row + 1]; q += kRowLanes) {
      const double* B = jp + 3 * (size_t)q;
      const double xj = xp[col[q]];
      p0 += B[0] * xj;
      p1 += B[1] * xj;
      p2 += B[2] * xj;
    }
  const double t0 = row_sum(p0), t1 = row_sum(p1), t2 = row_sum(p2);
  if (rl.live && rl.k == 0) {
    const int i = rl.row;
    r2[3 * i] = r[3 * i] - t0;
    r2[3 * i + 1] = r[3 * i + 1] - t1;
    r2[3 * i + 2] = r[3 * i + 2] - t2;
  }
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
  size_t s = 2 * al256(8 * 3 * (size_t)pb->n_cells) + al256(8 * 3 * (size_t)pb->nnzb) +
             al256(8 * (size_t)nc * nc);
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
  w.jp = take(8 * 3 * (size_t)pb->nnzb);
  for (int l = 0; l < L; ++l) {
    w.a[l] = take(8 * (size_t)g->nnz[l]);
    w.d[l] = take(8 * (size_t)g->n[l]);
    w.b[l] = take(8 * (size_t)g->n[l]);
    w.res[l] = take(8 * (size_t)g->n[l]);
    w.y[l] = take(8 * (size_t)g->n[l]);
  }
  w.inv = take(8 * (size_t)nc * nc);
  w.r2 = take(8 * 3 * (size_t)pb->n_cells);
  return w;
}

int cpr_setup(const opm_problem* pb, const double* J, const CprWork& w, int32_t* flags,
              hipStream_t s) {
  const opm_amg* g = pb->amg;
  const int n = pb->n_cells, L = g->n_levels;
  hipLaunchKernelGGL(k_cpr_weights, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, n,
                     pb->diag_pos, J, w.w, w.d[0], flags);
  hipLaunchKernelGGL(k_cpr_pressure, dim3(row_blocks(n)), dim3(kBlock), 0, s, n, pb->row_ptr, J,
                     w.w, w.a[0], w.jp);
  for (int l = 1; l < L; ++l) {
    hipLaunchKernelGGL(k_cpr_galerkin, dim3(blocks_for(g->nnz[l], kBlock)), dim3(kBlock), 0, s,
                       g->nnz[l], g->gmap_ptr[l], g->gmap[l], w.a[l - 1], w.a[l]);
    hipLaunchKernelGGL(k_cpr_diag, dim3(blocks_for(g->n[l], kBlock)), dim3(kBlock), 0, s,
                       g->n[l], g->dpos[l], w.a[l], w.d[l]);
  }
  hipLaunchKernelGGL(k_cpr_inverse, dim3(1), dim3(kGjThreads), 0, s, g->n[L - 1],
                     level_rows(pb, L - 1), level_cols(pb, L - 1), w.a[L - 1], w.inv, flags);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int cpr_vcycle(const opm_problem* pb, const CprWork& w, const double* r, const double* b0,
               hipStream_t s, const int32_t* skip) {
  const opm_amg* g = pb->amg;
  const int L = g->n_levels;
  auto src_of = [&](int l) {
    BArgs a{};
    if (l == 0) {
      a.w = w.w;
      a.r = r;
      a.b0 = b0;
    } else {
      a.child_ptr = g->child_ptr[l - 1];
      a.child = g->child[l - 1];
      a.res = w.res[l - 1];
    }
    return a;
  };
  for (int l = 0; l + 1 < L; ++l) {
    const dim3 grid(row_blocks(g->n[l]));
    const BArgs src = src_of(l);
    if (l > 0)
      hipLaunchKernelGGL(k_cpr_down<kChildren>, grid, dim3(kBlock), 0, s, g->n[l],
                         level_rows(pb, l), level_cols(pb, l), w.a[l], w.d[l], src, w.b[l],
                         w.res[l], skip);
    else if (r)
      hipLaunchKernelGGL(k_cpr_down<kFromR>, grid, dim3(kBlock), 0, s, g->n[l],
                         level_rows(pb, l), level_cols(pb, l), w.a[l], w.d[l], src, w.b[l],
                         w.res[l], skip);
    else
      hipLaunchKernelGGL(k_cpr_down<kGiven>, grid, dim3(kBlock), 0, s, g->n[l],
                         level_rows(pb, l), level_cols(pb, l), w.a[l], w.d[l], src, w.b[l],
                         w.res[l], skip);
  }
  const int lc = L - 1;
  const BArgs src = src_of(lc);
  if (lc > 0)
    hipLaunchKernelGGL(k_cpr_coarse<kChildren>, dim3(1), dim3(OPM_AMG_COARSE), 0, s, g->n[lc],
                       w.inv, src, w.y[lc], skip);
  else if (r)
    hipLaunchKernelGGL(k_cpr_coarse<kFromR>, dim3(1), dim3(OPM_AMG_COARSE), 0, s, g->n[lc],
                       w.inv, src, w.y[lc], skip);
  else
    hipLaunchKernelGGL(k_cpr_coarse<kGiven>, dim3(1), dim3(OPM_AMG_COARSE), 0, s, g->n[lc],
                       w.inv, src, w.y[lc], skip);
  for (int l = L - 2; l >= 0; --l)
    hipLaunchKernelGGL(k_cpr_up, dim3(row_blocks(g->n[l])), dim3(kBlock), 0, s, g->n[l],
                       level_rows(pb, l), level_cols(pb, l), w.a[l], w.d[l], w.b[l], g->agg[l],
                       w.y[l + 1], w.y[l], skip);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int cpr_apply(const opm_problem* pb, const double* J, void* ilu, int precision, const CprWork& w,
              const double* r, double* z, hipStream_t s, const int32_t* skip) {
  (void)J;
  const int n = pb->n_cells;
  OPM_TRY(cpr_vcycle(pb, w, r, nullptr, s, skip));
  hipLaunchKernelGGL(k_cpr_r2, dim3(row_blocks(n)), dim3(kBlock), 0, s, n, pb->row_ptr,
                     pb->col_idx, w.jp, r, w.y[0], w.r2, skip);
  OPM_TRY_HIP(hipGetLastError());
  OPM_TRY(ilu_apply(pb, ilu, precision, w.r2, z, s, skip));
  hipLaunchKernelGGL(k_cpr_add, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, n, w.y[0], z,
                     skip);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

}  // namespace opm
