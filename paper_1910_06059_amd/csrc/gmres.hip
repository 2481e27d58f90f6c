// Restarted GMRes, right preconditioned (paper sec. 2.3.1: the alternative
// Krylov method to the default BiCGStab), on the block-CSR SpMV and the
// ILU(0) / block-ILU0 solves of the other files.
//
// x0 = 0; each cycle starts from the residual r = b - A x, builds an
// orthonormal basis v_0 .. v_k of the Krylov space of A M^{-1} (at most
// `restart` vectors), reduces the Hessenberg least-squares problem with
// Givens rotations (|g_{j+1}| is the residual norm of the iterate), and ends
// with x += M^{-1} V y, R y = g.  Stop on |g_{j+1}| <= rtol ||b||, at the
// iteration cap, or on an exact breakdown h_{j+1,j} = 0.
//
// The preconditioned vectors z_j = M^{-1} v_j of the cycle are kept and the
// update is formed as Z y (the flexible form): for a linear M the same
// iterate as M^{-1} (V y), one preconditioner solve per cycle fewer, and with
// FP32 factors, whose solve is linear only up to FP32 rounding, an iterate
// whose residual is the one the rotations minimised.
//
// Orthogonalisation is classical Gram-Schmidt applied twice (CGS2): the
// j + 1 projections of one pass are one fused reduction (the first pass
// inside the SpMV), where modified Gram-Schmidt would need j + 1 dependent
// ones; the second pass restores the orthogonality modified Gram-Schmidt
// reaches.  All scalars stay on the device; every reduction is two-stage
// with per-workgroup partials summed in a fixed order, identically in every
// workgroup.  Per inner iteration: the preconditioner solve, SpMV + first
// projections, first update + second projections, second update + norm,
// the rotation step (one workgroup), and the normalisation of the next
// basis vector.  The host enqueues a cycle's iterations in chunks and reads
// the state word between chunks; kernels of an iteration that is no longer
// needed return at once.
#include <algorithm>

#include "krylov_dev.h"
#include "solver_dev.h"

namespace opm {

int ilu_apply(const opm_problem* pb, void* ilu, int precision, const double* r, double* x,
              hipStream_t s, const int32_t* skip);

namespace {

constexpr int kMaxRestart = 32;   // basis vectors per cycle (v_0 .. v_32 stored)
constexpr int kGmGrid = 256;      // workgroups of the vector kernels

enum GmState : int32_t { kGmRunning = 0, kGmCycleEnd = 1, kGmDone = 2 };

struct GmScalars {
  double H[(kMaxRestart + 1) * kMaxRestart];   // H[i * kMaxRestart + j]
  double cs[kMaxRestart], sn[kMaxRestart];
  double g[kMaxRestart + 1], y[kMaxRestart];
  double hcol[kMaxRestart + 1];                // projections of the current column
  double bnorm, tol, relres, scale;
  int32_t state;       // GmState
  int32_t no_update;   // cycle end: 1 when x keeps its value
  int32_t status, its, k_used, maxit, m, pad;
};

struct GmWork {
  double* V;      // [m + 1][Np] basis
  double* Z;      // [m][Np] preconditioned basis vectors
  double* w;      // [Np]
  double* pa;     // [kMaxRestart + 1][kGmGrid] partials
  double* pb;     // [kMaxRestart + 1][kGmGrid] partials
  double* pn;     // [kGmGrid] partials of a norm
  GmScalars* sc;
  int Np;
};

inline size_t np_of(int n) { return (3 * (size_t)n + 31) / 32 * 32; }

size_t gm_bytes(int n, int m) {
  const size_t Np = np_of(n);
  return sizeof(double) * ((size_t)(2 * m + 2) * Np + 2 * (kMaxRestart + 1) * kGmGrid + kGmGrid) +
         sizeof(GmScalars) + 256;
}

GmWork gm_carve(int n, int m, void* work) {
  GmWork w;
  w.Np = (int)np_of(n);
  double* d = (double*)work;
  w.V = d;
  d += (size_t)(m + 1) * w.Np;
  w.Z = d;
  d += (size_t)m * w.Np;
  w.w = d;
  d += w.Np;
  w.pa = d;
  d += (size_t)(kMaxRestart + 1) * kGmGrid;
  w.pb = d;
  d += (size_t)(kMaxRestart + 1) * kGmGrid;
  w.pn = d;
  d += kGmGrid;
  w.sc = (GmScalars*)d;
  return w;
}

inline int gm_grid(int N) { return std::min(kGmGrid, std::max(1, blocks_for(N, kBlock))); }

// Sum of the k + 1 rows of partials part[i][0 .. G) (i <= k) into h[i]:
// wavefront w sums rows w, w + 4, ..., lanes strided over the partials,
// then a fixed shuffle tree; h in LDS, one barrier.  Same order in every
// workgroup.
__device__ __forceinline__ void sum_rows(const double* part, int G, int k, double* h) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  for (int i = wv; i <= k; i += kBlock / kWave) {
    double v = 0.0;
    for (int q = lane; q < G; q += kWave) v += part[(size_t)i * kGmGrid + q];
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    if (lane == 0) h[i] = v;
  }
  __syncthreads();
}

// Per-workgroup partials of the k + 1 sums acc[i] (i <= k) into
// part[i][blockIdx.x].
__device__ __forceinline__ void store_rows(const double* acc, int k, double* part,
                                           double (*red)[kMaxRestart + 1]) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i <= kMaxRestart; ++i) {
    if (i <= k) {
      double v = acc[i];
      for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
      if (lane == 0) red[wv][i] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x <= k) {
    double s = 0.0;
    for (int q = 0; q < kBlock / kWave; ++q) s += red[q][threadIdx.x];
    part[(size_t)threadIdx.x * kGmGrid + blockIdx.x] = s;
  }
}

// x = 0 and partials of <b, b>.
__global__ __launch_bounds__(kBlock) void k_gm_init(int N, const double* b, double* x, GmWork w) {
  __shared__ double sh[kBlock / kWave];
  double bb = 0.0;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < N; k += gridDim.x * kBlock) {
    x[k] = 0.0;
    bb += b[k] * b[k];
  }
  const double s = block_sum<kBlock>(bb, sh);
  if (threadIdx.x == 0) w.pn[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_gm_init2(GmWork w, int G, double rtol, int maxit,
                                                      int m) {
  __shared__ double sh[kBlock / kWave];
  const double bb = kry::sum_partials<kBlock>(w.pn, G, sh);
  if (threadIdx.x == 0) {
    GmScalars& s = *w.sc;
    s.bnorm = sqrt(bb);
    s.tol = rtol * s.bnorm;
    s.relres = bb == 0.0 ? 0.0 : 1.0;
    s.its = 0;
    s.maxit = maxit;
    s.m = m;
    s.k_used = 0;
    s.no_update = 1;
    s.status = bb == 0.0 ? OPM_OK : OPM_ENOTCONV;
    s.state = bb == 0.0 ? kGmDone : kGmCycleEnd;
  }
}

// v_0 = b - A x (unscaled) and partials of its norm; skipped once done.
__global__ __launch_bounds__(kBlock) void k_gm_residual(int n, const int32_t* row_ptr,
                                                         const int32_t* col, const double* J,
                                                         const double* x, const double* b,
                                                         GmWork w) {
  __shared__ double sh[kBlock / kWave];
  if (w.sc->state == kGmDone) return;
  double acc = 0.0;
  const int lane = threadIdx.x & (kWave - 1), ng = ilu::spmv_groups(n);
  for (int g = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; g < ng;
       g += gridDim.x * (kBlock / kWave)) {
    int row, comp;
    double yv;
    if (ilu::spmv_group(n, row_ptr, col, J, x, g, lane, row, comp, yv)) {
      const double r = b[3 * row + comp] - yv;
      w.V[3 * row + comp] = r;
      acc += r * r;
    }
  }
  const double s = block_sum<kBlock>(acc, sh);
  if (threadIdx.x == 0) w.pn[blockIdx.x] = s;
}

// Start of a cycle: beta = ||r||; converged, or g = beta e_0 and run.
__global__ __launch_bounds__(kBlock) void k_gm_start(GmWork w, int G) {
  __shared__ double sh[kBlock / kWave];
  GmScalars& s = *w.sc;
  if (s.state == kGmDone) return;
  const double beta = sqrt(kry::sum_partials<kBlock>(w.pn, G, sh));
  if (threadIdx.x == 0) {
    s.relres = s.bnorm > 0.0 ? beta / s.bnorm : 0.0;
    s.k_used = 0;
    s.no_update = 1;
    if (s.its >= s.maxit) {   // only with maxit = 0: a cycle at the cap ends the solve
      s.status = OPM_ENOTCONV;
      s.state = kGmDone;
    } else if (beta <= s.tol) {
      s.status = OPM_OK;
      s.state = kGmDone;
    } else {
      for (int i = 0; i <= kMaxRestart; ++i) s.g[i] = 0.0;
      s.g[0] = beta;
      s.scale = 1.0 / beta;
      s.state = kGmRunning;
    }
  }
}

// dst = src * scale (the next basis vector), while running.
__global__ __launch_bounds__(kBlock) void k_gm_scale(int N, const double* src, double* dst,
                                                      GmWork w) {
  if (w.sc->state != kGmRunning) return;
  const double f = w.sc->scale;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < N; k += gridDim.x * kBlock)
    dst[k] = src[k] * f;
}

// w = A z_j and the partials of <v_i, w>, i <= j.
__global__ __launch_bounds__(kBlock) void k_gm_spmv_dots(int n, const int32_t* row_ptr,
                                                          const int32_t* col, const double* J,
                                                          GmWork w, int j) {
  const double* z = w.Z + (size_t)j * w.Np;
  __shared__ double red[kBlock / kWave][kMaxRestart + 1];
  if (w.sc->state != kGmRunning) return;
  double acc[kMaxRestart + 1];
#pragma unroll
  for (int i = 0; i <= kMaxRestart; ++i) acc[i] = 0.0;
  const int lane = threadIdx.x & (kWave - 1), ng = ilu::spmv_groups(n);
  for (int g = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; g < ng;
       g += gridDim.x * (kBlock / kWave)) {
    int row, comp;
    double yv;
    if (ilu::spmv_group(n, row_ptr, col, J, z, g, lane, row, comp, yv)) {
      const size_t e = 3 * (size_t)row + comp;
      w.w[e] = yv;
#pragma unroll
      for (int i = 0; i <= kMaxRestart; ++i)
        if (i <= j) acc[i] += w.V[(size_t)i * w.Np + e] * yv;
    }
  }
  store_rows(acc, j, w.pa, red);
}

// One Gram-Schmidt update w -= V_{0..j} h with h summed from `in`; then the
// partials of the next pass (<v_i, w>) or, in the last pass, of <w, w>.
// Workgroup 0 keeps the projections of the column: the first pass stores
// them, the second adds its own.
template <bool LAST>
__global__ __launch_bounds__(kBlock) void k_gm_cgs(int N, GmWork w, const double* in, int Gin,
                                                    double* out, int j) {
  __shared__ double h[kMaxRestart + 1];
  __shared__ double red[kBlock / kWave][kMaxRestart + 1];
  __shared__ double sh[kBlock / kWave];
  if (w.sc->state != kGmRunning) return;
  sum_rows(in, Gin, j, h);
  if (blockIdx.x == 0 && (int)threadIdx.x <= j)
    w.sc->hcol[threadIdx.x] = LAST ? w.sc->hcol[threadIdx.x] + h[threadIdx.x] : h[threadIdx.x];
  double acc[kMaxRestart + 1];
#pragma unroll
  for (int i = 0; i <= kMaxRestart; ++i) acc[i] = 0.0;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < N; k += gridDim.x * kBlock) {
    double v = w.w[k];
#pragma unroll
    for (int i = 0; i <= kMaxRestart; ++i)
      if (i <= j) v -= h[i] * w.V[(size_t)i * w.Np + k];
    w.w[k] = v;
    if (LAST) {
      acc[0] += v * v;
    } else {
#pragma unroll
      for (int i = 0; i <= kMaxRestart; ++i)
        if (i <= j) acc[i] += w.V[(size_t)i * w.Np + k] * v;
    }
  }
  if (LAST) {
    const double s = block_sum<kBlock>(acc[0], sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
  } else {
    store_rows(acc, j, out, red);
  }
}

// Column j of H, the rotations, the residual estimate and the decision
// (one workgroup).
__global__ __launch_bounds__(kBlock) void k_gm_givens(GmWork w, int G, int j) {
  __shared__ double sh[kBlock / kWave];
  GmScalars& s = *w.sc;
  if (s.state != kGmRunning) return;
  const double hn = sqrt(kry::sum_partials<kBlock>(w.pn, G, sh));
  if (threadIdx.x != 0) return;
  const int m = s.m;
  double* H = s.H;
  for (int i = 0; i <= j; ++i) H[i * kMaxRestart + j] = s.hcol[i];
  H[(j + 1) * kMaxRestart + j] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = H[i * kMaxRestart + j], c = H[(i + 1) * kMaxRestart + j];
    H[i * kMaxRestart + j] = s.cs[i] * a + s.sn[i] * c;
    H[(i + 1) * kMaxRestart + j] = -s.sn[i] * a + s.cs[i] * c;
  }
  const double d = hypot(H[j * kMaxRestart + j], H[(j + 1) * kMaxRestart + j]);
  s.cs[j] = d > 0.0 ? H[j * kMaxRestart + j] / d : 1.0;
  s.sn[j] = d > 0.0 ? H[(j + 1) * kMaxRestart + j] / d : 0.0;
  H[j * kMaxRestart + j] = d;
  H[(j + 1) * kMaxRestart + j] = 0.0;
  s.g[j + 1] = -s.sn[j] * s.g[j];
  s.g[j] = s.cs[j] * s.g[j];
  s.its += 1;
  s.k_used = j + 1;
  s.no_update = 0;
  s.relres = fabs(s.g[j + 1]) / s.bnorm;
  if (fabs(s.g[j + 1]) <= s.tol || hn == 0.0) {
    s.status = OPM_OK;
    s.state = kGmCycleEnd;   // the update ends the solve (status OK)
  } else if (j + 1 >= m || s.its >= s.maxit) {
    s.state = kGmCycleEnd;
  } else {
    s.scale = 1.0 / hn;
  }
}

// End of a cycle: y = R^{-1} g over the columns used (one thread).
__global__ __launch_bounds__(64) void k_gm_solve(GmWork w) {
  GmScalars& s = *w.sc;
  if (threadIdx.x != 0 || s.state == kGmDone) return;
  const int k = s.k_used;
  for (int i = k - 1; i >= 0; --i) {
    double t = s.g[i];
    for (int c = i + 1; c < k; ++c) t -= s.H[i * kMaxRestart + c] * s.y[c];
    const double d = s.H[i * kMaxRestart + i];
    if (d == 0.0) {
      s.status = OPM_EBREAKDOWN;
      s.state = kGmDone;
      s.no_update = 1;
      return;
    }
    s.y[i] = t / d;
  }
}

// x += Z y over the columns used.
__global__ __launch_bounds__(kBlock) void k_gm_xupdate(int N, double* x, GmWork w) {
  __shared__ double y[kMaxRestart];
  const GmScalars& s = *w.sc;
  if (s.state == kGmDone || s.no_update) return;
  const int k = s.k_used;
  if ((int)threadIdx.x < k) y[threadIdx.x] = s.y[threadIdx.x];
  __syncthreads();
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < N; e += gridDim.x * kBlock) {
    double u = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxRestart; ++i)
      if (i < k) u += y[i] * w.Z[(size_t)i * w.Np + e];
    x[e] += u;
  }
}

// Then the next cycle, or done (converged, or the iteration cap).
__global__ __launch_bounds__(64) void k_gm_close(GmWork w) {
  GmScalars& s = *w.sc;
  if (threadIdx.x != 0 || s.state == kGmDone) return;
  if (s.status == OPM_OK || s.its >= s.maxit) s.state = kGmDone;
}

}  // namespace

size_t gmres_bytes(const opm_problem* pb, int restart) {
  return gm_bytes(pb->n_cells, std::min(std::max(restart, 1), kMaxRestart));
}

int gmres(const opm_problem* pb, const double* J, void* ilu, int precision, const double* b,
          double* x, double rtol, int maxit, int restart, void* work, opm_solve_report* rep,
          hipStream_t st) {
  if (restart < 1 || restart > kMaxRestart || maxit < 0) return OPM_EINVAL;
  const int n = pb->n_cells, N = 3 * n, m = restart;
  GmWork w = gm_carve(n, m, work);
  const int G = gm_grid(N);
  const int Gs = std::min(kGmGrid, std::max(1, blocks_for(ilu::spmv_groups(n), kBlock / kWave)));
  hipLaunchKernelGGL(k_gm_init, dim3(G), dim3(kBlock), 0, st, N, b, x, w);
  hipLaunchKernelGGL(k_gm_init2, dim3(1), dim3(kBlock), 0, st, w, G, rtol, maxit, m);
  OPM_TRY_HIP(hipGetLastError());
  const int chunk = 6;
  GmScalars host;
  for (int cycle = 0;; ++cycle) {
    hipLaunchKernelGGL(k_gm_residual, dim3(Gs), dim3(kBlock), 0, st, n, pb->row_ptr, pb->col_idx,
                       J, x, b, w);
    hipLaunchKernelGGL(k_gm_start, dim3(1), dim3(kBlock), 0, st, w, Gs);
    hipLaunchKernelGGL(k_gm_scale, dim3(G), dim3(kBlock), 0, st, N, w.V, w.V, w);
    OPM_TRY_HIP(hipGetLastError());
    for (int j0 = 0; j0 < m; j0 += chunk) {
      for (int j = j0; j < std::min(m, j0 + chunk); ++j) {
        OPM_TRY(ilu_apply(pb, ilu, precision, w.V + (size_t)j * w.Np, w.Z + (size_t)j * w.Np, st,
                          &w.sc->state));
        hipLaunchKernelGGL(k_gm_spmv_dots, dim3(Gs), dim3(kBlock), 0, st, n, pb->row_ptr,
                           pb->col_idx, J, w, j);
        hipLaunchKernelGGL(k_gm_cgs<false>, dim3(G), dim3(kBlock), 0, st, N, w, w.pa, Gs, w.pb,
                           j);
        hipLaunchKernelGGL(k_gm_cgs<true>, dim3(G), dim3(kBlock), 0, st, N, w, w.pb, G, w.pn,
                           j);
        hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(kBlock), 0, st, w, G, j);
        if (j + 1 < m)
          hipLaunchKernelGGL(k_gm_scale, dim3(G), dim3(kBlock), 0, st, N, w.w,
                             w.V + (size_t)(j + 1) * w.Np, w);
        OPM_TRY_HIP(hipGetLastError());
      }
      OPM_TRY_HIP(hipMemcpyAsync(&host, w.sc, sizeof(GmScalars), hipMemcpyDeviceToHost, st));
      OPM_TRY_HIP(hipStreamSynchronize(st));
      if (host.state != kGmRunning) break;
    }
    // end of the cycle: x += Z y
    hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, st, w);
    hipLaunchKernelGGL(k_gm_xupdate, dim3(G), dim3(kBlock), 0, st, N, x, w);
    hipLaunchKernelGGL(k_gm_close, dim3(1), dim3(64), 0, st, w);
    OPM_TRY_HIP(hipGetLastError());
    OPM_TRY_HIP(hipMemcpyAsync(&host, w.sc, sizeof(GmScalars), hipMemcpyDeviceToHost, st));
    OPM_TRY_HIP(hipStreamSynchronize(st));
    if (host.state == kGmDone) break;
    if (cycle > maxit + 1) {   // cannot happen: every cycle adds an iteration or stops
      host.status = OPM_ENOTCONV;
      break;
    }
  }
  if (rep) {
    rep->status = host.status;
    rep->half = 0;
    rep->its = host.its;
    rep->rel_res = host.relres;
  }
  return OPM_OK;
}

}  // namespace opm
