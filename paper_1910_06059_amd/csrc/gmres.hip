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
// j + 1 projections of a pass are one fused reduction, where modified
// Gram-Schmidt would need j + 1 dependent ones; the second pass restores the
// orthogonality modified Gram-Schmidt reaches.  Per inner iteration six
// launches: the preconditioner solve, the SpMV, the first projections, the
// first update + second projections, the second update + norm, and the
// rotations + the next basis vector.
//
// All scalars stay on the device.  A reducing kernel writes one partial per
// workgroup (at most kGmGrid of them); the kernel that consumes the sum adds
// the partials in its prologue, in the same fixed order in every workgroup,
// so all workgroups hold the same bits and take the same decisions, and
// every run gives the same result.  A state word (running / cycle end /
// done), read once per workgroup, lets the kernels of iterations that are no
// longer needed return at once; the host enqueues a cycle's iterations in
// chunks and reads the state between chunks.
#include <algorithm>

#include "cpr_dev.h"
#include "solver_dev.h"

namespace opm {

int ilu_apply(const opm_problem* pb, void* ilu, int precision, const double* r, double* x,
              hipStream_t s, const int32_t* skip);

namespace {

constexpr int kMaxRestart = 32;   // basis vectors per cycle
constexpr int kGmGrid = 256;      // largest grid of the reducing kernels (partials per sum)
constexpr int kGmBlock = 512;     // threads of the vector kernels (8 wavefronts)

enum GmState : int32_t { kGmRunning = 0, kGmCycleEnd = 1, kGmDone = 2 };

struct GmScalars {
  double H[(kMaxRestart + 1) * kMaxRestart];   // H[i * kMaxRestart + j], rotated
  double cs[kMaxRestart], sn[kMaxRestart];
  double gr[kMaxRestart];           // rotated right-hand side of the least-squares problem
  double gres[kMaxRestart + 1];     // gres[j]: residual estimate after j iterations of the cycle
  double h1[kMaxRestart + 1], h2[kMaxRestart + 1];   // projections of the two passes
  // the part read by the host between chunks starts here
  double bnorm, tol, relres, scale;
  int32_t state;       // GmState
  int32_t status, its, k_used, maxit, m, its0, pad;
};

struct GmHostView {   // mirrors GmScalars from bnorm on
  double bnorm, tol, relres, scale;
  int32_t state, status, its, k_used, maxit, m, its0, pad;
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

inline int vec_grid(int N) { return std::min(kGmGrid, std::max(1, blocks_for(N, kGmBlock))); }

// Rows 0..k of the partials part[i][0 .. G) summed into out[i] (LDS), each
// row by one wavefront: lanes strided over the partials, then a fixed
// shuffle tree.  Same order in every workgroup.
__device__ __forceinline__ void sum_rows(const double* part, int G, int k, double* out) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  for (int i = wv; i <= k; i += kGmBlock / kWave) {
    double v = 0.0;
    for (int q = lane; q < G; q += kWave) v += part[(size_t)i * kGmGrid + q];
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    if (lane == 0) out[i] = v;
  }
  __syncthreads();
}

// The workgroup's sums of acc[i] (i <= k) into part[i][blockIdx.x].
template <int JB>
__device__ __forceinline__ void store_rows(const double (&acc)[JB], int k, double* part,
                                           double (*red)[JB]) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < JB; ++i) {
    if (i <= k) {
      double v = acc[i];
      for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
      if (lane == 0) red[wv][i] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x <= k) {
    double s = 0.0;
    for (int q = 0; q < kGmBlock / kWave; ++q) s += red[q][threadIdx.x];
    part[(size_t)threadIdx.x * kGmGrid + blockIdx.x] = s;
  }
}

__device__ __forceinline__ int read_state(const GmScalars* sc, int* word) {
  if (threadIdx.x == 0) *word = sc->state;
  __syncthreads();
  return *word;
}

// x = 0 and the partials of <b, b>.
__global__ __launch_bounds__(kGmBlock) void k_gm_init(int N, const double* b, double* x,
                                                       GmWork w) {
  __shared__ double sh[kGmBlock / kWave];
  double bb = 0.0;
  for (int k = blockIdx.x * kGmBlock + threadIdx.x; k < N; k += gridDim.x * kGmBlock) {
    x[k] = 0.0;
    bb += b[k] * b[k];
  }
  const double s = block_sum<kGmBlock>(bb, sh);
  if (threadIdx.x == 0) w.pn[blockIdx.x] = s;
}

__global__ __launch_bounds__(kGmBlock) void k_gm_init2(GmWork w, int G, double rtol, int maxit,
                                                        int m) {
  __shared__ double tot[1];
  sum_rows(w.pn, G, 0, tot);
  if (threadIdx.x == 0) {
    GmScalars& c = *w.sc;
    const double t = tot[0];
    c.bnorm = sqrt(t);
    c.tol = rtol * c.bnorm;
    c.relres = t == 0.0 ? 0.0 : 1.0;
    c.its = 0;
    c.its0 = 0;
    c.maxit = maxit;
    c.m = m;
    c.k_used = 0;
    c.status = t == 0.0 ? OPM_OK : OPM_ENOTCONV;
    c.state = t == 0.0 ? kGmDone : kGmCycleEnd;
  }
}

// y = A x (one group of three block rows per wavefront, the grid of the
// plain SpMV) while the state is `want`; with RES, y = b - A x.
template <bool RES>
__global__ __launch_bounds__(kBlock) void k_gm_spmv(int n, const int32_t* row_ptr,
                                                     const int32_t* col, const double* J,
                                                     const double* x, const double* b, double* y,
                                                     const GmScalars* sc, int want, WellCorr wc) {
  __shared__ int word;
  const int st = read_state(sc, &word);
  if (RES ? st == kGmDone : st != want) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int group = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (group >= ilu::spmv_groups(n)) return;   // whole wavefront
  int row, comp;
  double yv;
  if (ilu::spmv_group(n, row_ptr, col, J, x, group, lane, row, comp, yv, wc))
    y[3 * row + comp] = RES ? b[3 * row + comp] - yv : yv;
}

// Partials of ||v_0||^2 at the start of a cycle.
__global__ __launch_bounds__(kGmBlock) void k_gm_norm0(int N, GmWork w) {
  __shared__ double sh[kGmBlock / kWave];
  __shared__ int word;
  if (read_state(w.sc, &word) == kGmDone) return;
  double ss = 0.0;
  for (int k = blockIdx.x * kGmBlock + threadIdx.x; k < N; k += gridDim.x * kGmBlock)
    ss += w.V[k] * w.V[k];
  const double s = block_sum<kGmBlock>(ss, sh);
  if (threadIdx.x == 0) w.pn[blockIdx.x] = s;
}

// Start of a cycle (one workgroup): beta = ||r||; the iteration cap (only
// with maxit = 0, since a cycle that reaches it ends the solve), convergence,
// or g = beta e_0 and run.
__global__ __launch_bounds__(kGmBlock) void k_gm_start(GmWork w, int G) {
  __shared__ double tot[1];
  __shared__ int word;
  if (read_state(w.sc, &word) == kGmDone) return;
  sum_rows(w.pn, G, 0, tot);
  if (threadIdx.x != 0) return;
  GmScalars& c = *w.sc;
  const double beta = sqrt(tot[0]);
  c.relres = c.bnorm > 0.0 ? beta / c.bnorm : 0.0;
  c.k_used = 0;
  c.its0 = c.its;
  if (c.its >= c.maxit) {
    c.status = OPM_ENOTCONV;
    c.state = kGmDone;
  } else if (beta <= c.tol) {
    c.status = OPM_OK;
    c.state = kGmDone;
  } else {
    c.gres[0] = beta;
    c.scale = 1.0 / beta;
    c.state = kGmRunning;
  }
}

// v_0 *= 1 / beta, while running.
__global__ __launch_bounds__(kGmBlock) void k_gm_scale0(int N, GmWork w) {
  __shared__ int word;
  if (read_state(w.sc, &word) != kGmRunning) return;
  const double f = w.sc->scale;
  for (int k = blockIdx.x * kGmBlock + threadIdx.x; k < N; k += gridDim.x * kGmBlock)
    w.V[k] *= f;
}

// The first JB projection coefficients in LDS, zero past j: the update loops
// run over all JB basis rows without a branch (rows past j are read as row
// j, a cache hit, and weighted by zero), so all loads of an element are in
// flight at once.
template <int JB>
__device__ __forceinline__ void coeffs(const double* h, int j, double* hs) {
  if ((int)threadIdx.x < JB) hs[threadIdx.x] = (int)threadIdx.x <= j ? h[threadIdx.x] : 0.0;
  __syncthreads();
}

// Partials of the first projections h1_i = <v_i, w>, i <= j.
template <int JB>
__global__ __launch_bounds__(kGmBlock) void k_gm_dots(int N, GmWork w, int j) {
  __shared__ double red[kGmBlock / kWave][JB];
  __shared__ int word;
  if (read_state(w.sc, &word) != kGmRunning) return;
  double acc[JB];
#pragma unroll
  for (int i = 0; i < JB; ++i) acc[i] = 0.0;
  for (int k = blockIdx.x * kGmBlock + threadIdx.x; k < N; k += gridDim.x * kGmBlock) {
    double vk[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) vk[i] = w.V[(size_t)min(i, j) * w.Np + k];
    const double wk = w.w[k];
    __builtin_amdgcn_sched_barrier(0);   // every load of the element issued before the arithmetic
#pragma unroll
    for (int i = 0; i < JB; ++i) acc[i] += vk[i] * wk;
  }
  store_rows<JB>(acc, j, w.pa, red);
}

// First update w -= V h1 (h1 summed from the partials; workgroup 0 keeps
// it) and the partials of the second projections h2_i = <v_i, w>.
template <int JB>
__global__ __launch_bounds__(kGmBlock) void k_gm_cgs1(int N, GmWork w, int j, int G) {
  __shared__ double hsum[kMaxRestart + 1];
  __shared__ double h[JB];
  __shared__ double red[kGmBlock / kWave][JB];
  __shared__ int word;
  if (read_state(w.sc, &word) != kGmRunning) return;
  sum_rows(w.pa, G, j, hsum);
  if (blockIdx.x == 0 && (int)threadIdx.x <= j) w.sc->h1[threadIdx.x] = hsum[threadIdx.x];
  coeffs<JB>(hsum, j, h);
  double acc[JB];
#pragma unroll
  for (int i = 0; i < JB; ++i) acc[i] = 0.0;
  for (int k = blockIdx.x * kGmBlock + threadIdx.x; k < N; k += gridDim.x * kGmBlock) {
    double vk[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) vk[i] = w.V[(size_t)min(i, j) * w.Np + k];
    double v = w.w[k];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < JB; ++i) v -= h[i] * vk[i];
    w.w[k] = v;
#pragma unroll
    for (int i = 0; i < JB; ++i) acc[i] += vk[i] * v;
  }
  store_rows<JB>(acc, j, w.pb, red);
}

// Second update w -= V h2 (workgroup 0 keeps h2) and the partials of ||w||^2.
template <int JB>
__global__ __launch_bounds__(kGmBlock) void k_gm_cgs2(int N, GmWork w, int j, int G) {
  __shared__ double hsum[kMaxRestart + 1];
  __shared__ double h[JB];
  __shared__ double sh[kGmBlock / kWave];
  __shared__ int word;
  if (read_state(w.sc, &word) != kGmRunning) return;
  sum_rows(w.pb, G, j, hsum);
  if (blockIdx.x == 0 && (int)threadIdx.x <= j) w.sc->h2[threadIdx.x] = hsum[threadIdx.x];
  coeffs<JB>(hsum, j, h);
  double ss = 0.0;
  for (int k = blockIdx.x * kGmBlock + threadIdx.x; k < N; k += gridDim.x * kGmBlock) {
    double vk[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) vk[i] = w.V[(size_t)min(i, j) * w.Np + k];
    double v = w.w[k];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < JB; ++i) v -= h[i] * vk[i];
    w.w[k] = v;
    ss += v * v;
  }
  const double s = block_sum<kGmBlock>(ss, sh);
  if (threadIdx.x == 0) w.pn[blockIdx.x] = s;
}

// Column j of H (h1 + h2, then h_{j+1,j} = ||w||), the earlier rotations and
// the new one, the residual estimate and the decision: converged or an
// exact breakdown (end the cycle, then the solve), end of the cycle (restart
// length or iteration cap), or go on with v_{j+1} = w / h_{j+1,j}.  Every
// workgroup computes the rotation from values this kernel does not write,
// so all take the same decision; workgroup 0 records it.
__global__ __launch_bounds__(kGmBlock) void k_gm_rotate(int N, GmWork w, int j, int G) {
  __shared__ double tot[1];
  __shared__ double col[kMaxRestart + 1];
  __shared__ double dec[2];   // 1 / h_{j+1,j}, and 1 when the cycle goes on
  __shared__ int word;
  if (read_state(w.sc, &word) != kGmRunning) return;
  sum_rows(w.pn, G, 0, tot);
  GmScalars& c = *w.sc;
  if (threadIdx.x == 0) {
    const double hn = sqrt(tot[0]);
    for (int i = 0; i <= j; ++i) col[i] = c.h1[i] + c.h2[i];
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double a = col[i], d = col[i + 1];
      col[i] = c.cs[i] * a + c.sn[i] * d;
      col[i + 1] = -c.sn[i] * a + c.cs[i] * d;
    }
    const double d = hypot(col[j], col[j + 1]);
    const double cj = d > 0.0 ? col[j] / d : 1.0, sj = d > 0.0 ? col[j + 1] / d : 0.0;
    const double gj = c.gres[j];
    const double gnext = -sj * gj;
    const int its = c.its0 + j + 1;
    const bool conv = fabs(gnext) <= c.tol || hn == 0.0;
    const bool more = !conv && j + 1 < c.m && its < c.maxit;
    dec[0] = 1.0 / hn;
    dec[1] = more ? 1.0 : 0.0;
    if (blockIdx.x == 0) {
      for (int i = 0; i < j; ++i) c.H[i * kMaxRestart + j] = col[i];
      c.H[j * kMaxRestart + j] = d;
      c.cs[j] = cj;
      c.sn[j] = sj;
      c.gr[j] = cj * gj;
      c.gres[j + 1] = gnext;
      c.its = its;
      c.k_used = j + 1;
      c.relres = fabs(gnext) / c.bnorm;
      if (conv) c.status = OPM_OK;
      if (!more) c.state = kGmCycleEnd;
    }
  }
  __syncthreads();
  if (dec[1] == 0.0) return;
  const double f = dec[0];
  double* vn = w.V + (size_t)(j + 1) * w.Np;
  for (int k = blockIdx.x * kGmBlock + threadIdx.x; k < N; k += gridDim.x * kGmBlock)
    vn[k] = w.w[k] * f;
}

// End of a cycle: y = R^{-1} g over the k columns used (every workgroup
// solves the small triangular system from LDS, identically) and x += Z y,
// unless R is singular.
template <int JB>
__global__ __launch_bounds__(kGmBlock) void k_gm_finish(int N, double* x, GmWork w) {
  __shared__ double R[kMaxRestart * kMaxRestart];
  __shared__ double y[kMaxRestart];
  __shared__ int word, singular;
  if (read_state(w.sc, &word) == kGmDone) return;
  const GmScalars& c = *w.sc;
  const int k = c.k_used;
  for (int q = threadIdx.x; q < k * kMaxRestart; q += kGmBlock) R[q] = c.H[q];
  if ((int)threadIdx.x < kMaxRestart) y[threadIdx.x] = (int)threadIdx.x < k ? c.gr[threadIdx.x] : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    int bad = 0;
    for (int i = k - 1; i >= 0; --i) {
      double t = y[i];
      for (int q = i + 1; q < k; ++q) t -= R[i * kMaxRestart + q] * y[q];
      const double dg = R[i * kMaxRestart + i];
      if (dg == 0.0) {
        bad = 1;
        break;
      }
      y[i] = t / dg;
    }
    singular = bad;
  }
  __syncthreads();
  if (singular || k == 0) return;
  // y is zero past k - 1: rows past k - 1 are read as row k - 1
  for (int e = blockIdx.x * kGmBlock + threadIdx.x; e < N; e += gridDim.x * kGmBlock) {
    double zk[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) zk[i] = w.Z[(size_t)min(i, k - 1) * w.Np + e];
    const double xe = x[e];
    __builtin_amdgcn_sched_barrier(0);
    double u = 0.0;
#pragma unroll
    for (int i = 0; i < JB; ++i) u += y[i] * zk[i];
    x[e] = xe + u;
  }
}

// After the update (one thread): a singular R ends the solve with
// OPM_EBREAKDOWN (x keeps the previous cycles); convergence or the iteration
// cap end it; otherwise the next cycle starts.
__global__ void k_gm_close(GmWork w) {
  if (threadIdx.x != 0) return;
  GmScalars& c = *w.sc;
  if (c.state == kGmDone) return;
  for (int i = 0; i < c.k_used; ++i)
    if (c.H[i * kMaxRestart + i] == 0.0) {
      c.status = OPM_EBREAKDOWN;
      c.state = kGmDone;
      return;
    }
  if (c.status == OPM_OK || c.its >= c.maxit) c.state = kGmDone;
}

template <int JB>
void launch_projections(const GmWork& w, int j, int N, int G, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_dots<JB>, dim3(G), dim3(kGmBlock), 0, st, N, w, j);
  hipLaunchKernelGGL(k_gm_cgs1<JB>, dim3(G), dim3(kGmBlock), 0, st, N, w, j, G);
  hipLaunchKernelGGL(k_gm_cgs2<JB>, dim3(G), dim3(kGmBlock), 0, st, N, w, j, G);
}

template <int JB>
void launch_finish(const GmWork& w, double* x, int N, int G, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_finish<JB>, dim3(G), dim3(kGmBlock), 0, st, N, x, w);
}

int read_view(const GmWork& w, GmHostView* v, hipStream_t st) {
  OPM_TRY_HIP(hipMemcpyAsync(v, &w.sc->bnorm, sizeof(GmHostView), hipMemcpyDeviceToHost, st));
  OPM_TRY_HIP(hipStreamSynchronize(st));
  return OPM_OK;
}

}  // namespace

size_t gmres_bytes(const opm_problem* pb, int restart) {
  return gm_bytes(pb->n_cells, std::min(std::max(restart, 1), kMaxRestart));
}

// cpr (may be null): CPR-AMG set up for J, with ilu as its second stage.
// ws (may be null): standard wells, solved through their Schur complement
// (the operator subtracts sum_w C_w D_w^{-1} B_w of its argument).
int gmres(const opm_problem* pb, const double* J, void* ilu, int precision, const double* b,
          double* x, double rtol, int maxit, int restart, void* work, opm_solve_report* rep,
          hipStream_t st, const CprWork* cpr, const WellSchur* ws) {
  if (restart < 1 || restart > kMaxRestart || maxit < 0) return OPM_EINVAL;
  const int n = pb->n_cells, N = 3 * n, m = restart;
  GmWork w = gm_carve(n, m, work);
  const int G = vec_grid(N);
  const int Gs = std::max(1, blocks_for(ilu::spmv_groups(n), kBlock / kWave));
  hipLaunchKernelGGL(k_gm_init, dim3(G), dim3(kGmBlock), 0, st, N, b, x, w);
  hipLaunchKernelGGL(k_gm_init2, dim3(1), dim3(kGmBlock), 0, st, w, G, rtol, maxit, m);
  OPM_TRY_HIP(hipGetLastError());
  const int chunk = 6;
  GmHostView v{};
  const WellCorr wc = ws ? ws->wc() : WellCorr{nullptr, nullptr, nullptr};
  for (int cycle = 0;; ++cycle) {
    if (ws) OPM_TRY(well_op(*ws, x, nullptr, st));
    hipLaunchKernelGGL(k_gm_spmv<true>, dim3(Gs), dim3(kBlock), 0, st, n, pb->row_ptr,
                       pb->col_idx, J, x, b, w.V, w.sc, 0, wc);
    hipLaunchKernelGGL(k_gm_norm0, dim3(G), dim3(kGmBlock), 0, st, N, w);
    hipLaunchKernelGGL(k_gm_start, dim3(1), dim3(kGmBlock), 0, st, w, G);
    hipLaunchKernelGGL(k_gm_scale0, dim3(G), dim3(kGmBlock), 0, st, N, w);
    OPM_TRY_HIP(hipGetLastError());
    for (int j0 = 0; j0 < m; j0 += chunk) {
      for (int j = j0; j < std::min(m, j0 + chunk); ++j) {
        double* zj = w.Z + (size_t)j * w.Np;
        const double* vj = w.V + (size_t)j * w.Np;
        if (cpr)
          OPM_TRY(cpr_apply(pb, J, ilu, precision, *cpr, vj, zj, st, &w.sc->state));
        else
          OPM_TRY(ilu_apply(pb, ilu, precision, vj, zj, st, &w.sc->state));
        if (ws) OPM_TRY(well_op(*ws, zj, &w.sc->state, st));
        hipLaunchKernelGGL(k_gm_spmv<false>, dim3(Gs), dim3(kBlock), 0, st, n, pb->row_ptr,
                           pb->col_idx, J, zj, nullptr, w.w, w.sc, (int)kGmRunning, wc);
        if (j < 4)
          launch_projections<4>(w, j, N, G, st);
        else if (j < 8)
          launch_projections<8>(w, j, N, G, st);
        else if (j < 16)
          launch_projections<16>(w, j, N, G, st);
        else
          launch_projections<32>(w, j, N, G, st);
        hipLaunchKernelGGL(k_gm_rotate, dim3(G), dim3(kGmBlock), 0, st, N, w, j, G);
        OPM_TRY_HIP(hipGetLastError());
      }
      OPM_TRY(read_view(w, &v, st));
      if (v.state != kGmRunning) break;
    }
    // the state was read after the last chunk: k_used is final
    if (v.k_used <= 4)
      launch_finish<4>(w, x, N, G, st);
    else if (v.k_used <= 8)
      launch_finish<8>(w, x, N, G, st);
    else if (v.k_used <= 16)
      launch_finish<16>(w, x, N, G, st);
    else
      launch_finish<32>(w, x, N, G, st);
    hipLaunchKernelGGL(k_gm_close, dim3(1), dim3(64), 0, st, w);
    OPM_TRY_HIP(hipGetLastError());
    OPM_TRY(read_view(w, &v, st));
    if (v.state == kGmDone) break;
    if (cycle > maxit + 1) {   // cannot happen: every cycle adds an iteration or stops
      v.status = OPM_ENOTCONV;
      break;
    }
  }
  if (rep) {
    rep->status = v.status;
    rep->half = 0;
    rep->its = v.its;
    rep->rel_res = v.relres;
  }
  return OPM_OK;
}

}  // namespace opm
