// Block-CSR SpMV and right-preconditioned BiCGStab (paper sec. 2.3.1, the
// default Krylov method; van der Vorst's stabilised BiCG, x0 = 0, stopping on
// ||r||_2 <= rtol ||b||_2).
//
// The iteration runs without host round trips: every scalar (rho, alpha,
// omega, norms) lives in device memory, every dot product is a two-stage
// fixed-order reduction whose per-workgroup partials are summed by the
// consuming kernel itself (same order in every workgroup, so all of them see
// bit-identical scalars), and a small state word (running / half-step exit /
// done) lets kernels of an iteration that is no longer needed return at once.
// The host only enqueues iterations in chunks and reads the state word
// between chunks.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "cpr_dev.h"
#include "krylov_dev.h"
#include "solver_dev.h"

namespace opm {

int ilu_apply(const opm_problem* pb, void* ilu, int precision, const double* r, double* x,
              hipStream_t s, const int32_t* skip);
int ilu_apply_fused(const opm_problem* pb, void* ilu, int precision, int mode,
                    const kry::Fused& f, double* x, hipStream_t s);
int sweep_mode(const opm_problem* pb, int precision = OPM_PREC_FP64);

namespace {

using kry::kDone;
using kry::kHalfPending;
using kry::kMaxGrid;
using kry::kRunning;
using kry::Scalars;

struct Work {
  double *r, *rh, *p, *v, *ph, *s, *sh, *t;
  double *part_bb, *part_rr, *part_rhr, *part_rv, *part_ss, *part_ts, *part_tt;
  Scalars* sc;
};

inline int vec_grid(int n) { return std::min(kMaxGrid, std::max(1, blocks_for(n, kBlock))); }

Work carve(const opm_problem* pb, void* work) {
  const size_t N = 3 * (size_t)pb->n_cells;
  const size_t Np = (N + 31) / 32 * 32;
  double* d = (double*)work;
  Work w;
  double** vecs[8] = {&w.r, &w.rh, &w.p, &w.v, &w.ph, &w.s, &w.sh, &w.t};
  for (int k = 0; k < 8; ++k) {
    *vecs[k] = d;
    d += Np;
  }
  double** parts[7] = {&w.part_bb, &w.part_rr, &w.part_rhr, &w.part_rv,
                       &w.part_ss, &w.part_ts, &w.part_tt};
  for (int k = 0; k < 7; ++k) {
    *parts[k] = d;
    d += kMaxGrid;
  }
  w.sc = (Scalars*)d;
  return w;
}

__device__ __forceinline__ double sum_partials(const double* part, int G, double* sh) {
  return kry::sum_partials<kBlock>(part, G, sh);
}

template <int NT = kBlock>
__device__ __forceinline__ void store_partial(double v, double* part, double* sh) {
  const double s = block_sum<NT>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Keeps a value's computation (and the loads it waits for) ahead of the
// branches that follow.
__device__ __forceinline__ void keep_value(double v) { asm volatile("" ::"v"(v)); }

using ilu::kSpmvRowsPerWave;
using ilu::spmv_group;
using ilu::spmv_groups;

inline int spmv_blocks(int n) { return blocks_for(spmv_groups(n), kBlock / kWave); }

__global__ __launch_bounds__(kBlock) void k_spmv(int n, const int32_t* row_ptr, const int32_t* col,
                                                  const double* J, const double* x, double* y) {
  const int lane = threadIdx.x & (kWave - 1);
  const int group = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (group >= spmv_groups(n)) return;   // whole wavefront
  int row, comp;
  double yv;
  if (spmv_group(n, row_ptr, col, J, x, group, lane, row, comp, yv)) y[3 * row + comp] = yv;
}

// x = 0, r = r^ = b, p = v = 0; partials of <b,b>.
__global__ __launch_bounds__(kBlock) void k_init(int N, const double* b, double* x, Work w) {
  __shared__ double sh[kBlock / kWave];
  double bb = 0.0;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < N; k += gridDim.x * kBlock) {
    const double v = b[k];
    x[k] = 0.0;
    w.r[k] = v;
    w.rh[k] = v;
    w.p[k] = 0.0;
    w.v[k] = 0.0;
    bb += v * v;
  }
  store_partial(bb, w.part_bb, sh);
}

__global__ __launch_bounds__(kBlock) void k_init2(Work w, int G, double rtol, int maxit) {
  __shared__ double sh[kBlock / kWave];
  const double bb = sum_partials(w.part_bb, G, sh);
  if (threadIdx.x == 0) {
    Scalars& s = *w.sc;
    s.bnorm = sqrt(bb);
    s.tol = rtol * s.bnorm;
    s.rho0 = s.alpha = s.omega = 1.0;
    s.rho = 0.0;
    s.its = 0;
    s.half = 0;
    s.maxit = maxit;
    s.relres = bb == 0.0 ? 0.0 : 1.0;
    s.status = OPM_OK;
    s.state = bb == 0.0 ? kDone : kRunning;
  }
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < G; k += kBlock) {
      w.part_rr[k] = w.part_bb[k];    // r = b
      w.part_rhr[k] = w.part_bb[k];   // <r^, r> = <b, b>
    }
}

// Start of an iteration: convergence / cap / breakdown tests on the
// residual of the previous iteration, then p = r + beta (p - omega v).
__global__ __launch_bounds__(kBlock) void k_begin(int N, Work w, int G) {
  __shared__ double sh[kBlock / kWave];
  __shared__ int word;
  Scalars& s = *w.sc;
  const int state = kry::read_state(w.sc, &word);
  double beta, om;
  if (!kry::begin_iteration<kBlock>(s, state, w.part_rr, w.part_rhr, G, sh, beta, om)) return;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < N; k += gridDim.x * kBlock)
    w.p[k] = w.r[k] + beta * (w.p[k] - om * w.v[k]);
}

// v = A p^ (with standard wells the Schur-complement operator, wc) ;
// partials of <r^, v>.
template <int NT>
__global__ __launch_bounds__(NT) void k_spmv_rv(int n, const int32_t* row_ptr,
                                                     const int32_t* col, const double* J, Work w,
                                                     WellCorr wc) {
  __shared__ double sh[NT / kWave];
  const int state = w.sc->state;   // (not changed by this kernel)
  double acc = 0.0;
  const int lane = threadIdx.x & (kWave - 1), ng = spmv_groups(n);
  const int g0 = blockIdx.x * (NT / kWave) + threadIdx.x / kWave, gs = gridDim.x * (NT / kWave);
  // the first group's products are formed while the state word is read
  int row = 0, comp = 0;
  double yv = 0.0;
  bool own = false;
  if (g0 < ng) own = spmv_group(n, row_ptr, col, J, w.ph, g0, lane, row, comp, yv, wc);
  keep_value(yv);
  if (state != kRunning) return;
  if (own) {
    w.v[3 * row + comp] = yv;
    acc += w.rh[3 * row + comp] * yv;
  }
  for (int g = g0 + gs; g < ng; g += gs) {
    if (spmv_group(n, row_ptr, col, J, w.ph, g, lane, row, comp, yv, wc)) {
      w.v[3 * row + comp] = yv;
      acc += w.rh[3 * row + comp] * yv;
    }
  }
  store_partial<NT>(acc, w.part_rv, sh);
}

// alpha = rho / <r^, v>; s = r - alpha v; partials of <s, s>.
__global__ __launch_bounds__(kBlock) void k_s(int N, Work w, int G) {
  __shared__ double sh[kBlock / kWave];
  __shared__ int word;
  Scalars& sc = *w.sc;
  const int state = kry::read_state(w.sc, &word);
  double alpha;
  if (!kry::alpha_step<kBlock>(sc, state, w.part_rv, G, sh, alpha)) return;
  double ss = 0.0;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < N; k += gridDim.x * kBlock) {
    const double v = w.r[k] - alpha * w.v[k];
    w.s[k] = v;
    ss += v * v;
  }
  store_partial(ss, w.part_ss, sh);
}

// Half-step exit test ||s|| <= tol (one workgroup).
__global__ __launch_bounds__(kBlock) void k_s_check(Work w, int G) {
  __shared__ double sh[kBlock / kWave];
  __shared__ int word;
  const int state = kry::read_state(w.sc, &word);
  kry::half_step_check<kBlock>(*w.sc, state, w.part_ss, G, sh);
}

// t = A s^ ; partials of <t, s> and <t, t>.  With CHECK, first the
// half-step exit test on the nss partials of <s, s> (written by the sweep
// that computed s).
template <bool CHECK, int NT>
__global__ __launch_bounds__(NT) void k_spmv_t(int n, const int32_t* row_ptr,
                                                    const int32_t* col, const double* J, Work w,
                                                    int nss, WellCorr wc) {
  __shared__ double sh[NT / kWave];
  __shared__ int word;
  // the state word (read once for the workgroup) and the partials of
  // <s, s> go out first, the first group's products are formed while they
  // are in flight
  int st0 = 0;
  if (threadIdx.x == 0) st0 = w.sc->state;
  const double pss = CHECK ? kry::partial_first(w.part_ss, nss) : 0.0;
  const int lane = threadIdx.x & (kWave - 1), ng = spmv_groups(n);
  const int g0 = blockIdx.x * (NT / kWave) + threadIdx.x / kWave, gs = gridDim.x * (NT / kWave);
  int row = 0, comp = 0;
  double yv = 0.0;
  bool own = false;
  if (g0 < ng) own = spmv_group(n, row_ptr, col, J, w.sh, g0, lane, row, comp, yv, wc);
  keep_value(yv);
  keep_value(pss);
  if (threadIdx.x == 0) word = st0;
  __syncthreads();
  const int state = word;
  if (CHECK) {
    const double share = kry::partials_share<NT>(w.part_ss, nss, pss);
    if (!kry::half_step_check_share<NT>(*w.sc, state, share, sh)) return;
  } else if (state != kRunning) {
    return;
  }
  double ts = 0.0, tt = 0.0;
  if (own) {
    w.t[3 * row + comp] = yv;
    ts += yv * w.s[3 * row + comp];
    tt += yv * yv;
  }
  for (int g = g0 + gs; g < ng; g += gs) {
    if (spmv_group(n, row_ptr, col, J, w.sh, g, lane, row, comp, yv, wc)) {
      w.t[3 * row + comp] = yv;
      ts += yv * w.s[3 * row + comp];
      tt += yv * yv;
    }
  }
  store_partial<NT>(ts, w.part_ts, sh);
  store_partial<NT>(tt, w.part_tt, sh);
}

// omega = <t,s>/<t,t>; x += alpha p^ + omega s^; r = s - omega t; partials of
// <r, r> and <r^, r>.  On a half-step exit only x += alpha p^.
__global__ __launch_bounds__(kBlock) void k_x(int N, double* x, Work w, int G) {
  __shared__ double sh[kBlock / kWave];
  Scalars& sc = *w.sc;
  const int state = sc.state;
  const double alpha = sc.alpha;
  const double rho = sc.rho;   // (for the updates at the end)
  const int its = sc.its;
  // the first partials and the first element's vectors go out with the
  // scalars (clamped indices: no branch around the loads)
  const double pts = kry::partial_first(w.part_ts, G);
  const double ptt = kry::partial_first(w.part_tt, G);
  const int k0 = blockIdx.x * kBlock + threadIdx.x, ks = gridDim.x * kBlock;
  const int kc = min(k0, N - 1);
  const double x0 = x[kc], ph0 = w.ph[kc], sh0 = w.sh[kc], s0 = w.s[kc], t0 = w.t[kc],
               rh0 = w.rh[kc];
  keep_value(pts);
  keep_value(ptt);
  keep_value(x0);
  keep_value(ph0);
  keep_value(sh0);
  keep_value(s0);
  keep_value(t0);
  keep_value(rh0);
  if (state == kHalfPending) {
    for (int k = k0; k < N; k += ks) x[k] += alpha * w.ph[k];
    return;
  }
  if (state != kRunning) return;
  const double ts = block_sum<kBlock>(kry::partials_share<kBlock>(w.part_ts, G, pts), sh);
  const double tt = block_sum<kBlock>(kry::partials_share<kBlock>(w.part_tt, G, ptt), sh);
  if (tt == 0.0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc.status = OPM_EBREAKDOWN;
      sc.state = kDone;
    }
    return;
  }
  const double omega = ts / tt;
  double rr = 0.0, rhr = 0.0;
  if (k0 < N) {
    x[k0] = x0 + (alpha * ph0 + omega * sh0);
    const double r = s0 - omega * t0;
    w.r[k0] = r;
    rr += r * r;
    rhr += rh0 * r;
  }
  for (int k = k0 + ks; k < N; k += ks) {
    x[k] += alpha * w.ph[k] + omega * w.sh[k];
    const double r = w.s[k] - omega * w.t[k];
    w.r[k] = r;
    rr += r * r;
    rhr += w.rh[k] * r;
  }
  store_partial(rr, w.part_rr, sh);
  store_partial(rhr, w.part_rhr, sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc.omega = omega;
    sc.rho0 = rho;
    sc.its = its + 1;
  }
}

}  // namespace

// Iterations enqueued between two reads of the state word (0 = automatic).
int g_krylov_chunk = 0;
// Enqueue the chunks of iterations as a replayed HIP graph (1) or kernel by
// kernel (0).  Measured on the 9000-cell system with block ILU0: 4.39M
// cell-Newton-iterations/s kernel by kernel, 4.53M replayed (chunks of 6),
// 4.57M replayed in chunks of 8.
int g_krylov_graph = 1;
extern int g_sweep_mode;
extern int g_sweep_kernel;
extern int g_plane_sweep;
extern int g_plane_spin;
extern int g_block_depth;

int chunk_size(const opm_problem* pb) {
  if (g_krylov_chunk > 0) return g_krylov_chunk;
  const int mode = sweep_mode(pb);
  return mode == 1 ? 3 : mode == 2 ? 8 : 6;
}

size_t krylov_bytes(const opm_problem* pb) {
  const size_t N = 3 * (size_t)pb->n_cells;
  const size_t Np = (N + 31) / 32 * 32;
  return sizeof(double) * (8 * Np + 7 * kMaxGrid) + sizeof(Scalars) + 256;
}

int spmv(const opm_problem* pb, const double* J, const double* x, double* y, hipStream_t s) {
  if (pb->n_cells == 0) return OPM_OK;
  hipLaunchKernelGGL(k_spmv, dim3(spmv_blocks(pb->n_cells)), dim3(kBlock), 0, s,
                     pb->n_cells, pb->row_ptr, pb->col_idx, J, x, y);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

namespace {

// Graphs of a chunk of iterations, one per distinct set of launch
// arguments (the problem, the buffers, the precision, the launch-shape
// options and the device), kept until the process ends or evicted oldest
// first.  A chunk only launches kernels (no memset, no copy), and every
// kernel reads the iteration's state from device memory, so a replay is
// the same work as enqueuing the chunk again.  Besides the arguments
// themselves, enqueuing reads two host arrays whose contents set launch
// ranges baked into the graph: the level schedule (per-level launches of
// the ILU(0) of large systems) and the CPR hierarchy's level sizes; their
// contents enter the key through a hash, so a new schedule or hierarchy at
// a reused host address does not replay a stale graph.
struct ChunkKey {
  opm_problem pb;
  uint64_t host_hash;        // FNV-1a of level_ptr_h[0..n_levels] and *pb.amg
  const double* J;
  const void* ilu;
  const double* x;
  const void* work;
  hipStream_t st;
  int precision, chunk, device, sweep_mode, sweep_kernel, block_depth, plane_sweep, plane_spin;
  WellSchur ws;              // standard wells (all zero without)
  const double* cpr_base;    // CPR workspace (null without)
};
struct ChunkGraph {
  ChunkKey key;
  hipGraphExec_t exec;
};
std::vector<ChunkGraph> g_chunk_graphs;
constexpr size_t kMaxChunkGraphs = 16;
// Guards the graph cache and the capture streams: calls from several host
// threads look up, capture and evict one at a time.
std::mutex g_graph_mutex;

uint64_t fnv1a(uint64_t h, const void* data, size_t bytes) {
  const unsigned char* c = static_cast<const unsigned char*>(data);
  for (size_t k = 0; k < bytes; ++k) h = (h ^ c[k]) * 1099511628211ull;
  return h;
}

uint64_t host_schedule_hash(const opm_problem* pb) {
  uint64_t h = 1469598103934665603ull;
  if (pb->level_ptr_h)
    h = fnv1a(h, pb->level_ptr_h, sizeof(int32_t) * ((size_t)pb->n_levels + 1));
  if (pb->amg) h = fnv1a(h, pb->amg, sizeof(opm_amg));
  return h;
}

bool same_key(const ChunkKey& a, const ChunkKey& b) { return std::memcmp(&a, &b, sizeof a) == 0; }

// Capture needs a stream other than the null stream; capturing runs
// nothing, so the graph is recorded on a stream of the library's own (one
// per device, default priority) and launched on the caller's.
constexpr int kMaxDevices = 64;
hipStream_t g_capture_stream[kMaxDevices] = {};

int capture_stream(int device, hipStream_t* out) {
  if (device < 0 || device >= kMaxDevices) return OPM_EINVAL;
  if (!g_capture_stream[device])
    OPM_TRY_HIP(hipStreamCreateWithFlags(&g_capture_stream[device], hipStreamNonBlocking));
  *out = g_capture_stream[device];
  return OPM_OK;
}

}  // namespace

// Enqueue the whole solve; returns after reading the final scalars.
// ws (may be null): standard wells, solved through their Schur complement.
// cpr (may be null): CPR-AMG set up for J, with ilu as its second stage.
namespace {
// Per host thread and device: pinned host memory for two reads of the
// iteration's scalars and the events the host polls for their copies (the
// next chunk's read can be queued while the host waits for one); pending:
// the read of a chunk queued after the last solve's final read; last_its:
// the iterations the last solve took.
struct StateRead {
  int device = -1;
  hipEvent_t ev[2] = {nullptr, nullptr};
  Scalars* host = nullptr;
  hipEvent_t pending = nullptr;
  int last_its = 0;
};

StateRead* state_read() {
  static thread_local std::vector<StateRead> reads;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  for (auto& r : reads)
    if (r.device == dev) return &r;
  StateRead r;
  r.device = dev;
  void* p = nullptr;
  for (auto& e : r.ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  if (hipHostMalloc(&p, 2 * sizeof(Scalars), hipHostMallocDefault) != hipSuccess) return nullptr;
  r.host = (Scalars*)p;
  reads.push_back(r);
  return &reads.back();
}
}  // namespace

int bicgstab(const opm_problem* pb, const double* J, void* ilu, int precision, const double* b,
             double* x, double rtol, int maxit, void* work, opm_solve_report* rep,
             hipStream_t st, const WellSchur* ws, const CprWork* cpr) {
  StateRead* sr = state_read();
  if (!sr) return OPM_EHIP;
  // the last solve's read of a chunk queued after it ended has landed before
  // its buffer is written again
  if (sr->pending) {
    OPM_TRY_HIP(spin_wait(sr->pending));
    sr->pending = nullptr;
  }
  const int n = pb->n_cells, N = 3 * n;
  Work w = carve(pb, work);
  const int G = vec_grid(N), Gr = std::min(kMaxGrid, std::max(1, spmv_blocks(n)));
  hipLaunchKernelGGL(k_init, dim3(G), dim3(kBlock), 0, st, N, b, x, w);
  hipLaunchKernelGGL(k_init2, dim3(1), dim3(kBlock), 0, st, w, G, rtol, maxit);
  OPM_TRY_HIP(hipGetLastError());
  const int chunk = chunk_size(pb);
  // block ILU0 with one workgroup per subdomain: the p and s updates (and
  // the tests before them) run inside the preconditioner sweeps
  const bool fused = sweep_mode(pb, precision) == 2 && pb->n_sub <= kMaxGrid && !cpr;
  kry::Fused fb{w.r, w.p, w.v, nullptr, w.part_rr, w.part_rhr, G, nullptr, w.sc};
  kry::Fused fs{w.r, nullptr, w.v, w.s, w.part_rv, nullptr, Gr, w.part_ss, w.sc};
  Scalars host;
  const WellCorr wc = ws ? ws->wc() : WellCorr{nullptr, nullptr, nullptr};
  auto prec = [&](const double* r, double* z, hipStream_t st) -> int {
    return cpr ? cpr_apply(pb, J, ilu, precision, *cpr, r, z, st, &w.sc->state)
               : ilu_apply(pb, ilu, precision, r, z, st, &w.sc->state);
  };
  // With the grid capped at kMaxGrid workgroups (large systems) the two
  // SpMVs with reductions run 512-thread workgroups, twice the resident
  // waves of 256-thread ones over the same number of partial sums.
  const bool wide = spmv_blocks(n) > kMaxGrid;
  auto spmv_rv = [&](hipStream_t st) {
    if (wide)
      hipLaunchKernelGGL(k_spmv_rv<2 * kBlock>, dim3(Gr), dim3(2 * kBlock), 0, st, n,
                         pb->row_ptr, pb->col_idx, J, w, wc);
    else
      hipLaunchKernelGGL(k_spmv_rv<kBlock>, dim3(Gr), dim3(kBlock), 0, st, n, pb->row_ptr,
                         pb->col_idx, J, w, wc);
  };
  auto spmv_t = [&](hipStream_t st, bool check) {
    const int nss = check ? pb->n_sub : 0;
    if (wide && check)
      hipLaunchKernelGGL((k_spmv_t<true, 2 * kBlock>), dim3(Gr), dim3(2 * kBlock), 0, st, n,
                         pb->row_ptr, pb->col_idx, J, w, nss, wc);
    else if (wide)
      hipLaunchKernelGGL((k_spmv_t<false, 2 * kBlock>), dim3(Gr), dim3(2 * kBlock), 0, st, n,
                         pb->row_ptr, pb->col_idx, J, w, nss, wc);
    else if (check)
      hipLaunchKernelGGL((k_spmv_t<true, kBlock>), dim3(Gr), dim3(kBlock), 0, st, n,
                         pb->row_ptr, pb->col_idx, J, w, nss, wc);
    else
      hipLaunchKernelGGL((k_spmv_t<false, kBlock>), dim3(Gr), dim3(kBlock), 0, st, n,
                         pb->row_ptr, pb->col_idx, J, w, nss, wc);
  };
  auto enqueue_chunk = [&](hipStream_t st) -> int {
    for (int c = 0; c < chunk; ++c) {
      if (fused) {
        OPM_TRY(ilu_apply_fused(pb, ilu, precision, kry::kFuseBegin, fb, w.ph, st));
        if (ws) OPM_TRY(well_op(*ws, w.ph, &w.sc->state, st));
        spmv_rv(st);
        OPM_TRY(ilu_apply_fused(pb, ilu, precision, kry::kFuseS, fs, w.sh, st));
        if (ws) OPM_TRY(well_op(*ws, w.sh, &w.sc->state, st));
        spmv_t(st, true);
      } else {
        hipLaunchKernelGGL(k_begin, dim3(G), dim3(kBlock), 0, st, N, w, G);
        OPM_TRY(prec(w.p, w.ph, st));
        if (ws) OPM_TRY(well_op(*ws, w.ph, &w.sc->state, st));
        spmv_rv(st);
        hipLaunchKernelGGL(k_s, dim3(G), dim3(kBlock), 0, st, N, w, Gr);
        hipLaunchKernelGGL(k_s_check, dim3(1), dim3(kBlock), 0, st, w, G);
        OPM_TRY(prec(w.s, w.sh, st));
        if (ws) OPM_TRY(well_op(*ws, w.sh, &w.sc->state, st));
        spmv_t(st, false);
      }
      hipLaunchKernelGGL(k_x, dim3(G), dim3(kBlock), 0, st, N, x, w, Gr);
      OPM_TRY_HIP(hipGetLastError());
    }
    return OPM_OK;
  };
  ChunkKey key;
  std::memset(&key, 0, sizeof key);
  if (g_krylov_graph == 1) {
    key.pb = *pb;
    key.host_hash = host_schedule_hash(pb);
    key.J = J;
    key.ilu = ilu;
    key.x = x;
    key.work = work;
    key.st = st;
    key.precision = precision;
    key.chunk = chunk;
    OPM_TRY_HIP(hipGetDevice(&key.device));
    key.sweep_mode = g_sweep_mode;
    if (ws) std::memcpy(&key.ws, ws, sizeof *ws);   // ws is built zero-filled (padding too)
    key.cpr_base = cpr ? cpr->w : nullptr;
    key.sweep_kernel = g_sweep_kernel;
    key.block_depth = g_block_depth;
    key.plane_sweep = g_plane_sweep;
    key.plane_spin = g_plane_spin;
  }
  // One chunk and the read of the state after it (pass p: buffer p % 2).
  auto enqueue_pass = [&](int pass) -> int {
    hipGraphExec_t exec = nullptr;
    std::unique_lock<std::mutex> lock(g_graph_mutex, std::defer_lock);
    if (g_krylov_graph == 1) {
      lock.lock();
      for (auto& cg : g_chunk_graphs)
        if (same_key(cg.key, key)) exec = cg.exec;
    }
    // a chunk with no graph yet runs eagerly the first time (which also sets
    // the kernels' LDS attributes outside any capture) and is captured the
    // next time; once captured, every chunk of every solve with the same
    // arguments is a replay
    if (g_krylov_graph == 1 && (exec || pass > 0)) {
      if (!exec) {
        hipGraph_t graph;
        hipStream_t cs;
        OPM_TRY(capture_stream(key.device, &cs));
        OPM_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const int cst = enqueue_chunk(cs);
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (cst != OPM_OK) return cst;
        OPM_TRY_HIP(e);
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        OPM_TRY_HIP(ei);
        if (g_chunk_graphs.size() >= kMaxChunkGraphs) {
          (void)hipGraphExecDestroy(g_chunk_graphs.front().exec);
          g_chunk_graphs.erase(g_chunk_graphs.begin());
        }
        g_chunk_graphs.push_back({key, exec});
      }
      OPM_TRY_HIP(hipGraphLaunch(exec, st));
    } else {
      if (lock.owns_lock()) lock.unlock();
      OPM_TRY(enqueue_chunk(st));
    }
    if (lock.owns_lock()) lock.unlock();
    // a final begin turns a pending half-step exit into done and performs the
    // convergence test of the last full iteration
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(kBlock), 0, st, 0, w, G);
    OPM_TRY_HIP(hipMemcpyAsync(sr->host + (pass & 1), w.sc, sizeof(Scalars),
                               hipMemcpyDeviceToHost, st));
    OPM_TRY_HIP(hipEventRecord(sr->ev[pass & 1], st));
    return OPM_OK;
  };
  // A chunk goes out before the read of the one ahead of it where the last
  // solve's iterations say that it will be needed to the full (half a chunk
  // to spare), so that the device runs it while the host waits for that
  // read; otherwise the next chunk waits for the read.  A chunk queued past
  // the end of the solve finds the state done in every kernel and changes
  // nothing.
  int queued = 0;
  auto queue = [&]() -> int {
    OPM_TRY(enqueue_pass(queued));
    ++queued;
    return OPM_OK;
  };
  auto needed = [&](int q) {
    return (q + 1) * chunk + chunk / 2 <= sr->last_its && q * chunk <= maxit + 2;
  };
  OPM_TRY(queue());
  if (needed(1)) OPM_TRY(queue());
  int pass = 0;
  for (;; ++pass) {
    OPM_TRY_HIP(spin_wait(sr->ev[pass & 1]));
    host = sr->host[pass & 1];
    if (host.state == kDone) break;
    if ((pass + 1) * chunk > maxit + 2) {   // cannot happen: k_begin enforces maxit
      host.status = OPM_ENOTCONV;
      break;
    }
    if (queued == pass + 1) OPM_TRY(queue());
    if (queued == pass + 2 && needed(pass + 2)) OPM_TRY(queue());
  }
  sr->pending = queued > pass + 1 ? sr->ev[(pass + 1) & 1] : nullptr;
  sr->last_its = host.its;
  if (rep) {
    rep->status = host.status;
    rep->half = host.half;
    rep->its = host.its;
    rep->rel_res = host.relres;
  }
  return OPM_OK;
}

}  // namespace opm
