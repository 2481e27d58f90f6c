// Batched ensemble: many independent reservoir models (members with their own
// grids, rock and wells) advanced over several report steps in ONE launch of
// a persistent kernel.  One workgroup owns one member and runs that member's
// whole time loop on the device: time-step cutting (paper sec. 2.3), the
// Newton iteration (eq. linsystem), residual/Jacobian assembly (sec. 2.1.1,
// sec. 2.4), block ILU(0) and BiCGStab (sec. 2.3.1), the Appleyard chop and
// the CNV/MB test.  Workgroups never wait for each other, so members of
// different sizes and different Newton histories proceed independently and
// the launch contains no host decision: it can be captured in a graph as a
// single node.
//
// Inside a workgroup every vector operation is a strided loop over the
// member's rows, every dot product a fixed-order workgroup reduction, and
// the ILU(0) factorisation and sweeps walk the member's level schedule with
// workgroup barriers (the same device code as the single-system path, with
// the previous level kept in an LDS window).  The arithmetic per row is the
// single-system path's, so a member's result equals a single-system run of
// that member up to the order of summation in the reductions.
#include <algorithm>
#include <cstring>
#include <vector>

#include "assemble_dev.h"
#include "solver_dev.h"

namespace opm {
namespace {

using asmdev::AsmArgs;
using asmdev::CellAcc;
using asmdev::FaceProps;
using ilu::IluView;
using ilu::Topo;

struct EnsMember {
  opm_problem pb;
  double* y;
  double *y_save, *acc0, *R, *J, *d;
  void* ilu;
  double *r, *rh, *p, *v, *ph, *s, *sh, *t;
  double* backup;        // copy of y kept by the autotuner between trials
  int32_t ring;          // 1: ILU(0) sweeps through the LDS ring, 0: the LDS window
  uint32_t ring_mask;    // ring capacity - 1 (rows)
};

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

size_t member_bytes(const opm_problem& pb, int precision) {
  const size_t N = 3 * (size_t)pb.n_cells;
  const size_t ilu = precision == OPM_PREC_MIXED ? ilu::view_bytes<float>(pb.n_cells)
                                                 : ilu::view_bytes<double>(pb.n_cells);
  return 13 * al256(sizeof(double) * N) + al256(sizeof(double) * 9 * (size_t)pb.nnzb) +
         al256(ilu);
}

// LDS of the kernel: reduction scratch, sweep storage (the largest over the
// members of the window, 2 levels x 3 values per row, or the ring), factor
// window (previous level's pivots, when enabled).
constexpr size_t kEnsLds = 150 * 1024;
constexpr int kMaxFacWindowLevel = 640;

struct LdsPlan {
  size_t red, sweep, fac, total;
};

inline size_t window_bytes(size_t tsize, int max_level) { return tsize * 2 * 3 * (size_t)max_level; }
inline size_t ring_bytes(size_t tsize, const opm_problem& pb) {
  return tsize * 3 * (size_t)ilu::ring_rows(pb.sweep_span, pb.max_level);
}

LdsPlan lds_plan(size_t tsize, int threads, size_t sweep_bytes, int max_level, bool fac_window) {
  LdsPlan p;
  p.red = sizeof(double) * 2 * (threads / kWave);
  p.sweep = al256(sweep_bytes);
  p.fac = fac_window ? sizeof(double) * 2 * 9 * (size_t)max_level : 0;
  p.total = al256(p.red) + p.sweep + p.fac;
  return p;
}

template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red) {
  return block_sum<NT>(v, red);
}
template <int NT>
__device__ __forceinline__ double wg_max(double v, double* red) {
  return block_max<NT>(v, red);
}

// ---------------------------------------------------------------- BiCGStab
// Right-preconditioned BiCGStab for J d = b by one workgroup (x0 = 0).
template <typename T, int NT>
__device__ int wg_bicgstab(const EnsMember& M, const Topo& tp, IluView<T> iv, const double* b,
                           double* x, double rtol, int maxit, double* red, T* swin, bool ring,
                           int* its_out) {
  const int n = M.pb.n_cells, N = 3 * n;
  const int tid = threadIdx.x;
  double bb = 0.0;
  for (int k = tid; k < N; k += NT) {
    const double bv = b[k];
    x[k] = 0.0;
    M.r[k] = bv;
    M.rh[k] = bv;
    M.p[k] = 0.0;
    M.v[k] = 0.0;
    bb += bv * bv;
  }
  bb = wg_sum<NT>(bb, red);
  *its_out = 0;
  if (bb == 0.0) return OPM_OK;
  const double tol = rtol * sqrt(bb);
  double rho0 = 1.0, alpha = 1.0, omega = 1.0;
  double rho = bb;   // <r^, r> with r = r^ = b
  for (int it = 1; it <= maxit; ++it) {
    *its_out = it;
    if (fabs(rho) < 1e-300) return OPM_EBREAKDOWN;
    const double beta = it == 1 ? 0.0 : (rho / rho0) * (alpha / omega);
    for (int k = tid; k < N; k += NT) M.p[k] = M.r[k] + beta * (M.p[k] - omega * M.v[k]);
    __syncthreads();
    if (ring)
      ilu::apply_levels_ring<T, NT>(tp, iv, M.p, M.ph, swin, M.ring_mask);
    else
      ilu::apply_levels_wg<T, NT>(tp, iv, M.p, M.ph, swin);
    double rv = 0.0;
    for (int i = tid; i < n; i += NT) {
      double y3[3];
      ilu::spmv_row(M.pb.row_ptr, M.pb.col_idx, M.J, M.ph, i, y3);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        M.v[3 * i + c] = y3[c];
        rv += M.rh[3 * i + c] * y3[c];
      }
    }
    rv = wg_sum<NT>(rv, red);
    if (rv == 0.0) return OPM_EBREAKDOWN;
    alpha = rho / rv;
    double ss = 0.0;
    for (int k = tid; k < N; k += NT) {
      const double sv = M.r[k] - alpha * M.v[k];
      M.s[k] = sv;
      ss += sv * sv;
    }
    ss = wg_sum<NT>(ss, red);
    if (sqrt(ss) <= tol) {
      for (int k = tid; k < N; k += NT) x[k] += alpha * M.ph[k];
      __syncthreads();
      return OPM_OK;
    }
    if (ring)
      ilu::apply_levels_ring<T, NT>(tp, iv, M.s, M.sh, swin, M.ring_mask);
    else
      ilu::apply_levels_wg<T, NT>(tp, iv, M.s, M.sh, swin);
    double ts = 0.0, tt = 0.0;
    for (int i = tid; i < n; i += NT) {
      double y3[3];
      ilu::spmv_row(M.pb.row_ptr, M.pb.col_idx, M.J, M.sh, i, y3);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        M.t[3 * i + c] = y3[c];
        ts += y3[c] * M.s[3 * i + c];
        tt += y3[c] * y3[c];
      }
    }
    ts = wg_sum<NT>(ts, red);
    tt = wg_sum<NT>(tt, red);
    if (tt == 0.0) return OPM_EBREAKDOWN;
    omega = ts / tt;
    double rr = 0.0, rhr = 0.0;
    for (int k = tid; k < N; k += NT) {
      x[k] += alpha * M.ph[k] + omega * M.sh[k];
      const double rv2 = M.s[k] - omega * M.t[k];
      M.r[k] = rv2;
      rr += rv2 * rv2;
      rhr += M.rh[k] * rv2;
    }
    rr = wg_sum<NT>(rr, red);
    rhr = wg_sum<NT>(rhr, red);
    if (sqrt(rr) <= tol) return OPM_OK;
    if (omega == 0.0) return OPM_EBREAKDOWN;
    rho0 = rho;
    rho = rhr;
  }
  return OPM_ENOTCONV;
}

// ------------------------------------------------------------------ Newton
template <typename T, int NT, bool FACWIN>
__device__ int wg_newton(const EnsMember& M, const Topo& tp, IluView<T> iv, double h,
                         const opm_newton_opts& o, double* red, T* swin, bool ring, double* fwin,
                         int* flag, opm_ensemble_report& rep) {
  const int n = M.pb.n_cells;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += NT) {
    FaceProps P;
    CellAcc A;
    asmdev::properties<false>(M.pb.fluid, M.y_save[3 * i], M.y_save[3 * i + 1],
                              M.y_save[3 * i + 2], 0, P, &A);
#pragma unroll
    for (int c = 0; c < 3; ++c) M.acc0[3 * i + c] = A.A[c].v;
  }
  __syncthreads();
  AsmArgs a;
  a.n = n;
  a.y = M.y;
  a.acc0 = M.acc0;
  a.dt = h;
  a.trans = M.pb.trans;
  a.pv = M.pb.pore_vol;
  a.depth = M.pb.depth;
  a.row_ptr = M.pb.row_ptr;
  a.col_idx = M.pb.col_idx;
  a.blk_face = M.pb.blk_face;
  a.cell_conn_ptr = M.pb.cell_conn_ptr;
  a.cell_conn = M.pb.cell_conn;
  a.conn_kind = M.pb.conn_kind;
  a.conn_phase = M.pb.conn_phase;
  a.conn_wi = M.pb.conn_wi;
  a.conn_rate = M.pb.conn_rate;
  a.conn_bhp = M.pb.conn_bhp;
  a.fluid = M.pb.fluid;
  a.meaning = nullptr;   // dead oil only (opm_ensemble_prepare rejects live oil)
  a.n_wells = 0;         // and the simplified wells only
  a.conn_well = nullptr;
  a.well_state = nullptr;
  a.Cw = nullptr;
  a.R = M.R;
  a.J = M.J;
  a.partials = nullptr;
  for (int it = 0;; ++it) {
    double cmax[3] = {0.0, 0.0, 0.0}, sums[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = tid; i < n; i += NT) {
      double part[kNormStride];
      asmdev::assemble_row<false>(a, i, h, part);
#pragma unroll
      for (int c = 0; c < 3; ++c) cmax[c] = nan_max(cmax[c], part[c]);
#pragma unroll
      for (int k = 0; k < 7; ++k) sums[k] += part[3 + k];
    }
    double cnv[3], mb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) cnv[c] = wg_max<NT>(cmax[c], red);
#pragma unroll
    for (int k = 0; k < 7; ++k) sums[k] = wg_sum<NT>(sums[k], red);
    double cm = 0.0, mm = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mb[c] = h * fabs(sums[c]) / ((sums[3 + c] / n) * sums[6]);
      cm = nan_max(cm, cnv[c]);
      mm = nan_max(mm, mb[c]);
      rep.cnv[c] = cnv[c];
      rep.mb[c] = mb[c];
    }
    if (!isfinite(cm) || !isfinite(mm)) return OPM_ENONFINITE;
    if (cm <= o.tol_cnv && mm <= o.tol_mb) return OPM_OK;
    if (it >= o.max_newton) return OPM_ENOTCONV;
    // ILU(0)
    for (int pos = tid; pos < n; pos += NT) ilu::pack_row<T>(tp, M.J, iv, pos);
    if (tid == 0) *flag = 0;
    __syncthreads();
    ilu::factor_levels_wg<T, FACWIN, NT, false>(tp, M.J, iv, flag, fwin);
    if (*flag != 0) return OPM_ESINGULAR;
    // BiCGStab: J d = R, Newton update y <- y - chop(d)
    int lits = 0;
    const int st = wg_bicgstab<T, NT>(M, tp, iv, M.R, M.d, o.lin_rtol, o.lin_maxit, red, swin,
                                      ring, &lits);
    rep.lin_its += lits;
    if (st != OPM_OK) return st;
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int i = tid; i < n; i += NT) {
      const double p = M.y[3 * i];
      double dp = -M.d[3 * i];
      const double lim = o.dp_max_rel * fabs(p);
      if (dp > lim) dp = lim;
      if (dp < -lim) dp = -lim;
      double dsw = -M.d[3 * i + 1], dsg = -M.d[3 * i + 2];
      const double mx = fmax(fabs(dsw), fabs(dsg));
      if (mx > o.ds_max) {
        const double sc = o.ds_max / mx;
        dsw *= sc;
        dsg *= sc;
      }
      const double y0 = p + dp, y1 = M.y[3 * i + 1] + dsw, y2 = M.y[3 * i + 2] + dsg;
      M.y[3 * i] = y0;
      M.y[3 * i + 1] = y1;
      M.y[3 * i + 2] = y2;
      if (!isfinite(y0) || !isfinite(y1) || !isfinite(y2)) *flag = 1;
    }
    __syncthreads();
    rep.newton_its += 1;
    rep.cell_newton_its += (double)n;
    if (*flag != 0) return OPM_ENONFINITE;
  }
}

template <int NT>
__device__ __forceinline__ void wg_copy(double* dst, const double* src, int N) {
  for (int k = threadIdx.x; k < N; k += NT) dst[k] = src[k];
  __syncthreads();
}

template <typename T, int NT, bool FACWIN>
__global__ __launch_bounds__(NT) void k_ensemble(const EnsMember* tab, int n_steps, double dt_report,
                                                  opm_newton_opts o, size_t red_bytes,
                                                  size_t sweep_bytes, opm_ensemble_report* reps) {
  extern __shared__ double smem[];
  __shared__ int flag;
  double* red = smem;
  T* swin = reinterpret_cast<T*>(reinterpret_cast<char*>(smem) + red_bytes);
  double* fwin = reinterpret_cast<double*>(reinterpret_cast<char*>(smem) + red_bytes + sweep_bytes);
  const EnsMember M = tab[blockIdx.x];
  // the ring is used only if it fits the sweep storage of this launch
  const bool ring = M.ring && (size_t)(M.ring_mask + 1u) * 3u * sizeof(T) <= sweep_bytes;
  const Topo tp = ilu::topo_of(&M.pb);
  IluView<T> iv = ilu::view<T>(&M.pb, M.ilu);
  opm_ensemble_report rep = {};
  const int N = 3 * M.pb.n_cells;
  int status = OPM_OK;
  for (int step = 0; step < n_steps && status == OPM_OK; ++step) {
    wg_copy<NT>(M.y_save, M.y, N);
    double t = 0.0, dt_try = dt_report;
    int cuts = 0;
    while (dt_report - t > 1e-9 * dt_report) {
      const double h = fmin(dt_try, dt_report - t);
      const int st = wg_newton<T, NT, FACWIN>(M, tp, iv, h, o, red, swin, ring, fwin, &flag, rep);
      __syncthreads();
      if (st == OPM_OK) {
        t += h;
        rep.substeps += 1;
        wg_copy<NT>(M.y_save, M.y, N);
      } else {
        wg_copy<NT>(M.y, M.y_save, N);
        dt_try = 0.5 * h;
        rep.cuts += 1;
        if (++cuts > o.max_cuts) {
          status = st;
          break;
        }
      }
    }
    if (status == OPM_OK) rep.steps_done = step + 1;
  }
  rep.status = status;
  if (threadIdx.x == 0) reps[blockIdx.x] = rep;
}

// ------------------------------------------- several workgroups per member
// A member can get several workgroups, each owning a contiguous range of the
// member's block-ILU0 subdomains (sec. 2.5: the couplings between
// subdomains are dropped from the preconditioner only).  A workgroup
// assembles, updates and multiplies the rows of its subdomains and factors
// and sweeps them, walking its part of every local level (no other
// workgroup's rows are involved).  The member's workgroups meet at a barrier
// (an arrival counter and a generation word in device memory, ordered at
// device scope) wherever a phase reads rows of another workgroup (the SpMV's
// neighbours of the preconditioned vectors, the neighbours' state in the next
// assembly) and in every reduction: each workgroup writes its partials, and
// after the barrier every workgroup adds all of them in workgroup order, so
// all take the same decisions.  The waits are bounded: a barrier that gives
// up marks the member failed (OPM_EHIP in its report) and every workgroup of
// the member then stops instead of hanging.  Members get workgroups in
// proportion to their rows, so the largest no longer sets the launch time
// alone.
struct EnsHeader {
  int32_t n_members, precision, max_level, n_wgs;   // n_wgs: entries of the workgroup table
};
struct EnsWg {
  int32_t m;        // member
  int32_t w, g;     // this workgroup's index among the member's g
  int32_t s0, s1;   // subdomains [s0, s1) (0, 1 for a member walked whole)
  int32_t width;    // most rows of its range on one level (the LDS window's)
  int32_t pad[2];
};
struct EnsSync {
  int32_t count, gen, fail, pad[13];   // one 64-byte line per member
};
constexpr int kPartStride = 16;    // doubles per partial slot
constexpr int kMaxEnsWgs = 2048;   // workgroups of one launch

struct Grp {
  int w, g;
  double* part;   // the member's partials: [2][g][kPartStride]
  EnsSync* sync;
  unsigned spin;
  int parity;     // which half of the partials the next reduction uses
};

__device__ bool grp_barrier(const Grp& G, int* word) {
  __syncthreads();
  if (G.g == 1) return true;
  if (threadIdx.x == 0) {
    int ok = __hip_atomic_load(&G.sync->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    if (ok) {
      // the generation before this arrival (it moves only after every arrival)
      const int gen = __hip_atomic_load(&G.sync->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // release: this workgroup's writes; acquire: the earlier arrivals'
      const int arrived =
          __hip_atomic_fetch_add(&G.sync->count, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == G.g - 1) {
        __hip_atomic_store(&G.sync->count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&G.sync->gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        // polls at device scope without invalidating caches, one acquire after
        for (unsigned it = 0;
             __hip_atomic_load(&G.sync->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen;
             ++it) {
          if (it >= G.spin ||
              __hip_atomic_load(&G.sync->fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(4);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    if (!ok) __hip_atomic_store(&G.sync->fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *word = ok;
  }
  __syncthreads();
  return *word != 0;
}

// Sums (max where bit k of MAXMASK is set, NaN-propagating) of K per-thread
// values over the member, the same in every workgroup of the member.
template <int NT, int K, unsigned MAXMASK = 0>
__device__ bool grp_reduce(Grp& G, double* v, double* red, int* word) {
  double wv[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
    wv[k] = (MAXMASK >> k) & 1u ? wg_max<NT>(v[k], red) : wg_sum<NT>(v[k], red);
  if (G.g == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wv[k];
    return true;
  }
  double* P = G.part + (size_t)G.parity * G.g * kPartStride;
  G.parity ^= 1;
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) P[G.w * kPartStride + k] = wv[k];
  if (!grp_barrier(G, word)) return false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double a = P[k];
    for (int q = 1; q < G.g; ++q) {
      const double b = P[q * kPartStride + k];
      a = (MAXMASK >> k) & 1u ? nan_max(a, b) : a + b;
    }
    v[k] = a;
  }
  return true;
}

// f(position, cell) for every row this workgroup owns
template <int NT, typename F>
__device__ __forceinline__ void for_rows(const Topo& t, F f) {
  for (int l = 0; l < t.nlev; ++l) {
    const int p1 = ilu::lvl_end(t, l);
    for (int pos = ilu::lvl_begin(t, l) + (int)threadIdx.x; pos < p1; pos += NT)
      f(pos, t.perm[pos]);
  }
}

// Right-preconditioned BiCGStab for J d = b over the member's workgroups
// (the steps of wg_bicgstab, each on the workgroup's rows).
template <typename T, int NT>
__device__ int mw_bicgstab(const EnsMember& M, const Topo& tp, IluView<T> iv, Grp& G,
                           const double* b, double* x, double rtol, int maxit, double* red,
                           int* word, T* swin, int* its_out) {
  double bb = 0.0;
  for_rows<NT>(tp, [&](int, int i) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * i + c;
      const double bv = b[k];
      x[k] = 0.0;
      M.r[k] = bv;
      M.rh[k] = bv;
      M.p[k] = 0.0;
      M.v[k] = 0.0;
      bb += bv * bv;
    }
  });
  if (!grp_reduce<NT, 1>(G, &bb, red, word)) return OPM_EHIP;
  *its_out = 0;
  if (bb == 0.0) return OPM_OK;
  const double tol = rtol * sqrt(bb);
  double rho0 = 1.0, alpha = 1.0, omega = 1.0;
  double rho = bb;
  for (int it = 1; it <= maxit; ++it) {
    *its_out = it;
    if (fabs(rho) < 1e-300) return OPM_EBREAKDOWN;
    const double beta = it == 1 ? 0.0 : (rho / rho0) * (alpha / omega);
    for_rows<NT>(tp, [&](int, int i) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int k = 3 * i + c;
        M.p[k] = M.r[k] + beta * (M.p[k] - omega * M.v[k]);
      }
    });
    __syncthreads();
    ilu::apply_levels_wg<T, NT>(tp, iv, M.p, M.ph, swin);
    if (!grp_barrier(G, word)) return OPM_EHIP;   // the neighbours' ph
    double rv = 0.0;
    for_rows<NT>(tp, [&](int, int i) {
      double y3[3];
      ilu::spmv_row(M.pb.row_ptr, M.pb.col_idx, M.J, M.ph, i, y3);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        M.v[3 * i + c] = y3[c];
        rv += M.rh[3 * i + c] * y3[c];
      }
    });
    if (!grp_reduce<NT, 1>(G, &rv, red, word)) return OPM_EHIP;
    if (rv == 0.0) return OPM_EBREAKDOWN;
    alpha = rho / rv;
    double ss = 0.0;
    for_rows<NT>(tp, [&](int, int i) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int k = 3 * i + c;
        const double sv = M.r[k] - alpha * M.v[k];
        M.s[k] = sv;
        ss += sv * sv;
      }
    });
    if (!grp_reduce<NT, 1>(G, &ss, red, word)) return OPM_EHIP;
    if (sqrt(ss) <= tol) {
      for_rows<NT>(tp, [&](int, int i) {
#pragma unroll
        for (int c = 0; c < 3; ++c) x[3 * i + c] += alpha * M.ph[3 * i + c];
      });
      __syncthreads();
      return OPM_OK;
    }
    ilu::apply_levels_wg<T, NT>(tp, iv, M.s, M.sh, swin);
    if (!grp_barrier(G, word)) return OPM_EHIP;   // the neighbours' sh
    double tv[2] = {0.0, 0.0};
    for_rows<NT>(tp, [&](int, int i) {
      double y3[3];
      ilu::spmv_row(M.pb.row_ptr, M.pb.col_idx, M.J, M.sh, i, y3);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        M.t[3 * i + c] = y3[c];
        tv[0] += y3[c] * M.s[3 * i + c];
        tv[1] += y3[c] * y3[c];
      }
    });
    if (!grp_reduce<NT, 2>(G, tv, red, word)) return OPM_EHIP;
    if (tv[1] == 0.0) return OPM_EBREAKDOWN;
    omega = tv[0] / tv[1];
    double rv2[2] = {0.0, 0.0};
    for_rows<NT>(tp, [&](int, int i) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int k = 3 * i + c;
        x[k] += alpha * M.ph[k] + omega * M.sh[k];
        const double rk = M.s[k] - omega * M.t[k];
        M.r[k] = rk;
        rv2[0] += rk * rk;
        rv2[1] += M.rh[k] * rk;
      }
    });
    if (!grp_reduce<NT, 2>(G, rv2, red, word)) return OPM_EHIP;
    if (sqrt(rv2[0]) <= tol) return OPM_OK;
    if (omega == 0.0) return OPM_EBREAKDOWN;
    rho0 = rho;
    rho = rv2[1];
  }
  return OPM_ENOTCONV;
}

// The Newton iteration of wg_newton over the member's workgroups.
template <typename T, int NT, bool FACWIN>
__device__ int mw_newton(const EnsMember& M, const Topo& tp, IluView<T> iv, Grp& G, double h,
                         const opm_newton_opts& o, double* red, int* word, T* swin, double* fwin,
                         int* flag, opm_ensemble_report& rep) {
  const int n = M.pb.n_cells;
  for_rows<NT>(tp, [&](int, int i) {
    FaceProps P;
    CellAcc A;
    asmdev::properties<false>(M.pb.fluid, M.y_save[3 * i], M.y_save[3 * i + 1],
                              M.y_save[3 * i + 2], 0, P, &A);
#pragma unroll
    for (int c = 0; c < 3; ++c) M.acc0[3 * i + c] = A.A[c].v;
  });
  // the neighbours' state (restored or copied by their workgroups)
  if (!grp_barrier(G, word)) return OPM_EHIP;
  AsmArgs a;
  a.n = n;
  a.y = M.y;
  a.acc0 = M.acc0;
  a.dt = h;
  a.trans = M.pb.trans;
  a.pv = M.pb.pore_vol;
  a.depth = M.pb.depth;
  a.row_ptr = M.pb.row_ptr;
  a.col_idx = M.pb.col_idx;
  a.blk_face = M.pb.blk_face;
  a.cell_conn_ptr = M.pb.cell_conn_ptr;
  a.cell_conn = M.pb.cell_conn;
  a.conn_kind = M.pb.conn_kind;
  a.conn_phase = M.pb.conn_phase;
  a.conn_wi = M.pb.conn_wi;
  a.conn_rate = M.pb.conn_rate;
  a.conn_bhp = M.pb.conn_bhp;
  a.fluid = M.pb.fluid;
  a.meaning = nullptr;
  a.n_wells = 0;
  a.conn_well = nullptr;
  a.well_state = nullptr;
  a.Cw = nullptr;
  a.R = M.R;
  a.J = M.J;
  a.partials = nullptr;
  for (int it = 0;; ++it) {
    // max CNV (3, NaN-propagating) and the mass-balance sums (7)
    double nv[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for_rows<NT>(tp, [&](int, int i) {
      double part[kNormStride];
      asmdev::assemble_row<false>(a, i, h, part);
#pragma unroll
      for (int c = 0; c < 3; ++c) nv[c] = nan_max(nv[c], part[c]);
#pragma unroll
      for (int k = 0; k < 7; ++k) nv[3 + k] += part[3 + k];
    });
    if (!grp_reduce<NT, 10, 7u>(G, nv, red, word)) return OPM_EHIP;
    double cm = 0.0, mm = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double mb = h * fabs(nv[3 + c]) / ((nv[6 + c] / n) * nv[9]);
      cm = nan_max(cm, nv[c]);
      mm = nan_max(mm, mb);
      rep.cnv[c] = nv[c];
      rep.mb[c] = mb;
    }
    if (!isfinite(cm) || !isfinite(mm)) return OPM_ENONFINITE;
    if (cm <= o.tol_cnv && mm <= o.tol_mb) return OPM_OK;
    if (it >= o.max_newton) return OPM_ENOTCONV;
    // block ILU(0) of the workgroup's subdomains
    for_rows<NT>(tp, [&](int pos, int) { ilu::pack_row<T>(tp, M.J, iv, pos); });
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    ilu::factor_levels_wg<T, FACWIN, NT, false>(tp, M.J, iv, flag, fwin);
    __syncthreads();
    double sing = *flag != 0 ? 1.0 : 0.0;
    if (!grp_reduce<NT, 1, 1u>(G, &sing, red, word)) return OPM_EHIP;
    if (sing != 0.0) return OPM_ESINGULAR;
    int lits = 0;
    const int st = mw_bicgstab<T, NT>(M, tp, iv, G, M.R, M.d, o.lin_rtol, o.lin_maxit, red, word,
                                      swin, &lits);
    rep.lin_its += lits;
    if (st != OPM_OK) return st;
    double bad = 0.0;
    for_rows<NT>(tp, [&](int, int i) {
      const double p = M.y[3 * i];
      double dp = -M.d[3 * i];
      const double lim = o.dp_max_rel * fabs(p);
      if (dp > lim) dp = lim;
      if (dp < -lim) dp = -lim;
      double dsw = -M.d[3 * i + 1], dsg = -M.d[3 * i + 2];
      const double mx = fmax(fabs(dsw), fabs(dsg));
      if (mx > o.ds_max) {
        const double sc = o.ds_max / mx;
        dsw *= sc;
        dsg *= sc;
      }
      const double y0 = p + dp, y1 = M.y[3 * i + 1] + dsw, y2 = M.y[3 * i + 2] + dsg;
      M.y[3 * i] = y0;
      M.y[3 * i + 1] = y1;
      M.y[3 * i + 2] = y2;
      if (!isfinite(y0) || !isfinite(y1) || !isfinite(y2)) bad = 1.0;
    });
    // (also the barrier after which the next assembly reads the neighbours' y)
    if (!grp_reduce<NT, 1, 1u>(G, &bad, red, word)) return OPM_EHIP;
    rep.newton_its += 1;
    rep.cell_newton_its += (double)n;
    if (bad != 0.0) return OPM_ENONFINITE;
  }
}

template <int NT>
__device__ __forceinline__ void rows_copy(const Topo& t, double* dst, const double* src) {
  for_rows<NT>(t, [&](int, int i) {
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[3 * i + c] = src[3 * i + c];
  });
  __syncthreads();
}

template <typename T, int NT, bool FACWIN>
__global__ __launch_bounds__(NT) void k_ensemble_mw(const EnsMember* tab, const EnsHeader* hdr,
                                                     const EnsWg* wgs, EnsSync* sync,
                                                     double* part, unsigned spin, int n_steps,
                                                     double dt_report, opm_newton_opts o,
                                                     size_t red_bytes, size_t sweep_bytes,
                                                     opm_ensemble_report* reps) {
  extern __shared__ double smem[];
  __shared__ int flag, word;
  double* red = smem;
  T* swin = reinterpret_cast<T*>(reinterpret_cast<char*>(smem) + red_bytes);
  double* fwin = reinterpret_cast<double*>(reinterpret_cast<char*>(smem) + red_bytes + sweep_bytes);
  if ((int)blockIdx.x >= hdr->n_wgs) return;   // a grid larger than the configured table
  const EnsWg W = wgs[blockIdx.x];
  const EnsMember M = tab[W.m];
  Topo tp = ilu::topo_of(&M.pb);
  if (M.pb.n_sub > 0 && W.g > 1) {   // this workgroup's subdomains of every local level
    tp.level_ptr = M.pb.sub_level_ptr;
    tp.lstride = M.pb.n_sub + 1;
    tp.s0 = W.s0;
    tp.s1 = W.s1;
  }
  tp.max_level = W.width;
  Grp G{W.w, W.g, part + (size_t)2 * kPartStride * (blockIdx.x - W.w), sync + W.m, spin, 0};
  IluView<T> iv = ilu::view<T>(&M.pb, M.ilu);
  opm_ensemble_report rep = {};
  int status = OPM_OK;
  for (int step = 0; step < n_steps && status == OPM_OK; ++step) {
    rows_copy<NT>(tp, M.y_save, M.y);
    double t = 0.0, dt_try = dt_report;
    int cuts = 0;
    while (dt_report - t > 1e-9 * dt_report) {
      const double h = fmin(dt_try, dt_report - t);
      const int st = mw_newton<T, NT, FACWIN>(M, tp, iv, G, h, o, red, &word, swin, fwin, &flag,
                                              rep);
      __syncthreads();
      if (st == OPM_EHIP) {   // the member's workgroups lost each other
        status = st;
        break;
      }
      if (st == OPM_OK) {
        t += h;
        rep.substeps += 1;
        rows_copy<NT>(tp, M.y_save, M.y);
      } else {
        rows_copy<NT>(tp, M.y, M.y_save);
        dt_try = 0.5 * h;
        rep.cuts += 1;
        if (++cuts > o.max_cuts) {
          status = st;
          break;
        }
      }
    }
    if (status == OPM_OK) rep.steps_done = step + 1;
  }
  rep.status = status;
  if (threadIdx.x == 0 && W.w == 0) reps[W.m] = rep;
}

// Before a launch of k_ensemble_mw: counters at zero, no failure.
__global__ __launch_bounds__(64) void k_ens_sync_reset(EnsSync* sync, int n_members) {
  for (int m = blockIdx.x * 64 + threadIdx.x; m < n_members; m += gridDim.x * 64) {
    sync[m].count = 0;
    sync[m].fail = 0;
  }
}

// Raise the dynamic-LDS limit of every kernel instance (done at prepare
// time, outside any graph capture).
template <typename T>
int allow_ensemble_lds() {
  const void* k[4] = {reinterpret_cast<const void*>(k_ensemble<T, 256, true>),
                      reinterpret_cast<const void*>(k_ensemble<T, 256, false>),
                      reinterpret_cast<const void*>(k_ensemble<T, 128, true>),
                      reinterpret_cast<const void*>(k_ensemble<T, 128, false>)};
  for (const void* f : k)
    OPM_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kEnsLds));
  const void* kw[4] = {reinterpret_cast<const void*>(k_ensemble_mw<T, 256, true>),
                       reinterpret_cast<const void*>(k_ensemble_mw<T, 256, false>),
                       reinterpret_cast<const void*>(k_ensemble_mw<T, 128, true>),
                       reinterpret_cast<const void*>(k_ensemble_mw<T, 128, false>)};
  for (const void* f : kw)
    OPM_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kEnsLds));
  return OPM_OK;
}

}  // namespace
// Polls of a member barrier before it gives up (OPM_OPT_ENSEMBLE_SPIN).
int g_ens_spin = 1 << 22;
namespace {

// Every workgroup of a launch of k_ensemble_mw must be resident at once (a
// member's workgroups wait for each other).
template <typename K>
int check_resident(K kernel, int threads, size_t lds, int wgs) {
  int dev = 0, per_cu = 0;
  OPM_TRY_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  OPM_TRY_HIP(hipGetDeviceProperties(&prop, dev));
  OPM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds));
  return (long)per_cu * prop.multiProcessorCount >= wgs ? OPM_OK : OPM_EINVAL;
}

template <typename T>
int launch_ensemble(const EnsMember* tab, const EnsHeader* hdr, const EnsWg* wgs, EnsSync* sync,
                    double* part, int n_members, int max_level, const opm_ensemble_config& cfg,
                    double dt_report, int n_steps, const opm_newton_opts* o,
                    opm_ensemble_report* reps, hipStream_t s) {
  const LdsPlan lp = lds_plan(sizeof(T), cfg.threads, (size_t)cfg.sweep_bytes, max_level,
                              cfg.fac_window != 0);
  if (lp.total > kEnsLds) return OPM_EINVAL;
  const size_t red = al256(lp.red);
  if (cfg.wgs > 0) {
#define OPM_ENS_MW(NT, FW)                                                                       \
  do {                                                                                           \
    OPM_TRY(check_resident(k_ensemble_mw<T, NT, FW>, NT, lp.total, cfg.wgs));                    \
    hipLaunchKernelGGL(k_ens_sync_reset, dim3(1), dim3(64), 0, s, sync, n_members);              \
    hipLaunchKernelGGL((k_ensemble_mw<T, NT, FW>), dim3(cfg.wgs), dim3(NT), lp.total, s, tab,    \
                       hdr, wgs, sync, part, (unsigned)g_ens_spin, n_steps, dt_report, *o, red, \
                       lp.sweep, reps);                                                          \
  } while (0)
    if (cfg.threads == 256) {
      if (cfg.fac_window) OPM_ENS_MW(256, true);
      else OPM_ENS_MW(256, false);
    } else {
      if (cfg.fac_window) OPM_ENS_MW(128, true);
      else OPM_ENS_MW(128, false);
    }
#undef OPM_ENS_MW
    OPM_TRY_HIP(hipGetLastError());
    return OPM_OK;
  }
  const dim3 grid(n_members);
#define OPM_ENS_LAUNCH(NT, FW)                                                                   \
  hipLaunchKernelGGL((k_ensemble<T, NT, FW>), grid, dim3(NT), lp.total, s, tab, n_steps,        \
                     dt_report, *o, red, lp.sweep, reps)
  if (cfg.threads == 256) {
    if (cfg.fac_window) OPM_ENS_LAUNCH(256, true);
    else OPM_ENS_LAUNCH(256, false);
  } else {
    if (cfg.fac_window) OPM_ENS_LAUNCH(128, true);
    else OPM_ENS_LAUNCH(128, false);
  }
#undef OPM_ENS_LAUNCH
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}


bool valid_config(const opm_ensemble_config& c, int max_level) {
  return (c.threads == 128 || c.threads == 256) && (c.fac_window == 0 || c.fac_window == 1) &&
         (c.ring == 0 || c.ring == 1) && (!c.fac_window || max_level <= kMaxFacWindowLevel) &&
         c.wgs >= 0 && c.wgs <= kMaxEnsWgs && (c.wgs == 0 || (c.ring == 0 && c.fac_window == 0));
}

// Per-member sweep choice and the LDS the launch needs; false if it does not fit.
bool plan_members(const opm_problem* members, int n, int precision, opm_ensemble_config& c,
                  std::vector<int32_t>* ring, int* max_level_out) {
  const size_t ts = precision == OPM_PREC_MIXED ? sizeof(float) : sizeof(double);
  int max_level = 0;
  for (int m = 0; m < n; ++m) max_level = std::max(max_level, (int)members[m].max_level);
  if (!valid_config(c, max_level)) return false;
  const size_t fixed = lds_plan(ts, c.threads, 0, max_level, c.fac_window != 0).total;
  size_t sweep = 0;
  for (int m = 0; m < n; ++m) {
    size_t b = window_bytes(ts, members[m].max_level);
    int use_ring = 0;
    if (c.ring && members[m].sweep_span > 0 && al256(ring_bytes(ts, members[m])) + fixed <= kEnsLds) {
      b = ring_bytes(ts, members[m]);
      use_ring = 1;
    }
    if (ring) (*ring)[m] = use_ring;
    sweep = std::max(sweep, b);
  }
  c.sweep_bytes = (int32_t)al256(sweep);
  if (lds_plan(ts, c.threads, sweep, max_level, c.fac_window != 0).total > kEnsLds) return false;
  *max_level_out = max_level;
  return true;
}

// Workspace: header, member table, the autotuner's trial reports, the
// workgroup table, the members' barrier words, the reduction partials of
// k_ensemble_mw, members.
EnsMember* table_of(void* work) {
  return reinterpret_cast<EnsMember*>((char*)work + al256(sizeof(EnsHeader)));
}
size_t reports_offset(int n_members) {
  return al256(sizeof(EnsHeader)) + al256(sizeof(EnsMember) * (size_t)n_members);
}
opm_ensemble_report* trial_reports_of(void* work, int n_members) {
  return reinterpret_cast<opm_ensemble_report*>((char*)work + reports_offset(n_members));
}
size_t wgs_offset(int n_members) {
  return reports_offset(n_members) + al256(sizeof(opm_ensemble_report) * (size_t)n_members);
}
EnsWg* wgs_of(void* work, int n_members) {
  return reinterpret_cast<EnsWg*>((char*)work + wgs_offset(n_members));
}
size_t sync_offset(int n_members) {
  return wgs_offset(n_members) + al256(sizeof(EnsWg) * (size_t)kMaxEnsWgs);
}
EnsSync* sync_of(void* work, int n_members) {
  return reinterpret_cast<EnsSync*>((char*)work + sync_offset(n_members));
}
size_t part_offset(int n_members) {
  return sync_offset(n_members) + al256(sizeof(EnsSync) * (size_t)n_members);
}
double* part_of(void* work, int n_members) {
  return reinterpret_cast<double*>((char*)work + part_offset(n_members));
}
size_t members_offset(int n_members) {
  return part_offset(n_members) + al256(sizeof(double) * 2 * kPartStride * (size_t)kMaxEnsWgs);
}

// Workgroups per member for a launch of `budget` workgroups: in proportion
// to the rows, at least one, at most one per subdomain (one for a member
// without subdomains), each member's subdomains split into contiguous ranges
// of about equal rows.  Writes the table (members in order, a member's
// workgroups consecutive) and returns the number of workgroups.
int build_wg_table(const opm_problem* members, int n, int budget, std::vector<EnsWg>& out) {
  out.clear();
  if (budget < n) return OPM_EINVAL;
  double total = 0.0;
  for (int m = 0; m < n; ++m) total += members[m].n_cells;
  std::vector<int> g(n), cap(n);
  int used = 0;
  for (int m = 0; m < n; ++m) {
    cap[m] = members[m].n_sub > 1 ? members[m].n_sub : 1;
    g[m] = std::max(1, std::min(cap[m], (int)std::floor(budget * members[m].n_cells / total)));
    used += g[m];
  }
  // the floor and the minimum of one can overshoot: take back from the largest
  while (used > budget) {
    int mx = 0;
    for (int m = 1; m < n; ++m)
      if (g[m] > g[mx]) mx = m;
    if (g[mx] <= 1) return OPM_EINVAL;
    --g[mx];
    --used;
  }
  // what is left goes, one at a time, to the member with the most rows per
  // workgroup that can still take one
  while (used < budget) {
    int best = -1;
    for (int m = 0; m < n; ++m)
      if (g[m] < cap[m] &&
          (best < 0 || (double)members[m].n_cells / g[m] > (double)members[best].n_cells / g[best]))
        best = m;
    if (best < 0) break;
    ++g[best];
    ++used;
  }
  for (int m = 0; m < n; ++m) {
    const opm_problem& pb = members[m];
    if (g[m] == 1) {
      out.push_back(EnsWg{m, 0, 1, 0, 1, pb.max_level, {0, 0}});
      continue;
    }
    // rows per subdomain from the device copy of sub_level_ptr
    const size_t ns1 = (size_t)pb.n_sub + 1;
    std::vector<int32_t> slp((size_t)pb.n_levels * ns1);
    OPM_TRY_HIP(hipMemcpy(slp.data(), pb.sub_level_ptr, sizeof(int32_t) * slp.size(),
                          hipMemcpyDeviceToHost));
    std::vector<long> rows(pb.n_sub, 0);
    for (int l = 0; l < pb.n_levels; ++l)
      for (int sd = 0; sd < pb.n_sub; ++sd) rows[sd] += slp[l * ns1 + sd + 1] - slp[l * ns1 + sd];
    int s0 = 0;
    long acc = 0;
    for (int w = 0; w < g[m]; ++w) {
      // close range w once it reaches its share of the rows, leaving at
      // least one subdomain for each later workgroup
      const long target = (long)std::llround((double)pb.n_cells * (w + 1) / g[m]);
      int s1 = s0 + 1;
      acc += rows[s0];
      while (s1 < pb.n_sub - (g[m] - 1 - w) && acc + rows[s1] / 2 < target) acc += rows[s1++];
      if (w == g[m] - 1) {
        while (s1 < pb.n_sub) acc += rows[s1++];
      }
      int width = 0;
      for (int l = 0; l < pb.n_levels; ++l)
        width = std::max(width, slp[l * ns1 + s1] - slp[l * ns1 + s0]);
      out.push_back(EnsWg{m, w, g[m], s0, s1, width, {0, 0}});
      s0 = s1;
    }
  }
  return (int)out.size() <= kMaxEnsWgs ? OPM_OK : OPM_EINVAL;
}

}  // namespace
}  // namespace opm

using namespace opm;

extern "C" {

size_t opm_ensemble_bytes(const opm_problem* members, int32_t n_members, int precision) {
  if (!members || n_members <= 0 || (precision != OPM_PREC_FP64 && precision != OPM_PREC_MIXED))
    return 0;
  size_t b = members_offset(n_members);
  for (int m = 0; m < n_members; ++m) b += member_bytes(members[m], precision);
  return b;
}

int opm_ensemble_default_config(const opm_problem* members, int32_t n_members, int precision,
                                opm_ensemble_config* cfg) {
  if (!members || n_members <= 0 || !cfg ||
      (precision != OPM_PREC_FP64 && precision != OPM_PREC_MIXED))
    return OPM_EINVAL;
  int max_level = 0;
  for (int m = 0; m < n_members; ++m) max_level = std::max(max_level, (int)members[m].max_level);
  opm_ensemble_config c{256, max_level <= kMaxFacWindowLevel ? 1 : 0, 0, 0, 0};
  if (!plan_members(members, n_members, precision, c, nullptr, &max_level)) return OPM_EINVAL;
  *cfg = c;
  return OPM_OK;
}

int opm_ensemble_prepare(const opm_problem* members, double* const* y, int32_t n_members,
                         int precision, void* work, size_t work_bytes) {
  if (!members || !y || !work || n_members <= 0 ||
      work_bytes < opm_ensemble_bytes(members, n_members, precision))
    return OPM_EINVAL;
  int max_level = 0;
  for (int m = 0; m < n_members; ++m) {
    const opm_problem& pb = members[m];
    if (pb.n_cells <= 0 || pb.nnzb != pb.n_cells + 2 * pb.n_faces || pb.n_levels <= 0 || !y[m] ||
        pb.fluid.live != 0 || pb.n_wells != 0)
      return OPM_EINVAL;
    max_level = std::max(max_level, (int)pb.max_level);
  }
  std::vector<EnsMember> tab(n_members);
  char* base = (char*)work;
  char* cur = base + members_offset(n_members);
  for (int m = 0; m < n_members; ++m) {
    const opm_problem& pb = members[m];
    const size_t N = 3 * (size_t)pb.n_cells;
    EnsMember& e = tab[m];
    e.pb = pb;
    e.pb.level_ptr_h = nullptr;
    e.y = y[m];
    double** vecs[13] = {&e.y_save, &e.acc0, &e.R, &e.d, &e.r, &e.rh, &e.p,
                         &e.v,      &e.ph,   &e.s, &e.sh, &e.t, &e.backup};
    for (int k = 0; k < 13; ++k) {
      *vecs[k] = (double*)cur;
      cur += al256(sizeof(double) * N);
    }
    e.J = (double*)cur;
    cur += al256(sizeof(double) * 9 * (size_t)pb.nnzb);
    e.ilu = cur;
    cur += al256(precision == OPM_PREC_MIXED ? ilu::view_bytes<float>(pb.n_cells)
                                             : ilu::view_bytes<double>(pb.n_cells));
    e.ring = 0;
    e.ring_mask = (uint32_t)ilu::ring_rows(pb.sweep_span, pb.max_level) - 1u;
  }
  OPM_TRY(precision == OPM_PREC_MIXED ? allow_ensemble_lds<float>() : allow_ensemble_lds<double>());
  EnsHeader hdr{n_members, precision, max_level, 0};
  OPM_TRY_HIP(hipMemcpy(base, &hdr, sizeof(hdr), hipMemcpyHostToDevice));
  OPM_TRY_HIP(hipMemcpy(table_of(work), tab.data(), sizeof(EnsMember) * (size_t)n_members,
                        hipMemcpyHostToDevice));
  return OPM_OK;
}

int opm_ensemble_configure(const opm_problem* members, int32_t n_members, int precision,
                           void* work, opm_ensemble_config* cfg) {
  if (!members || n_members <= 0 || !work || !cfg ||
      (precision != OPM_PREC_FP64 && precision != OPM_PREC_MIXED))
    return OPM_EINVAL;
  std::vector<int32_t> ring(n_members, 0);
  int max_level = 0;
  opm_ensemble_config c = *cfg;
  std::vector<EnsWg> wt;
  if (c.wgs > 0) {
    // the LDS window holds the widest level range of one workgroup
    for (int m = 0; m < n_members; ++m) max_level = std::max(max_level, (int)members[m].max_level);
    if (!valid_config(c, max_level)) return OPM_EINVAL;
    OPM_TRY(build_wg_table(members, n_members, c.wgs, wt));
    int width = 0;
    for (const EnsWg& e : wt) width = std::max(width, e.width);
    const size_t ts = precision == OPM_PREC_MIXED ? sizeof(float) : sizeof(double);
    c.sweep_bytes = (int32_t)al256(window_bytes(ts, width));
    if (lds_plan(ts, c.threads, (size_t)c.sweep_bytes, width, false).total > kEnsLds)
      return OPM_EINVAL;
  } else if (!plan_members(members, n_members, precision, c, &ring, &max_level)) {
    return OPM_EINVAL;
  }
  std::vector<EnsMember> tab(n_members);
  OPM_TRY_HIP(hipMemcpy(tab.data(), table_of(work), sizeof(EnsMember) * (size_t)n_members,
                        hipMemcpyDeviceToHost));
  for (int m = 0; m < n_members; ++m) tab[m].ring = c.wgs > 0 ? 0 : ring[m];
  OPM_TRY_HIP(hipMemcpy(table_of(work), tab.data(), sizeof(EnsMember) * (size_t)n_members,
                        hipMemcpyHostToDevice));
  int32_t n_wgs = 0;
  if (c.wgs > 0) {
    OPM_TRY_HIP(hipMemcpy(wgs_of(work, n_members), wt.data(), sizeof(EnsWg) * wt.size(),
                          hipMemcpyHostToDevice));
    n_wgs = (int32_t)wt.size();
    c.wgs = n_wgs;
  }
  OPM_TRY_HIP(hipMemcpy(&reinterpret_cast<EnsHeader*>(work)->n_wgs, &n_wgs, sizeof n_wgs,
                        hipMemcpyHostToDevice));
  *cfg = c;
  return OPM_OK;
}

int opm_ensemble_launch_config(const void* work, int32_t n_members, int precision,
                               int32_t max_level, const opm_ensemble_config* cfg,
                               double dt_report, int32_t n_steps, const opm_newton_opts* opts,
                               opm_ensemble_report* reports, void* stream) {
  if (!work || n_members <= 0 || !opts || !reports || n_steps < 0 || !(dt_report > 0.0) ||
      max_level <= 0 || opts->max_newton < 0 || opts->lin_maxit < 0 || opts->max_cuts < 0 ||
      opts->krylov != OPM_KRYLOV_BICGSTAB || opts->precond != OPM_PRECOND_ILU0 || !cfg ||
      !valid_config(*cfg, max_level) ||
      cfg->sweep_bytes <= 0)
    return OPM_EINVAL;
  void* w = const_cast<void*>(work);
  const EnsMember* tab = table_of(w);
  const EnsHeader* hdr = reinterpret_cast<const EnsHeader*>(w);
  EnsWg* wgs = wgs_of(w, n_members);
  EnsSync* sync = sync_of(w, n_members);
  double* part = part_of(w, n_members);
  hipStream_t s = as_stream(stream);
  if (precision == OPM_PREC_MIXED)
    return launch_ensemble<float>(tab, hdr, wgs, sync, part, n_members, max_level, *cfg,
                                  dt_report, n_steps, opts, reports, s);
  if (precision == OPM_PREC_FP64)
    return launch_ensemble<double>(tab, hdr, wgs, sync, part, n_members, max_level, *cfg,
                                   dt_report, n_steps, opts, reports, s);
  return OPM_EINVAL;
}

int opm_ensemble_launch(const void* work, int32_t n_members, int precision, int32_t max_level,
                        double dt_report, int32_t n_steps, const opm_newton_opts* opts,
                        opm_ensemble_report* reports, void* stream) {
  if (precision != OPM_PREC_FP64 && precision != OPM_PREC_MIXED) return OPM_EINVAL;
  // default shape: 256 threads, factor window when it fits, window sweeps for
  // every member (a member flagged for the ring by opm_ensemble_configure
  // falls back to the window: the kernel checks the ring against this size)
  const size_t ts = precision == OPM_PREC_MIXED ? sizeof(float) : sizeof(double);
  opm_ensemble_config c{256, max_level > 0 && max_level <= kMaxFacWindowLevel ? 1 : 0, 0,
                        (int32_t)al256(window_bytes(ts, max_level)), 0};
  return opm_ensemble_launch_config(work, n_members, precision, max_level, &c, dt_report,
                                    n_steps, opts, reports, stream);
}

int opm_ensemble_autotune(const opm_problem* members, int32_t n_members, int precision,
                          void* work, double dt_report, const opm_newton_opts* opts,
                          opm_ensemble_config* best, double* seconds, int32_t* n_tried,
                          void* stream) {
  if (!members || n_members <= 0 || !work || !opts || !best || !(dt_report > 0.0) ||
      opts->krylov != OPM_KRYLOV_BICGSTAB || opts->precond != OPM_PRECOND_ILU0 ||
      (precision != OPM_PREC_FP64 && precision != OPM_PREC_MIXED))
    return OPM_EINVAL;
  hipStream_t s = as_stream(stream);
  int max_level = 0;
  for (int m = 0; m < n_members; ++m) max_level = std::max(max_level, (int)members[m].max_level);
  std::vector<EnsMember> tab(n_members);
  OPM_TRY_HIP(hipMemcpy(tab.data(), table_of(work), sizeof(EnsMember) * (size_t)n_members,
                        hipMemcpyDeviceToHost));
  // the backup slot of each member keeps its state between trials
  auto copy_states = [&](bool to_backup) -> int {
    for (int m = 0; m < n_members; ++m) {
      const size_t bytes = sizeof(double) * 3 * (size_t)members[m].n_cells;
      OPM_TRY_HIP(hipMemcpyAsync(to_backup ? tab[m].backup : tab[m].y,
                                 to_backup ? tab[m].y : tab[m].backup, bytes,
                                 hipMemcpyDeviceToDevice, s));
    }
    return OPM_OK;
  };
  OPM_TRY(copy_states(true));
  opm_ensemble_report* reps = trial_reports_of(work, n_members);
  hipEvent_t e0, e1;
  OPM_TRY_HIP(hipEventCreate(&e0));
  OPM_TRY_HIP(hipEventCreate(&e1));
  int tried = 0, passed = 0;
  std::vector<opm_ensemble_report> trial(n_members);
  double best_t = INFINITY;
  opm_ensemble_config best_c{};
  int status = OPM_OK;
  // several workgroups per member: one launch of as many workgroups as the
  // device has compute units, when some member has subdomains to share out
  int split_wgs = 0;
  for (int m = 0; m < n_members; ++m)
    if (members[m].n_sub > 1) {
      int dev = 0;
      hipDeviceProp_t prop;
      if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        split_wgs = std::min(kMaxEnsWgs, prop.multiProcessorCount);
      break;
    }
  std::vector<int> wgs_choices{0};
  if (split_wgs >= n_members) wgs_choices.push_back(split_wgs);
  for (int wgs : wgs_choices)
  for (int threads : {256, 128})
    for (int ring : {0, 1})
      for (int facw : {1, 0}) {
        opm_ensemble_config c{threads, facw, ring, 0, wgs};
        if (!valid_config(c, max_level)) continue;
        if (opm_ensemble_configure(members, n_members, precision, work, &c) != OPM_OK) continue;
        status = copy_states(false);
        if (status != OPM_OK) break;
        (void)hipEventRecord(e0, s);
        status = opm_ensemble_launch_config(work, n_members, precision, max_level, &c, dt_report,
                                            1, opts, reps, s);
        (void)hipEventRecord(e1, s);
        if (status != OPM_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
          status = OPM_EHIP;
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (seconds) seconds[tried] = ms * 1e-3;
        ++tried;
        // a trial in which a member failed (or ran out of cuts) stopped
        // early: its time says nothing about the shape, so it cannot win
        if (hipMemcpy(trial.data(), reps, sizeof(opm_ensemble_report) * (size_t)n_members,
                      hipMemcpyDeviceToHost) != hipSuccess) {
          status = OPM_EHIP;
          break;
        }
        bool complete = true;
        for (const opm_ensemble_report& r : trial)
          complete = complete && r.status == OPM_OK && r.steps_done >= 1;
        if (complete) ++passed;
        if (complete && ms * 1e-3 < best_t) {
          best_t = ms * 1e-3;
          best_c = c;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == OPM_OK) status = copy_states(false);
  if (status == OPM_OK && hipStreamSynchronize(s) != hipSuccess) status = OPM_EHIP;
  if (status != OPM_OK) return status;
  if (tried == 0) return OPM_EINVAL;
  if (n_tried) *n_tried = tried;
  if (passed == 0) return OPM_ENOTCONV;
  OPM_TRY(opm_ensemble_configure(members, n_members, precision, work, &best_c));
  *best = best_c;
  if (n_tried) *n_tried = tried;
  return OPM_OK;
}

}  // extern "C"
