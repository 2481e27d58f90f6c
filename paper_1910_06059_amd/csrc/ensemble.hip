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
  return OPM_OK;
}

template <typename T>
int launch_ensemble(const EnsMember* tab, int n_members, int max_level,
                    const opm_ensemble_config& cfg, double dt_report, int n_steps,
                    const opm_newton_opts* o, opm_ensemble_report* reps, hipStream_t s) {
  const LdsPlan lp = lds_plan(sizeof(T), cfg.threads, (size_t)cfg.sweep_bytes, max_level,
                              cfg.fac_window != 0);
  if (lp.total > kEnsLds) return OPM_EINVAL;
  const size_t red = al256(lp.red);
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

struct EnsHeader {
  int32_t n_members, precision, max_level, pad;
};

bool valid_config(const opm_ensemble_config& c, int max_level) {
  return (c.threads == 128 || c.threads == 256) && (c.fac_window == 0 || c.fac_window == 1) &&
         (c.ring == 0 || c.ring == 1) && (!c.fac_window || max_level <= kMaxFacWindowLevel);
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

// Workspace: header, member table, the autotuner's trial reports, members.
EnsMember* table_of(void* work) {
  return reinterpret_cast<EnsMember*>((char*)work + al256(sizeof(EnsHeader)));
}
opm_ensemble_report* trial_reports_of(void* work, int n_members) {
  return reinterpret_cast<opm_ensemble_report*>(
      (char*)work + al256(sizeof(EnsHeader)) + al256(sizeof(EnsMember) * (size_t)n_members));
}
size_t members_offset(int n_members) {
  return al256(sizeof(EnsHeader)) + al256(sizeof(EnsMember) * (size_t)n_members) +
         al256(sizeof(opm_ensemble_report) * (size_t)n_members);
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
  opm_ensemble_config c{256, max_level <= kMaxFacWindowLevel ? 1 : 0, 0, 0};
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
  opm_ensemble_config c;
  OPM_TRY(opm_ensemble_default_config(members, n_members, precision, &c));
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
  if (!plan_members(members, n_members, precision, c, &ring, &max_level)) return OPM_EINVAL;
  std::vector<EnsMember> tab(n_members);
  OPM_TRY_HIP(hipMemcpy(tab.data(), table_of(work), sizeof(EnsMember) * (size_t)n_members,
                        hipMemcpyDeviceToHost));
  for (int m = 0; m < n_members; ++m) tab[m].ring = ring[m];
  OPM_TRY_HIP(hipMemcpy(table_of(work), tab.data(), sizeof(EnsMember) * (size_t)n_members,
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
  const EnsMember* tab = table_of(const_cast<void*>(work));
  hipStream_t s = as_stream(stream);
  if (precision == OPM_PREC_MIXED)
    return launch_ensemble<float>(tab, n_members, max_level, *cfg, dt_report, n_steps, opts,
                                  reports, s);
  if (precision == OPM_PREC_FP64)
    return launch_ensemble<double>(tab, n_members, max_level, *cfg, dt_report, n_steps, opts,
                                   reports, s);
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
                        (int32_t)al256(window_bytes(ts, max_level))};
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
  for (int threads : {256, 128})
    for (int ring : {0, 1})
      for (int facw : {1, 0}) {
        opm_ensemble_config c{threads, facw, ring, 0};
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
