// Newton-Raphson time step and report-step driver (paper sec. 2.3, eq.
// linsystem: J(y_n)(y_{n+1} - y_n) = -R(y_n) from the previous step's state,
// Appleyard-type chop of each update, time-step cutting on failure), and the
// C-ABI entry points of the library.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "cpr_dev.h"
#include "wells_dev.h"

namespace opm {

extern int g_sweep_mode;
extern int g_block_depth;
extern int g_sweep_kernel;
extern int g_krylov_chunk;
extern int g_krylov_graph;
int launch_assemble(const opm_problem* pb, const double* y, const double* acc0, double dt,
                    double* R, double* J, double* norms, hipStream_t s, double* Cw = nullptr);
int launch_assemble_noalloc(const opm_problem* pb, const double* y, const double* acc0, double dt,
                            double* R, double* J, double* norms, hipStream_t s);
int assemble_scratch_setup(int device);
long assemble_noalloc_max_cells();
long assemble_workgroups(const opm_problem* pb, const double* Cw);
long assemble_max_workgroups(const opm_problem* pb);
extern int g_assembly_kernel;
extern int g_plane_sweep;
extern int g_plane_spin;
extern int g_ens_spin;
int launch_accumulation(const opm_problem* pb, const double* y, double* acc0, hipStream_t s);
size_t ilu_bytes(const opm_problem* pb, int precision);
int ilu_factor(const opm_problem* pb, const double* J, void* ilu, int precision, int32_t* status,
               hipStream_t s);
int ilu_apply(const opm_problem* pb, void* ilu, int precision, const double* r, double* x,
              hipStream_t s, const int32_t* skip);
size_t krylov_bytes(const opm_problem* pb);
int spmv(const opm_problem* pb, const double* J, const double* x, double* y, hipStream_t s);
int bicgstab(const opm_problem* pb, const double* J, void* ilu, int precision, const double* b,
             double* x, double rtol, int maxit, void* work, opm_solve_report* rep,
             hipStream_t st, const WellSchur* ws = nullptr, const CprWork* cpr = nullptr);
size_t gmres_bytes(const opm_problem* pb, int restart);
int gmres(const opm_problem* pb, const double* J, void* ilu, int precision, const double* b,
          double* x, double rtol, int maxit, int restart, void* work, opm_solve_report* rep,
          hipStream_t st, const CprWork* cpr = nullptr, const WellSchur* ws = nullptr);

int guess_infer(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                const double* y_nm1, double* y_guess, void* work, hipStream_t s,
                const double** y_extrap = nullptr);

namespace {

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// partials for whichever assembly kernel runs (the option may change
// between sizing and use)
size_t norms_bytes(const opm_problem* pb) {
  return sizeof(double) * (8 + (size_t)kNormStride * assemble_max_workgroups(pb));
}

struct NewtonWork {
  double* acc0;
  double* R;
  double* J;
  double* d;
  double* norms;
  int32_t* flags;   // [0] factor status, [1] non-finite update
  uint8_t* mean_save;   // [n] variable meanings of the last accepted state (live oil)
  WellWork wells;       // standard wells (unset without)
  void* cpr;            // CPR-AMG workspace (problems with a hierarchy)
  void* ilu;
  void* krylov;
};

// The Krylov workspace is last: its size depends on the method.
size_t newton_bytes(const opm_problem* pb, int precision, int krylov = OPM_KRYLOV_BICGSTAB,
                    int restart = 0) {
  const size_t N = 3 * (size_t)pb->n_cells;
  const size_t kb = krylov == OPM_KRYLOV_GMRES ? gmres_bytes(pb, restart) : krylov_bytes(pb);
  return align256(sizeof(double) * N) * 3 + align256(sizeof(double) * 9 * (size_t)pb->nnzb) +
         align256(norms_bytes(pb)) + 256 + align256((size_t)pb->n_cells) +
         align256(wells_bytes(pb)) + align256(cpr_bytes(pb)) + align256(ilu_bytes(pb, precision)) +
         align256(kb);
}

NewtonWork carve(const opm_problem* pb, int precision, void* work) {
  const size_t N = 3 * (size_t)pb->n_cells;
  char* c = (char*)work;
  NewtonWork w;
  w.acc0 = (double*)c;
  c += align256(sizeof(double) * N);
  w.R = (double*)c;
  c += align256(sizeof(double) * N);
  w.d = (double*)c;
  c += align256(sizeof(double) * N);
  w.J = (double*)c;
  c += align256(sizeof(double) * 9 * (size_t)pb->nnzb);
  // the flags end their 256-byte slot, right before the norms: one copy
  // reads both
  w.flags = (int32_t*)(c + 256 - 4 * sizeof(int32_t));
  c += 256;
  w.norms = (double*)c;
  c += align256(norms_bytes(pb));
  w.mean_save = (uint8_t*)c;
  c += align256((size_t)pb->n_cells);
  std::memset(&w.wells, 0, sizeof w.wells);
  if (pb->n_wells > 0) w.wells = wells_carve(pb, c);
  c += align256(wells_bytes(pb));
  w.cpr = c;
  c += align256(cpr_bytes(pb));
  w.ilu = c;
  c += align256(ilu_bytes(pb, precision));
  w.krylov = c;
  return w;
}

__global__ void k_clear_flags(int32_t* flags) {
  if (threadIdx.x < 4) flags[threadIdx.x] = 0;
}

// y <- y - chop(d) where J d = R (so -d is the Newton update): |dp| is
// bounded by dp_max_rel |p|; the saturation part is scaled so that its
// largest component is at most ds_max (the third variable counts only where
// it is s_g: a change of r_go is not chopped).  With live oil (meaning
// non-null) the variable switch follows (eq. primaryVariableMeaning, with a
// threshold against oscillation, sec. 2.3): free gas below -eps -> x =
// r_go = r_s(p); dissolved gas above r_s(p) (1 + eps) -> x = s_g = 0; a
// negative r_go is set to 0.  Wet gas (rv_c > 0): oil below -eps (s_o =
// 1 - s_w - s_g) -> x = r_og = r_v(p); vaporised oil above r_v(p) (1 + eps)
// -> x = s_g = 1 - s_w; a negative r_og is set to 0.
__global__ __launch_bounds__(kBlock) void k_update(int n, double* y, const double* d,
                                                    double ds_max, double dp_max_rel,
                                                    uint8_t* meaning, double rs_c, double rv_c,
                                                    double eps, int32_t* flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int mean = meaning ? meaning[i] : 0;
  const double p = y[3 * i];
  double dp = -d[3 * i];
  const double lim = dp_max_rel * fabs(p);
  if (dp > lim) dp = lim;
  if (dp < -lim) dp = -lim;
  double dsw = -d[3 * i + 1], dx = -d[3 * i + 2];
  const double mx = mean == 0 ? fmax(fabs(dsw), fabs(dx)) : fabs(dsw);
  if (mx > ds_max) {
    const double sc = ds_max / mx;
    dsw *= sc;
    if (mean == 0) dx *= sc;
  }
  const double y0 = p + dp, y1 = y[3 * i + 1] + dsw;
  double y2 = y[3 * i + 2] + dx;
  if (meaning) {
    const double rs = rs_c * y0, rv = rv_c * y0;
    if (mean == 0) {
      if (y2 < -eps) {
        meaning[i] = 1;
        y2 = rs;
      } else if (rv_c > 0.0 && 1.0 - y1 - y2 < -eps) {
        meaning[i] = 2;
        y2 = rv;
      }
    } else if (mean == 1) {
      if (y2 > rs * (1.0 + eps)) {
        meaning[i] = 0;
        y2 = 0.0;
      } else if (y2 < 0.0) {
        y2 = 0.0;
      }
    } else if (y2 > rv * (1.0 + eps)) {
      meaning[i] = 0;
      y2 = 1.0 - y1;
    } else if (y2 < 0.0) {
      y2 = 0.0;
    }
  }
  y[3 * i] = y0;
  y[3 * i + 1] = y1;
  y[3 * i + 2] = y2;
  if (!isfinite(y0) || !isfinite(y1) || !isfinite(y2)) flags[1] = 1;
}

// Phase events of two consecutive Newton iterations (the times of an
// iteration's factorisation, solve and update are read at the next wait),
// and pinned host words for the step's status reads (the norms and flags
// after the assembly, the factorisation's flag, whose copy then does not
// hold the host until the factorisation ends).
struct Events {
  hipEvent_t e[2][5];
  hipEvent_t done = nullptr;   // polled for the status reads
  double* nrm = nullptr;     // [8]
  int32_t* flags = nullptr;  // [4]
  bool ok = false;
};

Events* events() {
  static thread_local Events ev;
  if (!ev.ok) {
    for (auto& set : ev.e)
      if (set[0] == nullptr)
        for (auto& x : set)
          if (hipEventCreate(&x) != hipSuccess) return nullptr;
    if (!ev.done && hipEventCreateWithFlags(&ev.done, hipEventDisableTiming) != hipSuccess)
      return nullptr;
    if (!ev.nrm) {
      void* p = nullptr;
      if (hipHostMalloc(&p, 8 * sizeof(double) + 4 * sizeof(int32_t), hipHostMallocDefault) !=
          hipSuccess)
        return nullptr;
      ev.flags = (int32_t*)p;   // [flags][norms], as in the workspace
      ev.nrm = (double*)((char*)p + 4 * sizeof(int32_t));
    }
    ev.ok = true;
  }
  return &ev;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms * 1e-3f;
}

bool valid_problem(const opm_problem* pb) {
  if (!pb || pb->n_cells < 0 || pb->n_faces < 0 || pb->nnzb != pb->n_cells + 2 * pb->n_faces)
    return false;
  if (pb->n_cells == 0) return true;
  return pb->trans && pb->pore_vol && pb->depth && pb->row_ptr && pb->col_idx && pb->blk_face &&
         pb->diag_pos && pb->level_ptr && pb->level_ptr_h && pb->perm && pb->iperm &&
         pb->lo_blk && pb->lo_tblk && pb->lo_pos && pb->up_blk && pb->up_pos &&
         pb->cell_conn_ptr && (pb->n_conns == 0 || (pb->cell_conn && pb->conn_kind &&
                                                     pb->conn_phase && pb->conn_wi &&
                                                     pb->conn_rate && pb->conn_bhp)) &&
         pb->n_levels > 0 && pb->level_ptr_h[pb->n_levels] == pb->n_cells &&
         (pb->fluid.live == 0 || (pb->fluid.live == 1 && pb->meaning && pb->fluid.rs_c >= 0.0 &&
                                  pb->fluid.bo_r >= 0.0 && pb->fluid.muo_r >= 0.0 &&
                                  pb->fluid.eps_switch >= 0.0 && pb->fluid.rv_c >= 0.0)) &&
         (pb->n_wells == 0 ||
          (pb->n_wells > 0 && pb->n_conns > 0 && pb->well_conn_ptr && pb->conn_cell &&
           pb->conn_well && pb->well_kind && pb->well_phase && pb->well_target && pb->well_vol &&
           pb->well_state && (!pb->well_limit || pb->well_ctrl)));
}

bool valid_prec(int p) { return p == OPM_PREC_FP64 || p == OPM_PREC_MIXED; }

int newton_step(const opm_problem* pb, double* y, const double* y_prev, double dt,
                const opm_newton_opts* o, void* work, opm_newton_report* rep, hipStream_t s) {
  const int n = pb->n_cells;
  NewtonWork w = carve(pb, o->precision, work);
  Events* evp = events();
  if (!evp) return OPM_EHIP;
  Events& ev = *evp;
  memset(rep, 0, sizeof(*rep));
  OPM_TRY(launch_accumulation(pb, y_prev, w.acc0, s));
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, w.flags);
  // standard wells: the well state at entry is the one at the start of the
  // step (its wellbore storage)
  const bool std_wells = pb->n_wells > 0;
  const WellWork& ww = w.wells;
  if (std_wells) OPM_TRY(well_storage0(pb, pb->well_state, ww.A0, s));
  WellSchur ws;
  std::memset(&ws, 0, sizeof ws);
  if (std_wells) ws = well_schur(pb, ww);
  std::vector<double> wn(std_wells ? pb->n_wells : 0);
  const bool use_cpr = o->precond == OPM_PRECOND_CPR;
  CprWork cw;
  std::memset(&cw, 0, sizeof cw);
  if (use_cpr) cw = cpr_carve(pb, w.cpr);
  int status = OPM_ENOTCONV;
  int pend = -1;   // the event set of an iteration whose later phases are not yet timed
  auto time_rest = [&](hipEvent_t* E) {
    rep->t_factor += elapsed(E[1], E[2]);
    rep->t_krylov += elapsed(E[2], E[3]);
  };
  // the previous convergence test's norms relative to the tolerances
  double far_c = HUGE_VAL, far_m = HUGE_VAL;
  for (int it = 0;; ++it) {
    hipEvent_t* E = ev.e[it & 1];
    OPM_TRY_HIP(hipEventRecord(E[0], s));
    OPM_TRY(launch_assemble(pb, y, w.acc0, dt, w.R, w.J, w.norms, s, std_wells ? ww.C : nullptr));
    if (std_wells) OPM_TRY(well_system(pb, y, dt, ww, w.flags, s));
    OPM_TRY_HIP(hipEventRecord(E[1], s));
    double* nrm = ev.nrm;
    int32_t* flags = ev.flags;
    OPM_TRY_HIP(hipMemcpyAsync(flags, w.flags, 4 * sizeof(int32_t) + 8 * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    if (std_wells)
      OPM_TRY_HIP(hipMemcpyAsync(wn.data(), ww.wn, sizeof(double) * wn.size(),
                                 hipMemcpyDeviceToHost, s));
    OPM_TRY_HIP(hipEventRecord(ev.done, s));
    // Where the previous test was far from converging (more than a thousand
    // times a tolerance; the first test of a step), the factorisation is
    // queued before the host reads this test's norms, so that the device
    // factorises while the host decides; a test that then converges leaves
    // a factorisation nobody reads (the flag words and norms were copied
    // before it).
    const bool ahead = it < o->max_newton && (far_c > 1e3 || far_m > 1e3);
    auto factor = [&]() -> int {
      OPM_TRY(ilu_factor(pb, w.J, w.ilu, o->precision, &w.flags[0], s));
      if (use_cpr) OPM_TRY(cpr_setup(pb, w.J, cw, &w.flags[0], s));
      return OPM_OK;
    };
    if (ahead) OPM_TRY(factor());
    OPM_TRY_HIP(spin_wait(ev.done));
    rep->t_assemble += elapsed(E[0], E[1]);
    if (pend >= 0) {
      time_rest(ev.e[pend]);
      rep->t_update += elapsed(ev.e[pend][3], ev.e[pend][4]);
      pend = -1;
    }
    for (int c = 0; c < 3; ++c) {
      rep->cnv[c] = nrm[c];
      rep->mb[c] = nrm[3 + c];
    }
    double cmax = nrm[6];
    for (double v : wn) cmax = std::isnan(v) ? v : std::fmax(cmax, v);
    far_c = cmax / o->tol_cnv;
    far_m = nrm[7] / o->tol_mb;
    if (flags[1] || !std::isfinite(cmax) || !std::isfinite(nrm[7])) {
      status = OPM_ENONFINITE;
      break;
    }
    if (flags[0] != 0) {   // a singular well matrix D
      status = flags[0];
      break;
    }
    if (cmax <= o->tol_cnv && nrm[7] <= o->tol_mb) {
      status = OPM_OK;
      break;
    }
    if (it >= o->max_newton) {
      status = OPM_ENOTCONV;
      break;
    }
    if (!ahead) OPM_TRY(factor());
    // the factorisation's flag (pinned: the copy is queued, the solver's
    // launches follow at once; read once the solve has been waited for)
    OPM_TRY_HIP(hipMemcpyAsync(flags, w.flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    OPM_TRY_HIP(hipEventRecord(E[2], s));
    opm_solve_report lr;
    if (std_wells) OPM_TRY(well_rhs(pb, ww, w.R, s));   // R_r - sum C D^-1 R_w
    if (o->krylov == OPM_KRYLOV_GMRES)
      OPM_TRY(gmres(pb, w.J, w.ilu, o->precision, w.R, w.d, o->lin_rtol, o->lin_maxit, o->restart,
                    w.krylov, &lr, s, use_cpr ? &cw : nullptr, std_wells ? &ws : nullptr));
    else
      OPM_TRY(bicgstab(pb, w.J, w.ilu, o->precision, w.R, w.d, o->lin_rtol, o->lin_maxit,
                       w.krylov, &lr, s, std_wells ? &ws : nullptr, use_cpr ? &cw : nullptr));
    OPM_TRY_HIP(hipEventRecord(E[3], s));
    rep->lin_its += lr.its;
    OPM_TRY_HIP(hipEventSynchronize(E[2]));   // (the flag's copy; the solve waited past it)
    if (flags[0] != 0 || lr.status != OPM_OK) {
      OPM_TRY_HIP(hipEventSynchronize(E[3]));
      time_rest(E);
      status = flags[0] != 0 ? flags[0] : lr.status;
      break;
    }
    if (std_wells)
      OPM_TRY(well_update(pb, ww, w.d, o->ds_max, o->dp_max_rel, w.flags, s));
    uint8_t* mean = pb->fluid.live ? pb->meaning : nullptr;
    hipLaunchKernelGGL(k_update, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, n, y, w.d,
                       o->ds_max, o->dp_max_rel, mean, pb->fluid.rs_c, pb->fluid.rv_c,
                       pb->fluid.eps_switch,
                       w.flags);
    OPM_TRY_HIP(hipGetLastError());
    OPM_TRY_HIP(hipEventRecord(E[4], s));
    pend = it & 1;
    rep->newton_its++;
    rep->cell_newton_its += (double)n;
  }
  rep->status = status;
  return status;
}

// Start of a Newton solve: y_prev or one of the candidates, whichever has the
// lowest max CNV (earlier entries win ties; non-finite norms never win).
// chosen = 0 for y_prev, k + 1 for cand[k]; cnv[0 .. ncand] the norms.
int guess_select(const opm_problem* pb, double* y, const double* y_prev,
                 const double* const* cand, int ncand, double dt, void* work, int32_t* chosen,
                 double* cnv, hipStream_t s) {
  NewtonWork w = carve(pb, OPM_PREC_FP64, work);
  OPM_TRY(launch_accumulation(pb, y_prev, w.acc0, s));
  double best = 0.0;
  int take = 0;
  for (int k = 0; k <= ncand; ++k) {
    const double* yk = k == 0 ? y_prev : cand[k - 1];
    double c = 0.0;
    OPM_TRY(launch_assemble(pb, yk, w.acc0, dt, w.R, w.J, w.norms, s));
    OPM_TRY_HIP(hipMemcpyAsync(&c, w.norms + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    OPM_TRY_HIP(hipStreamSynchronize(s));
    if (cnv) cnv[k] = c;
    if (k == 0 || (std::isfinite(c) && c < best)) {
      if (k == 0 && !std::isfinite(c)) best = INFINITY;
      else best = c;
      take = k;
    }
  }
  const double* src = take == 0 ? y_prev : cand[take - 1];
  const size_t bytes = sizeof(double) * 3 * (size_t)pb->n_cells;
  if (src != y) OPM_TRY_HIP(hipMemcpyAsync(y, src, bytes, hipMemcpyDeviceToDevice, s));
  OPM_TRY_HIP(hipStreamSynchronize(s));
  if (chosen) *chosen = take;
  return OPM_OK;
}

// Report step with cuts (sec. 2.3); the first full-length attempt may start
// from the learned guess or from its extrapolation path alone.
int advance(const opm_problem* pb, double* y, const double* y_nm1, double dt,
            const opm_newton_opts* opts, const opm_guess_net* net, void* guess_work,
            double* y_guess, void* work, double* y_save, opm_newton_report* report,
            int32_t* guess_used, hipStream_t s) {
  const size_t bytes = sizeof(double) * 3 * (size_t)pb->n_cells;
  memset(report, 0, sizeof(*report));
  if (guess_used) *guess_used = 0;
  // live oil: the variable meanings are saved and restored with the state
  uint8_t* mean_save = pb->fluid.live ? carve(pb, opts->precision, work).mean_save : nullptr;
  const size_t mbytes = (size_t)pb->n_cells;
  // standard wells: the well state likewise
  double* wsave = pb->n_wells > 0 ? carve(pb, opts->precision, work).wells.save : nullptr;
  const size_t wbytes = sizeof(double) * 4 * (size_t)pb->n_wells;
  // and the wells' active controls
  int32_t* csave = pb->n_wells > 0 && pb->well_limit
                       ? carve(pb, opts->precision, work).wells.save_ctrl : nullptr;
  const size_t cbytes = sizeof(int32_t) * (size_t)pb->n_wells;
  OPM_TRY_HIP(hipMemcpyAsync(y_save, y, bytes, hipMemcpyDeviceToDevice, s));
  if (mean_save)
    OPM_TRY_HIP(hipMemcpyAsync(mean_save, pb->meaning, mbytes, hipMemcpyDeviceToDevice, s));
  if (wsave)
    OPM_TRY_HIP(hipMemcpyAsync(wsave, pb->well_state, wbytes, hipMemcpyDeviceToDevice, s));
  if (csave)
    OPM_TRY_HIP(hipMemcpyAsync(csave, pb->well_ctrl, cbytes, hipMemcpyDeviceToDevice, s));
  double t = 0.0, dt_try = dt;
  int status = OPM_OK;
  bool first = true;
  while (dt - t > 1e-9 * dt) {
    const double h = fmin(dt_try, dt - t);
    if (first && net) {
      const double* y_ext = nullptr;
      OPM_TRY(guess_infer(pb, net, y_save, y_nm1, y_guess, guess_work, s, &y_ext));
      const double* cand[2] = {y_guess, y_ext};
      OPM_TRY(guess_select(pb, y, y_save, cand, 2, h, work, guess_used, nullptr, s));
    }
    first = false;
    opm_newton_report r1;
    int st = newton_step(pb, y, y_save, h, opts, work, &r1, s);
    if (st == OPM_EHIP || st == OPM_EINVAL) return st;
    report->newton_its += r1.newton_its;
    report->lin_its += r1.lin_its;
    report->cell_newton_its += r1.cell_newton_its;
    report->t_assemble += r1.t_assemble;
    report->t_factor += r1.t_factor;
    report->t_krylov += r1.t_krylov;
    report->t_update += r1.t_update;
    if (st == OPM_OK) {
      for (int c = 0; c < 3; ++c) {
        report->cnv[c] = r1.cnv[c];
        report->mb[c] = r1.mb[c];
      }
      OPM_TRY_HIP(hipMemcpyAsync(y_save, y, bytes, hipMemcpyDeviceToDevice, s));
      if (mean_save)
        OPM_TRY_HIP(hipMemcpyAsync(mean_save, pb->meaning, mbytes, hipMemcpyDeviceToDevice, s));
      if (wsave)
        OPM_TRY_HIP(hipMemcpyAsync(wsave, pb->well_state, wbytes, hipMemcpyDeviceToDevice, s));
      if (csave)
        OPM_TRY_HIP(hipMemcpyAsync(csave, pb->well_ctrl, cbytes, hipMemcpyDeviceToDevice, s));
      t += h;
      report->substeps++;
    } else {
      OPM_TRY_HIP(hipMemcpyAsync(y, y_save, bytes, hipMemcpyDeviceToDevice, s));
      if (mean_save)
        OPM_TRY_HIP(hipMemcpyAsync(pb->meaning, mean_save, mbytes, hipMemcpyDeviceToDevice, s));
      if (wsave)
        OPM_TRY_HIP(hipMemcpyAsync(pb->well_state, wsave, wbytes, hipMemcpyDeviceToDevice, s));
      if (csave)
        OPM_TRY_HIP(hipMemcpyAsync(pb->well_ctrl, csave, cbytes, hipMemcpyDeviceToDevice, s));
      dt_try = 0.5 * h;
      report->cuts++;
      if (report->cuts > opts->max_cuts) {
        status = st;
        break;
      }
    }
  }
  Events* evp = events();
  if (!evp) return OPM_EHIP;
  OPM_TRY_HIP(hipEventRecord(evp->done, s));
  OPM_TRY_HIP(spin_wait(evp->done));
  report->status = status;
  return status;
}

}  // namespace
}  // namespace opm

using namespace opm;

extern "C" {

int opm_init(void) {
  int dev = 0;
  OPM_TRY_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  OPM_TRY_HIP(hipGetDeviceProperties(&prop, dev));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return OPM_EHIP;
  (void)events();
  return assemble_scratch_setup(dev);
}

int opm_set_option(int option, int value) {
  switch (option) {
    case OPM_OPT_SWEEP_MODE:
      if (value < -1 || value > 2) return OPM_EINVAL;
      g_sweep_mode = value;
      return OPM_OK;
    case OPM_OPT_KRYLOV_GRAPH:
      if (value < 0 || value > 1) return OPM_EINVAL;
      g_krylov_graph = value;
      return OPM_OK;
    case OPM_OPT_ASSEMBLY:
      if (value < 0 || value > 1) return OPM_EINVAL;
      g_assembly_kernel = value;
      return OPM_OK;
    case OPM_OPT_PLANE_SWEEP:
      if (value < 0 || value > 1) return OPM_EINVAL;
      g_plane_sweep = value;
      return OPM_OK;
    case OPM_OPT_PLANE_SPIN:
      if (value < 0) return OPM_EINVAL;
      g_plane_spin = value;
      return OPM_OK;
    case OPM_OPT_ENSEMBLE_SPIN:
      if (value < 0) return OPM_EINVAL;
      g_ens_spin = value;
      return OPM_OK;
    case OPM_OPT_KRYLOV_CHUNK:
      if (value < 0) return OPM_EINVAL;
      g_krylov_chunk = value;
      return OPM_OK;
    case OPM_OPT_SWEEP_KERNEL:
      if (value < 0 || value > 6) return OPM_EINVAL;
      g_sweep_kernel = value;
      return OPM_OK;
    case OPM_OPT_BLOCK_DEPTH:
      if (value < 0 || value > 2) return OPM_EINVAL;
      g_block_depth = value;
      return OPM_OK;
    default:
      return OPM_EINVAL;
  }
}

const char* opm_strerror(int code) {
  switch (code) {
    case OPM_OK: return "ok";
    case OPM_EINVAL: return "invalid argument";
    case OPM_ESINGULAR: return "singular 3x3 pivot block in ILU(0)";
    case OPM_ENOTCONV: return "not converged";
    case OPM_EBREAKDOWN: return "BiCGStab breakdown";
    case OPM_ENONFINITE: return "non-finite residual or state";
    case OPM_EHIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

int opm_accumulation(const opm_problem* pb, const double* y, double* acc0, void* stream) {
  if (!valid_problem(pb) || (pb->n_cells > 0 && (!y || !acc0))) return OPM_EINVAL;
  if (pb->n_cells == 0) return OPM_OK;
  return launch_accumulation(pb, y, acc0, as_stream(stream));
}

size_t opm_norms_bytes(const opm_problem* pb) { return pb ? norms_bytes(pb) : 0; }

int opm_assemble(const opm_problem* pb, const double* y, const double* acc0, double dt, double* R,
                 double* J, double* norms, void* stream) {
  if (!valid_problem(pb) || !(dt > 0.0) || (pb->n_cells > 0 && (!y || !acc0 || !R)))
    return OPM_EINVAL;
  if (pb->n_cells == 0) return OPM_OK;
  return launch_assemble(pb, y, acc0, dt, R, J, norms, as_stream(stream));
}

int opm_assemble_noalloc(const opm_problem* pb, const double* y, const double* acc0, double dt,
                         double* R, double* J, double* norms, void* stream) {
  if (pb && ((long)pb->n_cells > assemble_noalloc_max_cells() ||
             assemble_workgroups(pb, nullptr) > assemble_noalloc_max_cells() / kBlock))
    return OPM_EINVAL;
  if (!valid_problem(pb) || !(dt > 0.0) || (pb->n_cells > 0 && (!y || !acc0 || !R)))
    return OPM_EINVAL;
  if (pb->n_cells == 0) return OPM_OK;
  return launch_assemble_noalloc(pb, y, acc0, dt, R, J, norms, as_stream(stream));
}

size_t opm_ilu0_bytes(const opm_problem* pb, int precision) {
  return pb && valid_prec(precision) ? ilu_bytes(pb, precision) : 0;
}

int opm_ilu0_factor(const opm_problem* pb, const double* J, void* ilu, int precision,
                    int32_t* status, void* stream) {
  if (!valid_problem(pb) || !valid_prec(precision) || (pb->n_cells > 0 && (!J || !ilu)))
    return OPM_EINVAL;
  if (pb->n_cells == 0) return OPM_OK;
  return ilu_factor(pb, J, ilu, precision, status, as_stream(stream));
}

int opm_ilu0_apply(const opm_problem* pb, const void* ilu, int precision, const double* r,
                   double* x, void* stream) {
  if (!valid_problem(pb) || !valid_prec(precision) || (pb->n_cells > 0 && (!ilu || !r || !x)) ||
      (pb->n_cells > 0 && r == x))
    return OPM_EINVAL;
  if (pb->n_cells == 0) return OPM_OK;
  return ilu_apply(pb, const_cast<void*>(ilu), precision, r, x, as_stream(stream), nullptr);
}

int opm_spmv(const opm_problem* pb, const double* J, const double* x, double* y, void* stream) {
  if (!valid_problem(pb) || (pb->n_cells > 0 && (!J || !x || !y))) return OPM_EINVAL;
  return spmv(pb, J, x, y, as_stream(stream));
}

size_t opm_krylov_bytes(const opm_problem* pb) { return pb ? krylov_bytes(pb) : 0; }

int opm_bicgstab(const opm_problem* pb, const double* J, const void* ilu, int precision,
                 const double* b, double* x, double rtol, int32_t maxit, void* work,
                 opm_solve_report* report, void* stream) {
  if (!valid_problem(pb) || !valid_prec(precision) || !(rtol >= 0.0) || maxit < 0 || !report ||
      (pb->n_cells > 0 && (!J || !ilu || !b || !x || !work)))
    return OPM_EINVAL;
  if (pb->n_cells == 0) {
    memset(report, 0, sizeof(*report));
    return OPM_OK;
  }
  return bicgstab(pb, J, const_cast<void*>(ilu), precision, b, x, rtol, maxit, work, report,
                  as_stream(stream));
}

size_t opm_gmres_bytes(const opm_problem* pb, int32_t restart) {
  return pb && restart >= 1 && restart <= OPM_GMRES_MAX_RESTART ? gmres_bytes(pb, restart) : 0;
}

int opm_gmres(const opm_problem* pb, const double* J, const void* ilu, int precision,
              const double* b, double* x, double rtol, int32_t maxit, int32_t restart, void* work,
              opm_solve_report* report, void* stream) {
  if (!valid_problem(pb) || !valid_prec(precision) || !(rtol >= 0.0) || maxit < 0 || !report ||
      restart < 1 || restart > OPM_GMRES_MAX_RESTART ||
      (pb->n_cells > 0 && (!J || !ilu || !b || !x || !work)))
    return OPM_EINVAL;
  if (pb->n_cells == 0) {
    memset(report, 0, sizeof(*report));
    return OPM_OK;
  }
  return gmres(pb, J, const_cast<void*>(ilu), precision, b, x, rtol, maxit, restart, work,
               report, as_stream(stream));
}

size_t opm_wells_bytes(const opm_problem* pb) {
  return pb && pb->n_wells > 0 ? wells_bytes(pb) : 0;
}

int opm_assemble_wells(const opm_problem* pb, const double* y, const double* acc0,
                       const double* well_state0, double dt, double* R, double* J, double* Rw,
                       double* B, double* C, double* D, void* work, void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || pb->n_wells <= 0 || !y || !acc0 ||
      !well_state0 || !(dt > 0.0) || !R || !J || !Rw || !B || !C || !D || !work)
    return OPM_EINVAL;
  hipStream_t s = as_stream(stream);
  WellWork ww = wells_carve(pb, work);
  ww.Rw = Rw;
  ww.B = B;
  ww.C = C;
  ww.D = D;
  int32_t* flags = (int32_t*)ww.save;   // scratch for the status word
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, flags);
  OPM_TRY(well_storage0(pb, well_state0, ww.A0, s));
  OPM_TRY(launch_assemble(pb, y, acc0, dt, R, J, nullptr, s, C));
  OPM_TRY(well_system(pb, y, dt, ww, flags, s));
  int32_t f = 0;
  OPM_TRY_HIP(hipMemcpyAsync(&f, flags, sizeof f, hipMemcpyDeviceToHost, s));
  OPM_TRY_HIP(hipStreamSynchronize(s));
  return f;
}

size_t opm_newton_bytes(const opm_problem* pb, int precision) {
  return pb && valid_prec(precision) ? newton_bytes(pb, precision) : 0;
}

static bool valid_krylov(const opm_newton_opts* o) {
  return o->krylov == OPM_KRYLOV_BICGSTAB ||
         (o->krylov == OPM_KRYLOV_GMRES && o->restart >= 1 &&
          o->restart <= OPM_GMRES_MAX_RESTART);
}

size_t opm_newton_work_bytes(const opm_problem* pb, const opm_newton_opts* opts) {
  return pb && opts && valid_prec(opts->precision) && valid_krylov(opts)
             ? newton_bytes(pb, opts->precision, opts->krylov, opts->restart)
             : 0;
}

static bool valid_opts(const opm_newton_opts* o) {
  return o && valid_prec(o->precision) && o->max_newton >= 0 && o->lin_maxit >= 0 &&
         o->max_cuts >= 0 && o->ds_max > 0.0 && o->dp_max_rel > 0.0 && o->lin_rtol >= 0.0 &&
         o->tol_cnv >= 0.0 && o->tol_mb >= 0.0 && valid_krylov(o) &&
         (o->precond == OPM_PRECOND_ILU0 || o->precond == OPM_PRECOND_CPR);
}

// The CPR hierarchy referenced by the problem fits it: level 0 is the block
// pattern, the coarsest level has at most OPM_AMG_COARSE unknowns and every
// array a level needs is there.
static bool valid_amg(const opm_problem* pb) {
  const opm_amg* g = pb->amg;
  if (!g || g->n_levels < 1 || g->n_levels > OPM_AMG_MAX_LEVELS || g->n[0] != pb->n_cells ||
      g->nnz[0] != pb->nnzb || g->n[g->n_levels - 1] > OPM_AMG_COARSE ||
      g->n[g->n_levels - 1] < 1)
    return false;
  for (int l = 0; l < g->n_levels; ++l) {
    if (l >= 1 && (!g->row_ptr[l] || !g->col[l] || !g->dpos[l] || !g->gmap_ptr[l] ||
                   !g->gmap[l] || g->n[l] < 1 || g->nnz[l] < g->n[l]))
      return false;
    if (l + 1 < g->n_levels && (!g->agg[l] || !g->child_ptr[l] || !g->child[l])) return false;
  }
  return true;
}

// CPR needs the hierarchy.
static bool valid_wells_opts(const opm_problem* pb, const opm_newton_opts* o) {
  return o->precond == OPM_PRECOND_ILU0 || valid_amg(pb);
}

size_t opm_cpr_bytes(const opm_problem* pb) {
  return pb && pb->n_cells > 0 && valid_amg(pb) ? cpr_bytes(pb) : 0;
}

int opm_cpr_setup(const opm_problem* pb, const double* J, void* cpr, int32_t* status,
                  void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !valid_amg(pb) || !J || !cpr || !status)
    return OPM_EINVAL;
  return cpr_setup(pb, J, cpr_carve(pb, cpr), status, as_stream(stream));
}

int opm_cpr_vcycle(const opm_problem* pb, const void* cpr, const double* b, double* x,
                   void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !valid_amg(pb) || !cpr || !b || !x)
    return OPM_EINVAL;
  hipStream_t s = as_stream(stream);
  const CprWork w = cpr_carve(pb, const_cast<void*>(cpr));
  OPM_TRY(cpr_vcycle(pb, w, nullptr, b, s, nullptr));
  OPM_TRY_HIP(hipMemcpyAsync(x, w.y[0], sizeof(double) * pb->n_cells, hipMemcpyDeviceToDevice,
                             s));
  return OPM_OK;
}

int opm_cpr_apply(const opm_problem* pb, const double* J, const void* ilu, int precision,
                  const void* cpr, const double* r, double* z, void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !valid_amg(pb) || !valid_prec(precision) || !J ||
      !ilu || !cpr || !r || !z || r == z)
    return OPM_EINVAL;
  return cpr_apply(pb, J, const_cast<void*>(ilu), precision,
                   cpr_carve(pb, const_cast<void*>(cpr)), r, z, as_stream(stream), nullptr);
}

int opm_cpr_values(const opm_problem* pb, const void* cpr, int32_t level, double* a,
                   double* w, void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !valid_amg(pb) || !cpr || level < 0 ||
      level >= pb->amg->n_levels)
    return OPM_EINVAL;
  hipStream_t s = as_stream(stream);
  const CprWork cw = cpr_carve(pb, const_cast<void*>(cpr));
  if (a)
    OPM_TRY_HIP(hipMemcpyAsync(a, cw.a[level], sizeof(double) * pb->amg->nnz[level],
                               hipMemcpyDeviceToDevice, s));
  if (w)
    OPM_TRY_HIP(hipMemcpyAsync(w, cw.w, sizeof(double) * 3 * pb->n_cells,
                               hipMemcpyDeviceToDevice, s));
  return OPM_OK;
}

int opm_bicgstab_cpr(const opm_problem* pb, const double* J, const void* ilu, int precision,
                     const void* cpr, const double* b, double* x, double rtol, int32_t maxit,
                     void* work, opm_solve_report* report, void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !valid_amg(pb) || !valid_prec(precision) ||
      !(rtol >= 0.0) || maxit < 0 || !report || !J || !ilu || !cpr || !b || !x || !work)
    return OPM_EINVAL;
  const CprWork cw = cpr_carve(pb, const_cast<void*>(cpr));
  return bicgstab(pb, J, const_cast<void*>(ilu), precision, b, x, rtol, maxit, work, report,
                  as_stream(stream), nullptr, &cw);
}

int opm_newton_step(const opm_problem* pb, double* y, const double* y_prev, double dt,
                    const opm_newton_opts* opts, void* work, opm_newton_report* report,
                    void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !valid_opts(opts) || !(dt > 0.0) || !y ||
      !y_prev || !work || !report || !valid_wells_opts(pb, opts))
    return OPM_EINVAL;
  return newton_step(pb, y, y_prev, dt, opts, work, report, as_stream(stream));
}

int opm_advance(const opm_problem* pb, double* y, double dt, const opm_newton_opts* opts,
                void* work, double* y_save, opm_newton_report* report, void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !valid_opts(opts) || !(dt > 0.0) || !y ||
      !y_save || !work || !report || !valid_wells_opts(pb, opts))
    return OPM_EINVAL;
  return advance(pb, y, nullptr, dt, opts, nullptr, nullptr, nullptr, work, y_save, report,
                 nullptr, as_stream(stream));
}

int opm_guess_select(const opm_problem* pb, double* y, const double* y_prev,
                     const double* y_guess, double dt, void* work, int32_t* chosen, double* cnv,
                     void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !(dt > 0.0) || !y || !y_prev || !y_guess ||
      !work || pb->fluid.live != 0 || pb->n_wells != 0)
    return OPM_EINVAL;
  return guess_select(pb, y, y_prev, &y_guess, 1, dt, work, chosen, cnv, as_stream(stream));
}

int opm_advance_guess(const opm_problem* pb, double* y, const double* y_nm1, double dt,
                      const opm_newton_opts* opts, const opm_guess_net* net, void* guess_work,
                      double* y_guess, void* work, double* y_save, opm_newton_report* report,
                      int32_t* guess_used, void* stream) {
  if (!valid_problem(pb) || pb->n_cells == 0 || !valid_opts(opts) || !(dt > 0.0) || !y ||
      !y_save || !work || !report)
    return OPM_EINVAL;
  if (!valid_wells_opts(pb, opts) ||
      (net && (!y_nm1 || !guess_work || !y_guess || opm_guess_work_bytes(pb, net) == 0 ||
               pb->fluid.live != 0 || pb->n_wells != 0)))
    return OPM_EINVAL;
  return advance(pb, y, y_nm1, dt, opts, net, guess_work, y_guess, work, y_save, report,
                 guess_used, as_stream(stream));
}

}  // extern "C"
