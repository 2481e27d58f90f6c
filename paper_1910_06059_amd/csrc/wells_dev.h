// The Schur complement of the standard-well equations (paper sec. 2.2.1,
// eq. wellequation) as the Krylov solvers see it: the operator
// y = A x - sum_w C_w D_w^{-1} B_w x is the block-CSR SpMV with a
// per-connection correction subtracted from the rows of perforated cells.
#pragma once

#include "common.h"

namespace opm {

// Correction read by the SpMV: row i subtracts corr[t] for each connection
// t of cell i (cell_conn_ptr / cell_conn).  corr == nullptr: no wells.
struct WellCorr {
  const int32_t* ccp;
  const int32_t* cc;
  const double* corr;   // [n_conns][3]
};

// What the correction kernel needs: per well its connections, the blocks
// B [n_conns][4][3] and C [n_conns][3][4], and D^{-1} [n_wells][4][4].
struct WellSchur {
  int n_wells;
  const int32_t* well_conn_ptr;
  const int32_t* conn_cell;
  const double* B;
  const double* C;
  const double* Dinv;
  double* corr;
  const int32_t* ccp;
  const int32_t* cc;
  WellCorr wc() const { return WellCorr{ccp, cc, corr}; }
};

// corr = C D^{-1} B x per connection (one workgroup per well); returns at
// once while *skip != 0 (skip may be null).
int well_op(const WellSchur& ws, const double* x, const int32_t* skip, hipStream_t s);

// Device workspace of the standard wells (part of the Newton workspace):
// R_w [nw][4], B [nc][4][3], C [nc][3][4], D and D^{-1} [nw][4][4], the
// per-connection correction [nc][3], the storage at the step start
// [nw][3], the wells' convergence measures [nw] and a saved state [nw][4].
struct WellWork {
  double *Rw, *B, *C, *D, *Dinv, *corr, *A0, *wn, *save;
  int32_t* save_ctrl;   // the active controls saved with the well state
};
size_t wells_bytes(const opm_problem* pb);
WellWork wells_carve(const opm_problem* pb, void* p);
WellSchur well_schur(const opm_problem* pb, const WellWork& ww);
// A0 = V_w mix_a of the well state wx.
int well_storage0(const opm_problem* pb, const double* wx, double* A0, hipStream_t s);
// R_w, B, D, D^{-1} and the convergence measures at y (flags[0] =
// OPM_ESINGULAR on a singular D).
int well_system(const opm_problem* pb, const double* y, double dt, const WellWork& ww,
                int32_t* flags, hipStream_t s);
// R -= sum_w C_w D_w^{-1} R_w.
int well_rhs(const opm_problem* pb, const WellWork& ww, double* R, hipStream_t s);
// x_w -= D^{-1} (R_w - B d) with the chop (flags[1] on a non-finite state).
int well_update(const opm_problem* pb, const WellWork& ww, const double* d, double ds_max,
                double dp_max_rel, int32_t* flags, hipStream_t s);

}  // namespace opm
