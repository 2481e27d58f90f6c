// CPR-AMG preconditioner (paper sec. 2.3.1): the device workspace and the
// host entry points used by the Krylov solvers and the Newton step.
#pragma once

#include "common.h"

namespace opm {

// Device workspace: the quasi-IMPES weights, the pressure column of every
// block of J (stored compactly for the second-stage residual), per level the
// matrix values, diagonal, right-hand side, restricted-to-be residual and
// smoothed solution, the inverse of the coarsest matrix, and the
// second-stage residual.
struct CprWork {
  double* w;
  double* jp;
  double* a[OPM_AMG_MAX_LEVELS];
  double* d[OPM_AMG_MAX_LEVELS];
  double* b[OPM_AMG_MAX_LEVELS];
  double* res[OPM_AMG_MAX_LEVELS];
  double* y[OPM_AMG_MAX_LEVELS];
  double* inv;
  double* r2;
};

size_t cpr_bytes(const opm_problem* pb);
CprWork cpr_carve(const opm_problem* pb, void* p);
// Setup for the Jacobian J; flags[0] (device) gets OPM_ESINGULAR on a
// singular diagonal block or coarsest matrix.
int cpr_setup(const opm_problem* pb, const double* J, const CprWork& w, int32_t* flags,
              hipStream_t s);
// x_p = V-cycle(b), the result in w.y[0]; b = w^T r when r is set, else
// the given b0 (n values).
int cpr_vcycle(const opm_problem* pb, const CprWork& w, const double* r, const double* b0,
               hipStream_t s, const int32_t* skip);
// z = CPR(r) with the (block-)ILU(0) factors ilu of J; nothing while
// *skip != 0 (skip may be null).
int cpr_apply(const opm_problem* pb, const double* J, void* ilu, int precision, const CprWork& w,
              const double* r, double* z, hipStream_t s, const int32_t* skip);

}  // namespace opm
