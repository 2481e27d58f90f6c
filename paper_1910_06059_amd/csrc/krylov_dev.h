// Device-side state of the BiCGStab iteration (paper sec. 2.3.1), shared by
// the Krylov kernels (krylov.hip) and the block-ILU0 sweeps that fuse a
// vector update of the iteration into their right-hand side (ilu0.hip).
//
// Every scalar lives in device memory; every dot product is a two-stage
// fixed-order reduction whose per-workgroup partials are summed by the
// consuming kernel itself, in the same order in every workgroup, so all
// workgroups of a kernel see bit-identical scalars and take the same
// decisions.  A state word (running / half-step exit / done) lets kernels of
// an iteration that is no longer needed return at once.
#pragma once

#include "common.h"

namespace opm {
namespace kry {

constexpr int kMaxGrid = 1024;   // workgroups of the vector kernels (partials per reduction)

enum State : int32_t { kRunning = 0, kHalfPending = 1, kDone = 2 };

struct Scalars {
  double rho, rho0, alpha, omega, bnorm, tol, relres, pad;
  int32_t state, status, its, half, maxit, pad2[3];
};

// A vector update of the iteration computed by a block-ILU0 sweep for the
// rows of its subdomain, as the right-hand side of the preconditioner solve.
enum FusedMode : int { kFuseNone = 0, kFuseBegin = 1, kFuseS = 2 };
struct Fused {
  const double* r;          // residual
  double* p;                // kFuseBegin: search direction, updated in place
  const double* v;          // A p^
  double* s;                // kFuseS: s = r - alpha v (out)
  const double* part_a;     // kFuseBegin: partials of <r,r>; kFuseS: of <r^,v>
  const double* part_b;     // kFuseBegin: partials of <r^,r>
  int n_part;               // number of those partials
  double* part_out;         // kFuseS: partials of <s,s>, one per workgroup
  Scalars* sc;
};

// Sum of the G partials of a reduction by NT threads (identical in every
// workgroup of the same size).
// A thread's partials are loaded eight at a time (clamped indices, those
// past G taken as exact zeros: v starts at +0 and never becomes -0, so
// adding +0 changes nothing) and added in index order, the same sum as one
// load at a time with all eight loads in flight together.
template <int NT>
__device__ __forceinline__ double sum_partials(const double* part, int G, double* sh) {
  double v = 0.0;
  for (int k0 = threadIdx.x; k0 < G; k0 += 8 * NT) {
    double p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u * NT;
      const double pv = part[min(k, G - 1)];
      p[u] = k < G ? pv : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v += p[u];
  }
  return block_sum<NT>(v, sh);
}

// The first of this thread's partials of a sum of G >= 1 (a clamped index:
// no branch around the load, so that it can go out early).
__device__ __forceinline__ double partial_first(const double* part, int G) {
  return part[min((int)threadIdx.x, G - 1)];
}

// This thread's share of the sum of G partials (sum_partials before its
// workgroup sum, in the same order) from its first partial.
template <int NT>
__device__ __forceinline__ double partials_share(const double* part, int G, double first) {
  double v = 0.0;
  if ((int)threadIdx.x < G) v += first;
  // the rest eight at a time, as in sum_partials
  for (int k0 = threadIdx.x + NT; k0 < G; k0 += 8 * NT) {
    double p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u * NT;
      const double pv = part[min(k, G - 1)];
      p[u] = k < G ? pv : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) v += p[u];
  }
  return v;
}

// Start of an iteration: the convergence / iteration-cap / breakdown tests
// on the residual of the previous iteration.  Returns true if the iteration
// runs, with beta and omega of p = r + beta (p - omega v).  `state` is the
// state word as read once for the whole workgroup.
template <int NT>
__device__ __forceinline__ bool begin_iteration(Scalars& s, int state, const double* part_rr,
                                                const double* part_rhr, int G, double* sh,
                                                double& beta, double& om) {
  if (state != kRunning) {
    if (state == kHalfPending && blockIdx.x == 0 && threadIdx.x == 0) s.state = kDone;
    return false;
  }
  // the iteration's scalars (not written by this kernel) and both first
  // partials go out before either sum waits (no load moves above the sums'
  // barriers)
  const int its = s.its, maxit = s.maxit;
  const double tol = s.tol, om_prev = s.omega, rho0 = s.rho0, alpha = s.alpha;
  const double f_rr = partial_first(part_rr, G), f_rhr = partial_first(part_rhr, G);
  const double rr = block_sum<NT>(partials_share<NT>(part_rr, G, f_rr), sh);
  const double rho = block_sum<NT>(partials_share<NT>(part_rhr, G, f_rhr), sh);
  const double rnorm = sqrt(rr);
  int verdict = kRunning, status = OPM_OK;
  if (rnorm <= tol) {
    verdict = kDone;
  } else if (its > 0 && om_prev == 0.0) {
    verdict = kDone;
    status = OPM_EBREAKDOWN;
  } else if (its >= maxit) {
    verdict = kDone;
    status = OPM_ENOTCONV;
  } else if (fabs(rho) < 1e-300) {
    verdict = kDone;
    status = OPM_EBREAKDOWN;
  }
  if (verdict == kDone) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      s.status = status;
      s.relres = s.bnorm > 0.0 ? rnorm / s.bnorm : 0.0;
      s.state = kDone;
    }
    return false;
  }
  beta = its == 0 ? 0.0 : (rho / rho0) * (alpha / om_prev);
  om = om_prev;
  if (blockIdx.x == 0 && threadIdx.x == 0) s.rho = rho;
  return true;
}

// alpha = rho / <r^, v> (breakdown on a zero denominator).  Returns true if
// the iteration goes on.
template <int NT>
__device__ __forceinline__ bool alpha_step(Scalars& sc, int state, const double* part_rv, int G,
                                           double* sh, double& alpha) {
  if (state != kRunning) return false;
  const double rho = sc.rho;   // (read before the sum's barriers)
  const double rv = sum_partials<NT>(part_rv, G, sh);
  if (rv == 0.0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc.status = OPM_EBREAKDOWN;
      sc.state = kDone;
    }
    return false;
  }
  alpha = rho / rv;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc.alpha = alpha;
  return true;
}

// Half-step exit test ||s|| <= tol on the threads' shares of the partials
// of <s, s>.  Returns true if the iteration goes on.
template <int NT>
__device__ __forceinline__ bool half_step_check_share(Scalars& sc, int state, double share,
                                                      double* sh) {
  if (state != kRunning) return false;
  const double tol = sc.tol;   // (read before the sum's barriers)
  const double snorm = sqrt(block_sum<NT>(share, sh));
  if (snorm <= tol) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc.half = 1;
      sc.relres = snorm / sc.bnorm;
      sc.its += 1;
      sc.state = kHalfPending;
    }
    return false;
  }
  return true;
}

// Half-step exit test ||s|| <= tol.  Returns true if the iteration goes on.
template <int NT>
__device__ __forceinline__ bool half_step_check(Scalars& sc, int state, const double* part_ss,
                                                int G, double* sh) {
  if (state != kRunning) return false;
  return half_step_check_share<NT>(sc, state,
                                   partials_share<NT>(part_ss, G, partial_first(part_ss, G)), sh);
}

// The state word read once per workgroup (every wavefront of the workgroup
// takes the same branch even if another workgroup changes the word).
__device__ __forceinline__ int read_state(const Scalars* sc, int* shared_word) {
  if (threadIdx.x == 0) *shared_word = sc->state;
  __syncthreads();
  return *shared_word;
}

}  // namespace kry
}  // namespace opm
