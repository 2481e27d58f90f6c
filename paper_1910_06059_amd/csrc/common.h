// Internal helpers shared by the HIP sources of the library (not part of the
// ABI): error handling, launch geometry and fixed-order block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "opm_gpu.h"

// A failed HIP call is reported as OPM_EHIP; the runtime's last-error state
// is cleared so that the caller's next HIP call does not inherit it.
#define OPM_TRY_HIP(call)                      \
  do {                                         \
    hipError_t opm_e_ = (call);                \
    if (opm_e_ != hipSuccess) {                \
      (void)hipGetLastError();                 \
      return OPM_EHIP;                         \
    }                                          \
  } while (0)

#define OPM_TRY(call)                \
  do {                               \
    int opm_s_ = (call);             \
    if (opm_s_ != OPM_OK) return opm_s_; \
  } while (0)

namespace opm {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kBlock = 256;         // default workgroup: 4 waves
constexpr int kNormStride = 10;     // per-block partials of the CNV/MB norms

inline int blocks_for(long n, int per_block) { return (int)((n + per_block - 1) / per_block); }

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Host wait for an event by polling it (a blocking wait may put the thread
// to sleep and wake it well after the work ended, with the device idle
// until the next launch); after about four million polls it blocks.
inline hipError_t spin_wait(hipEvent_t e) {
  for (long k = 0; k < (1L << 22); ++k) {
    const hipError_t q = hipEventQuery(e);
    if (q != hipErrorNotReady) return q;
  }
  return hipEventSynchronize(e);
}

// Sum over a workgroup, fixed tree order (deterministic).  All threads of the
// block must call it; the result is returned to every thread.  `sh` needs
// blockDim.x / 64 doubles of LDS.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < NT / kWave; ++k) s += sh[k];
  return s;
}

// max that propagates NaN (fmax would drop it and hide a non-finite residual)
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a != a || a > b) ? a : b;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
  for (int off = kWave / 2; off > 0; off >>= 1) v = nan_max(v, __shfl_down(v, off, kWave));
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = sh[0];
  for (int k = 1; k < NT / kWave; ++k) s = nan_max(s, sh[k]);
  return s;
}

// 3x3 helpers (row-major) -----------------------------------------------
template <typename T>
__device__ __forceinline__ void matvec3(const T* A, const T* x, T* y) {
  y[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
  y[1] = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
  y[2] = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
}

}  // namespace opm
