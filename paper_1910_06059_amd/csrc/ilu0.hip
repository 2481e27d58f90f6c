// Block ILU(0) preconditioner (paper sec. 2.3.1: the default ILU0 with
// BiCGStab, on block-CSR storage).
//
// For a pattern whose graph has no triangles (the 7-point TPFA stencil of a
// Cartesian grid: two neighbours of a cell are never neighbours of each
// other), ILU(0) creates no update of any off-diagonal block, so the factors
// are L_ik = A_ik D_k^{-1} (k < i), U_ij = A_ij (j > i) and the pivot blocks
//   D_i = A_ii - sum_{k<i, k in C(i)} A_ik D_k^{-1} A_ki .
// Only D_i^{-1} has to be computed.  Rows are processed by dependency level
// (all lower neighbours of a row sit on earlier levels), which gives the same
// factors as the natural order.  The triangular solves of M = LU become
//   forward:  y_i = D_i^{-1} (r_i - sum_{k<i} A_ik y_k)        (y = D^{-1} w)
//   backward: x_i = y_i - D_i^{-1} sum_{j>i} A_ij x_j .
//
// Data layout: everything the sweeps read is in level order (position p of
// the schedule, rows of one level contiguous) and structure-of-arrays
// (element e of row p at [e * ns + p]), so a wavefront reads consecutive
// addresses: the three lower and three upper off-diagonal blocks of each row,
// D^{-1}, and a level-ordered scratch vector z that holds y after the
// forward sweep and x after the backward sweep.  In mixed precision these
// arrays are FP32 while D^{-1} is still computed in FP64.
//
// Launch shapes:
//  - one workgroup walks all levels with workgroup barriers (systems whose
//    widest level is small): the results of the previous level stay in an
//    LDS window, and the matrix data of the next level is loaded before the
//    barrier so that its latency overlaps the current level;
//  - one launch per level over many workgroups (large systems).
// Packing the off-diagonal blocks into level order does not depend on the
// levels and runs as one wide kernel over all rows.
#include "krylov_dev.h"
#include "solver_dev.h"

namespace opm {

extern int g_sweep_kernel;
extern int g_block_depth;
extern int g_plane_sweep;
extern int g_plane_spin;

namespace {

using namespace ilu;

constexpr int kWgThreads = 512;        // threads of the one-workgroup sweep
constexpr int kFacThreads = 256;       // threads of the one-workgroup factorisation
constexpr int kMaxWindowRows = 2048;   // widest level served by the one-workgroup sweep
constexpr int kMaxFactorWindowRows = 640;
constexpr size_t kMaxRingBytes = 128 * 1024;   // LDS budget of the sweep ring
constexpr size_t kMaxBlockLds = 150 * 1024;    // LDS budget of a block-ILU0 workgroup

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack(Topo t, const double* J, IluView<T> v) {
  const int pos = blockIdx.x * kBlock + threadIdx.x;
  if (pos < t.n) pack_row<T>(t, J, v, pos);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_factor_level(Topo t, const double* J, IluView<T> v,
                                                          int p0, int p1, int32_t* status) {
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos >= p1) return;
  FacJob j;
  load_fac(t, J, pos, j);
  double inv[9];
  finish_fac<T>(j, pos, v,
                [&](int kp, double* Dk) {
#pragma unroll
                  for (int e = 0; e < 9; ++e) Dk[e] = v.dinv64[(size_t)e * v.ns + kp];
                },
                status, inv);
}

template <typename T, bool WINDOW>
__global__ __launch_bounds__(kFacThreads) void k_factor_wg(Topo t, const double* J, IluView<T> v,
                                                            int32_t* status) {
  extern __shared__ double fwin[];
  factor_levels_wg<T, WINDOW, kFacThreads>(t, J, v, status, fwin);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd_level(Topo t, IluView<T> v, int p0, int p1,
                                                       const double* r, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos >= p1) return;
  SweepJob<T> j;
  load_fwd(t, v, r, pos, j);
  T y[3];
  solve_row<T, true>(j, [&](int kp, T* xv) {
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[c] = v.z[(size_t)c * v.ns + kp];
  }, y);
#pragma unroll
  for (int c = 0; c < 3; ++c) v.z[(size_t)c * v.ns + pos] = y[c];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bwd_level(Topo t, IluView<T> v, int p0, int p1,
                                                       double* x, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int pos = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (pos >= p1) return;
  SweepJob<T> j;
  load_bwd(t, v, pos, j);
  T xo[3];
  solve_row<T, false>(j, [&](int kp, T* xv) {
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[c] = v.z[(size_t)c * v.ns + kp];
  }, xo);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v.z[(size_t)c * v.ns + pos] = xo[c];
    x[3 * j.cell + c] = (double)xo[c];
  }
}

template <typename T>
__global__ __launch_bounds__(kWgThreads) void k_apply_ring(Topo t, IluView<T> v, const double* r,
                                                            double* x, const int32_t* skip,
                                                            unsigned mask) {
  if (skip && *skip != 0) return;
  extern __shared__ unsigned char smem[];
  apply_levels_ring<T, kWgThreads>(t, v, r, x, reinterpret_cast<T*>(smem), mask);
}

// r gathered into z4 in level order (the right-hand side of the record sweep).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_rhs(int n, const int32_t* perm, IluView<T> v,
                                                       const double* r, const int32_t* skip) {
  if (skip && *skip != 0) return;
  const int pos = blockIdx.x * kBlock + threadIdx.x;
  if (pos >= n) return;
  const size_t cell = (size_t)perm[pos];
#pragma unroll
  for (int c = 0; c < 3; ++c) v.z4[4 * (size_t)pos + c] = (T)r[3 * cell + c];
  v.z4[4 * (size_t)pos + 3] = (T)0;
}

// Sweep records of every row position (after the factorisation): the
// forward record holds the lower blocks and D^{-1}, the backward one the
// upper blocks and D^{-1}, each with the neighbour positions and the row.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pack_records(Topo t, IluView<T> v) {
  const int pos = blockIdx.x * kBlock + threadIdx.x;
  if (pos >= t.n) return;
  constexpr size_t kV = 16 / sizeof(T);
  const size_t ns = (size_t)v.ns, p = (size_t)pos;
#pragma unroll
  for (int e = 0; e < kRecValues; ++e) {
    const size_t a = ((size_t)e / kV * ns + p) * kV + (size_t)e % kV;
    v.rec_f[a] = e < 27 ? v.lov[e * ns + p] : v.dinv[(e - 27) * ns + p];
    v.rec_b[a] = e < 27 ? v.upv[e * ns + p] : v.dinv[(e - 27) * ns + p];
  }
  const int cell = t.perm[pos];
  v.idx_f[pos] = int4v{t.lo_pos[3 * p], t.lo_pos[3 * p + 1], t.lo_pos[3 * p + 2], cell};
  v.idx_b[pos] = int4v{t.up_pos[3 * p], t.up_pos[3 * p + 1], t.up_pos[3 * p + 2], cell};
}

// The end of a level: a workgroup barrier, or for a one-wavefront
// workgroup a wavefront-scope fence (the wavefront's LDS operations are
// performed in order, so the next level's reads see this level's writes
// without waiting for them to complete).
template <int NT>
__device__ __forceinline__ void level_barrier() {
  if (NT == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// ------------------------------------------------------------ block ILU0
// One workgroup per subdomain (the blocks of the block ILU0 are independent,
// so the whole factorisation and each whole preconditioner solve are one
// launch).  Inside a subdomain the rows go level by level with workgroup
// barriers.  The rows of subdomain s on level l are the positions
// [slp[l (nsub+1) + s], slp[l (nsub+1) + s + 1]).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_factor_blocks(Topo t, const double* J, IluView<T> v,
                                                       const int32_t* slp, int nsub,
                                                       int max_width, int32_t* status) {
  // inverse pivots of the previous and the current level of the subdomain
  // (every lower neighbour in the subdomain lies on the previous level)
  extern __shared__ double fwin[];   // [2][max_width][9]
  const int s = blockIdx.x;
  auto range = [&](int l, int& p0, int& p1) {
    p0 = slp[(size_t)l * (nsub + 1) + s];
    p1 = slp[(size_t)l * (nsub + 1) + s + 1];
  };
  int p0, p1;
  range(0, p0, p1);
  FacJob next;
  if (p0 + (int)threadIdx.x < p1) load_fac(t, J, p0 + threadIdx.x, next);
  int prev0 = 0, prev1 = 0, buf = 0;
  for (int l = 0; l < t.nlev; ++l) {
    int q0 = 0, q1 = 0;
    if (l + 1 < t.nlev) range(l + 1, q0, q1);
    const FacJob cur = next;
    // the next level's blocks load while this level is computed
    if (q0 + (int)threadIdx.x < q1) load_fac(t, J, q0 + threadIdx.x, next);
    auto finish = [&](const FacJob& j, int pos) {
      double inv[9];
      finish_fac<T>(j, pos, v,
                    [&](int kp, double* Dk) {
                      if (kp >= prev0 && kp < prev1) {
                        const double* w = fwin + ((size_t)(buf ^ 1) * max_width + (kp - prev0)) * 9;
#pragma unroll
                        for (int e = 0; e < 9; ++e) Dk[e] = w[e];
                      } else {
#pragma unroll
                        for (int e = 0; e < 9; ++e) Dk[e] = v.dinv64[(size_t)e * v.ns + kp];
                      }
                    },
                    status, inv);
      double* w = fwin + ((size_t)buf * max_width + (pos - p0)) * 9;
#pragma unroll
      for (int e = 0; e < 9; ++e) w[e] = inv[e];
    };
    if (p0 + (int)threadIdx.x < p1) finish(cur, p0 + threadIdx.x);
    // rows of levels wider than the workgroup
    for (int pos = p0 + NT + (int)threadIdx.x; pos < p1; pos += NT) {
      FacJob extra;
      load_fac(t, J, pos, extra);
      finish(extra, pos);
    }
    __syncthreads();
    prev0 = p0;
    prev1 = p1;
    buf ^= 1;
    p0 = q0;
    p1 = q1;
  }
}

// The data load_fac reads, split in its three dependent parts: the row's
// cell and lower-block indices, the diagonal block's index, the blocks.
struct FacIdx {
  int i;
  int blk[3], tblk[3], kpos[3];
};

__device__ __forceinline__ void load_fac_idx(const Topo& t, int pos, FacIdx& a) {
  a.i = t.perm[pos];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    a.blk[s] = t.lo_blk[3 * pos + s];
    a.tblk[s] = t.lo_tblk[3 * pos + s];
    a.kpos[s] = t.lo_pos[3 * pos + s];
  }
}

__device__ __forceinline__ void load_fac_blocks(const double* J, int dpos, const FacIdx& a,
                                                FacJob& j) {
  const double* Aii = J + 9 * (size_t)dpos;
#pragma unroll
  for (int e = 0; e < 9; ++e) j.D[e] = Aii[e];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int b = a.blk[s];
    j.kp[s] = b < 0 ? -1 : a.kpos[s];
    const double* A = J + 9 * (size_t)(b < 0 ? 0 : b);
    const double* B = J + 9 * (size_t)(b < 0 ? 0 : a.tblk[s]);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      j.Aik[s][e] = A[e];
      j.Aki[s][e] = B[e];
    }
  }
}

// Block-ILU0 pivot recursion of a subdomain of at most 64 levels (their
// bounds in registers, lane l holding level l's), its loads spread over
// three levels: while level l is computed, the blocks of level l+1, the
// diagonal-block index of level l+2 and the indices of level l+3 are
// loaded, each from values loaded a level earlier, so that no level waits
// for load_fac's chain of three dependent loads.  Lanes past a level's end
// load a clamped row and compute nothing.  The values and the arithmetic
// are k_factor_blocks' (bitwise equal pivots).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_factor_blocks_pipe(Topo t, const double* J, IluView<T> v,
                                                            const int32_t* slp, int nsub,
                                                            int max_width, int32_t* status) {
  extern __shared__ double fwin[];   // [2][max_width][9]
  const int s = blockIdx.x, nlev = t.nlev, tid = (int)threadIdx.x;
  int rb = 0, re = 0;
  {
    const int lane = tid & 63;
    if (lane < nlev) {
      rb = slp[(size_t)lane * (nsub + 1) + s];
      re = slp[(size_t)lane * (nsub + 1) + s + 1];
    }
  }
  auto pos_of = [&](int l) {
    const int lc = min(l, nlev - 1);
    const int p0 = __builtin_amdgcn_readlane(rb, lc), p1 = __builtin_amdgcn_readlane(re, lc);
    return max(min(p0 + tid, p1 - 1), 0);
  };
  FacIdx a1, a2, a3;
  int b1, b2;
  FacJob next;
  {
    FacIdx a0;
    load_fac_idx(t, pos_of(0), a0);
    load_fac_idx(t, pos_of(1), a1);
    load_fac_idx(t, pos_of(2), a2);
    const int b0 = t.diag_pos[a0.i];
    b1 = t.diag_pos[a1.i];
    load_fac_blocks(J, b0, a0, next);
  }
  int prev0 = 0, prev1 = 0, buf = 0;
  for (int l = 0; l < nlev; ++l) {
    const int p0 = __builtin_amdgcn_readlane(rb, l), p1 = __builtin_amdgcn_readlane(re, l);
    const FacJob cur = next;
    load_fac_blocks(J, b1, a1, next);
    b2 = t.diag_pos[a2.i];
    load_fac_idx(t, pos_of(l + 3), a3);
    auto finish = [&](const FacJob& j, int pos) {
      double inv[9];
      finish_fac<T>(j, pos, v,
                    [&](int kp, double* Dk) {
                      if (kp >= prev0 && kp < prev1) {
                        const double* w = fwin + ((size_t)(buf ^ 1) * max_width + (kp - prev0)) * 9;
#pragma unroll
                        for (int e = 0; e < 9; ++e) Dk[e] = w[e];
                      } else {
#pragma unroll
                        for (int e = 0; e < 9; ++e) Dk[e] = v.dinv64[(size_t)e * v.ns + kp];
                      }
                    },
                    status, inv);
      double* w = fwin + ((size_t)buf * max_width + (pos - p0)) * 9;
#pragma unroll
      for (int e = 0; e < 9; ++e) w[e] = inv[e];
    };
    if (p0 + tid < p1) finish(cur, p0 + tid);
    // rows of levels wider than the workgroup
    for (int pos = p0 + NT + tid; pos < p1; pos += NT) {
      FacJob extra;
      load_fac(t, J, pos, extra);
      finish(extra, pos);
    }
    level_barrier<NT>();
    prev0 = p0;
    prev1 = p1;
    buf ^= 1;
    a1 = a2;
    a2 = a3;
    b1 = b2;
  }
}

// Sweep records of the block ILU0, straight from the Jacobian (after the
// pivot recursion).  Record (row, a) holds row a of the three off-diagonal
// blocks (lower ones forward, upper ones backward) and row a of D^{-1}: 12
// values as 16-byte chunks, chunk c of (position p, a) at [(c ns + p) 3 + a]
// so that the three lanes of a row and consecutive rows read consecutive
// chunks.  Index records: neighbours by slot in the subdomain, and the cell.
// A workgroup packs 32 consecutive positions: their Jacobian rows (at most
// 7 blocks each, contiguous in J) are read into LDS by 8 lanes per row, then
// 96 threads write the forward and 96 the backward records, each thread one
// (position, a) for every chunk, so consecutive threads write consecutive
// chunks.
constexpr int kPackRows = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_pack_block_records(Topo t, const int32_t* row_ptr,
                                                            const double* J, IluView<T> v,
                                                            const int32_t* slot) {
  typedef typename Vec16<T>::type V;
  constexpr unsigned kV = 16 / sizeof(T), kC = 12 / kV;
  __shared__ double rows[kPackRows][64];
  __shared__ int rbase[kPackRows];
  const int p0 = blockIdx.x * kPackRows;
  {
    const int g = threadIdx.x >> 3, l = threadIdx.x & 7, pos = p0 + g;
    if (pos < t.n) {
      const int cell = t.perm[pos];
      const int b0 = row_ptr[cell], nv = 9 * (row_ptr[cell + 1] - b0);
      const double* src = J + 9 * (size_t)b0;
      for (int e = l; e < nv; e += 8) rows[g][e] = src[e];
      if (l == 0) rbase[g] = b0;
    }
  }
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < 192) {
    const bool fwd = tid < 96;
    const int q = fwd ? tid : tid - 96, g = q / 3, a = q % 3, pos = p0 + g;
    if (pos < t.n) {
      const size_t ns = (size_t)v.ns, up = (size_t)pos;
      const int32_t* blk = (fwd ? t.lo_blk : t.up_blk) + 3 * up;
      int loc[3];
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) loc[sl] = blk[sl] < 0 ? -1 : blk[sl] - rbase[g];
      V* rec = reinterpret_cast<V*>(fwd ? v.rec_f : v.rec_b);
#pragma unroll
      for (unsigned c = 0; c < kC; ++c) {
        V w;
#pragma unroll
        for (unsigned qq = 0; qq < kV; ++qq) {
          const unsigned e = c * kV + qq;
          T val;
          if (e < 9u) {
            const int sl = (int)e / 3, col = (int)e % 3;
            val = loc[sl] < 0 ? (T)0 : (T)rows[g][9 * loc[sl] + 3 * a + col];
          } else {
            val = v.dinv[(size_t)(3 * a + (int)e - 9) * ns + up];
          }
          w[qq] = val;
        }
        rec[(c * ns + up) * 3 + a] = w;
      }
    }
  } else if (tid < 192 + kPackRows) {
    const int pos = p0 + tid - 192;
    if (pos < t.n) {
      const size_t p = (size_t)pos;
      auto nb = [&](int kp) { return kp < 0 ? kp : slot[kp]; };
      const int cell = t.perm[pos];
      v.idx_f[pos] = int4v{nb(t.lo_pos[3 * p]), nb(t.lo_pos[3 * p + 1]), nb(t.lo_pos[3 * p + 2]), cell};
      v.idx_b[pos] = int4v{nb(t.up_pos[3 * p]), nb(t.up_pos[3 * p + 1]), nb(t.up_pos[3 * p + 2]), cell};
    }
  }
}

// Block-ILU0 sweep rows are spread over a quad of lanes, lane a < 3 per
// equation a: lane a holds row a of the three neighbour blocks and of
// D^{-1} (12 values, the record of (row, a)), computes its partial sum
//   acc_a = r_a - sum_s A_s[a][.] x_s   (forward; backward with + and 0),
// takes acc_b of the two other lanes of the quad by DPP quad permutation
// and finishes with D^{-1}[a][.] acc.  The arithmetic and its order per
// value are those of the other sweep kernels (bitwise equal results).  A
// wavefront holds 16 rows (lanes 4q + a; lane 4q + 3 repeats lane 4q + 2's
// work and stores nothing), the widest level of a 4x4 column.  Records,
// right-hand sides and the index are read with buffer loads (one 32-bit
// offset per level, chunk offsets in scalar registers).
constexpr int kRowsPerWave = 16;
// Word 3 of a raw buffer resource on gfx9 (32-bit data format, no swizzle).
constexpr int kBufferWord3 = 0x00020000;
// A value in LDS (address space 3: 32-bit addresses).
template <typename T>
using Lds = __attribute__((address_space(3))) T;

__device__ __forceinline__ int block_lane_row() {
  return (int)(threadIdx.x >> 6) * kRowsPerWave + (int)(threadIdx.x & 63u) / 4;
}
__device__ __forceinline__ int block_lane_eq() { return (int)(threadIdx.x & 3u); }

// Value of lane K of the lane's quad (DPP quad permutation: a VALU move, no
// LDS round trip).
template <int K>
__device__ __forceinline__ double quad_lane(double x) {
  constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int K>
__device__ __forceinline__ float quad_lane(float x) {
  constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), ctrl, 0xf, 0xf, false));
}

template <typename T>
struct BlockJob {
  T a[9];      // row a of the three neighbour blocks
  T d[3];      // row a of D^{-1}
  T rhs;       // backward: component a of y
  double u[3]; // forward: the vector values the right-hand side is made of
  int kp[3];   // neighbour slots (-1 if absent)
  int cell;
  int slot;
  bool live;
};

// Forward right-hand side of a sweep: r itself, or (fused with BiCGStab)
// p = r + beta (p - omega v) or s = r - alpha v, written back for the rows
// of the level.
struct BlockRhs {
  const double* r;
  kry::Fused f;
  double beta, omega, alpha;
};

// A sweep of one subdomain is a three-stage pipeline over its levels: the
// neighbour slots and cells of level k+2 and the records and right-hand
// sides of level k+1 are loaded while level k is computed.  The right-hand
// side of the forward sweep is r at the row's cell, so its address needs
// the index loaded earlier; loading the index in the same stage would make
// the wait for it (the load counter drains in order) also wait for the
// previous level's data.  No branch separates a load from its use (lanes
// past a level's end load a clamped row and store nothing), so the
// compiler never has to assume a load of an earlier level still in flight.

// Level k of the sweep (ascending levels forward, descending backward;
// past the last one: the last one), the lane's clamped row position and
// the row's index record; the data stage reuses the bounds.
struct BlockStage {
  int4v ix;
  int p0, p1, pos;
  bool in;   // k is a level of the sweep
};

__device__ const int32_t kZeroWord = 0;

// Level bounds of the workgroup's subdomain: from the LDS table, or (at
// most 64 levels) from registers, lane l of every wavefront holding level
// l's bounds (a read is then a lane read, no LDS round trip).
template <bool REG>
struct LevelBounds {
  const int* lp;
  int b, e;
  __device__ __forceinline__ int begin(int l) const {
    return REG ? __builtin_amdgcn_readlane(b, l) : lp[2 * l];
  }
  __device__ __forceinline__ int end(int l) const {
    return REG ? __builtin_amdgcn_readlane(e, l) : lp[2 * l + 1];
  }
};

template <typename T, bool FWD, typename LB>
__device__ __forceinline__ BlockStage block_index(IluView<T> v, const LB& lb, int nlev, int k,
                                                  int row) {
  BlockStage st;
  const int kk = k < nlev ? k : nlev - 1;
  const int l = FWD ? kk : nlev - 1 - kk;
  st.p0 = lb.begin(l);
  st.p1 = lb.end(l);
  st.pos = max(min(st.p0 + row, st.p1 - 1), 0);
  st.in = k < nlev;
  st.ix = (FWD ? v.idx_f : v.idx_b)[(unsigned)st.pos];
  return st;
}

// base: rows of the subdomain before the level (forward) or up to and
// including it (backward).  Missing neighbours (index -1) read the zero row
// at slot zslot.
template <typename T, bool FWD, int MODE>
__device__ __forceinline__ void block_data(IluView<T> v, const BlockRhs& q, const Lds<T>* zl, int row,
                                           int base, int zslot, const BlockStage& st,
                                           BlockJob<T>& j) {
  typedef typename Vec16<T>::type V;
  constexpr unsigned kV = 16 / sizeof(T), kC = 12 / kV;
  const int eq = block_lane_eq();
  const unsigned a = (unsigned)min(eq, 2);
  j.live = st.in && st.p0 + row < st.p1 && eq < 3;
  const unsigned ns = (unsigned)v.ns, up = (unsigned)st.pos;
  // (an absent neighbour, -1, is the largest unsigned value: the zero row)
  j.kp[0] = (int)min((unsigned)st.ix.x, (unsigned)zslot);
  j.kp[1] = (int)min((unsigned)st.ix.y, (unsigned)zslot);
  j.kp[2] = (int)min((unsigned)st.ix.z, (unsigned)zslot);
  j.cell = st.ix.w;
  j.slot = (FWD ? base : base - (st.p1 - st.p0)) + (st.pos - st.p0);
  // buffer loads: one 32-bit lane offset per level, the chunk offsets in
  // scalar registers (no 64-bit address arithmetic per load); reads past
  // the records return zero
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(FWD ? v.rec_f : v.rec_b), (short)0, (int)(kC * ns * 48u), kBufferWord3);
  const int voff = (int)((up * 3u + a) * 16u);
#pragma unroll
  for (unsigned c = 0; c < kC; ++c) {
    const V w = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(
                                          rs, voff, (int)(c * ns * 48u), 0));
#pragma unroll
    for (unsigned qq = 0; qq < kV; ++qq) {
      const unsigned e = c * kV + qq;
      if (e < 9u)
        j.a[e] = w[qq];
      else
        j.d[e - 9u] = w[qq];
    }
  }
  if (FWD) {
    const int off = (int)((3u * (unsigned)j.cell + a) * 8u);
    auto ld = [&](const double* base) {
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          (void*)base, (short)0, 0x7fffffff, kBufferWord3);
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    };
    if (MODE == kry::kFuseNone) j.u[0] = ld(q.r);
    if (MODE == kry::kFuseBegin) {
      j.u[0] = ld(q.f.r);
      j.u[1] = ld(q.f.p);
      j.u[2] = ld(q.f.v);
    }
    if (MODE == kry::kFuseS) {
      j.u[0] = ld(q.f.r);
      j.u[1] = ld(q.f.v);
    }
  } else {
    // y of the row (forward result); slots of lanes past the level's end
    // stay inside the subdomain
    j.rhs = zl[__umul24((unsigned)max(j.slot, 0), 3u) + a];
  }
  // keep every load of the stage here, ahead of the computation of the
  // current level (the compiler would otherwise sink some of them to their
  // first use, behind the next stage's loads), and keep the arithmetic on
  // them after this point (hoisted above the loads it would wait for them
  // at once)
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// The neighbour values of a row (the previous level's results).  A missing
// neighbour reads the zero row: x = 0 exactly, as in the other sweep
// kernels (slots are below 2^24: 24-bit multiplies).
template <typename T>
__device__ __forceinline__ void block_x(const BlockJob<T>& j, const Lds<T>* zl, T* xv) {
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const Lds<T>* w = zl + __umul24((unsigned)j.kp[s], 3u);
    xv[3 * s] = w[0];
    xv[3 * s + 1] = w[1];
    xv[3 * s + 2] = w[2];
  }
}

// Every lane computes (the shuffles need all lanes); only rows of the level
// store.  xv: block_x of the row.
template <typename T, bool FWD, int MODE>
__device__ __forceinline__ void block_row(const BlockJob<T>& j, const T* xv, Lds<T>* zl,
                                          double* x, const BlockRhs& q, double& ss) {
  const int eq = block_lane_eq();
  const unsigned a = (unsigned)min(eq, 2);
  // forward right-hand side (the same expressions as the unfused vector
  // kernels of the iteration)
  double u = j.u[0];
  if (FWD && MODE == kry::kFuseBegin) u = j.u[0] + q.beta * (j.u[1] - q.omega * j.u[2]);
  if (FWD && MODE == kry::kFuseS) u = j.u[0] - q.alpha * j.u[1];
  const T rhs = FWD ? (T)u : j.rhs;
  T acc = FWD ? rhs : (T)0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const T t = j.a[3 * s] * xv[3 * s] + j.a[3 * s + 1] * xv[3 * s + 1] +
                j.a[3 * s + 2] * xv[3 * s + 2];
    acc = FWD ? acc - t : acc + t;
  }
  const T acc0 = quad_lane<0>(acc), acc1 = quad_lane<1>(acc), acc2 = quad_lane<2>(acc);
  const T d = j.d[0] * acc0 + j.d[1] * acc1 + j.d[2] * acc2;
  const T out = FWD ? d : j.rhs - d;
  if (!j.live) return;
  zl[__umul24((unsigned)j.slot, 3u) + a] = out;
  if (!FWD) x[3u * (unsigned)j.cell + a] = (double)out;
  if (FWD && MODE == kry::kFuseBegin) q.f.p[3u * (unsigned)j.cell + a] = u;
  if (FWD && MODE == kry::kFuseS) {
    q.f.s[3u * (unsigned)j.cell + a] = u;
    ss += u * u;
  }
}

// Rows of a level beyond the first NT / 64 * 16 (subdomains with wider
// levels).
template <typename T, int NT, bool FWD, int MODE, typename LB>
__device__ __forceinline__ void block_extra(IluView<T> v, const BlockRhs& q, Lds<T>* zl, double* x,
                                            const LB& lb, int nlev, int k, int base, int zslot,
                                            double& ss) {
  constexpr int kRows = NT / 64 * kRowsPerWave;
  const int l = FWD ? k : nlev - 1 - k;
  const int w = lb.end(l) - lb.begin(l);
  // uniform trip count: every lane joins the shuffles of every round
  for (int r0 = kRows; r0 < w; r0 += kRows) {
    const int row = r0 + block_lane_row();
    const BlockStage st = block_index<T, FWD>(v, lb, nlev, k, row);
    BlockJob<T> j;
    block_data<T, FWD, MODE>(v, q, zl, row, base, zslot, st, j);
    T xv[9];
    block_x(j, zl, xv);
    block_row<T, FWD, MODE>(j, xv, zl, x, q, ss);
  }
}

// DEPTH: levels whose data is in flight while a level is computed.  At the
// step that computes level s the index stage loads level s + DEPTH + 2 and
// the data stage loads level s + DEPTH from the index loaded two steps
// earlier, so no load waits for one issued in the previous step.  The
// stages rotate through register rings (3 indices, DEPTH + 1 jobs), fully
// unrolled over a period of P steps so that every ring slot is a register.
template <typename T, int NT, bool FWD, bool WIDE, int DEPTH, int MODE, typename LB,
          typename Gate>
__device__ __forceinline__ bool block_sweep(IluView<T> v, BlockRhs& q, Lds<T>* zl, double* x,
                                            const LB& lb, int nlev, int nrows, int zslot,
                                            double& ss, Gate gate) {
  constexpr int ND = DEPTH + 1, NI = 3;
  // (two turns of the rings at DEPTH 2: the waits at a period's end drain
  // the loads in flight, so a longer period drains less often)
  constexpr int P = ND % NI == 0 ? 2 * ND : ND * NI;
  const int row = block_lane_row();
  auto next_base = [&](int b, int k) {
    const int l = FWD ? k : nlev - 1 - k;
    const int w = k < nlev ? lb.end(l) - lb.begin(l) : 0;
    return FWD ? b + w : b - w;
  };
  int ik = 0;                                 // index stage: next level
  int dk = 0, db = FWD ? 0 : nrows;           // data stage: next level and its base
  int ck = 0, cb = db;                        // compute stage
  auto index = [&]() { return block_index<T, FWD>(v, lb, nlev, ik++, row); };
  auto data = [&](const BlockStage& st, BlockJob<T>& j) {
    block_data<T, FWD, MODE>(v, q, zl, row, db, zslot, st, j);
    const int w = st.in ? st.p1 - st.p0 : 0;
    db = FWD ? db + w : db - w;
    ++dk;
  };
  auto compute = [&](const BlockJob<T>& j, const T* xv) {
    block_row<T, FWD, MODE>(j, xv, zl, x, q, ss);
    if (WIDE) block_extra<T, NT, FWD, MODE>(v, q, zl, x, lb, nlev, ck, cb, zslot, ss);
    cb = next_base(cb, ck++);
    level_barrier<NT>();
  };
  BlockJob<T> jobs[ND];
  BlockStage idx[NI];
  // prologue: data of levels 0 .. DEPTH-1, indices of DEPTH and DEPTH+1
  // (each index slot is read before it is loaded again)
#pragma unroll
  for (int q = 0; q < DEPTH; ++q) {
    idx[q % NI] = index();
    data(idx[q % NI], jobs[q % ND]);
  }
  idx[DEPTH % NI] = index();
  idx[(DEPTH + 1) % NI] = index();
  // with the first levels' loads in flight: the decisions that need the
  // iteration's scalars (their loads overlap those of the sweep)
  if (!gate(q)) return false;
  // whole periods of P steps without an exit between their steps (an exit
  // per step would leave the compiler, where the exits join, without a
  // count of the loads in flight, and it would wait for all of them at the
  // next period), then the last partial period step by step
  // the current level's neighbour reads go out first: their LDS latency
  // overlaps the issue of the later levels' loads
  auto step = [&](int qq) __attribute__((always_inline)) {
    T xv[9];
    block_x(jobs[qq % ND], zl, xv);
    __builtin_amdgcn_sched_barrier(0);
    idx[(qq + DEPTH + 2) % NI] = index();
    data(idx[(qq + DEPTH) % NI], jobs[(qq + DEPTH) % ND]);
    compute(jobs[qq % ND], xv);
  };
  int k = 0;
  for (; k + P <= nlev; k += P) {
#pragma unroll
    for (int qq = 0; qq < P; ++qq) step(qq);
  }
#pragma unroll
  for (int qq = 0; qq < P - 1; ++qq) {
    if (k + qq >= nlev) break;
    step(qq);
  }
  return true;
}

// x = M^{-1} r for the block ILU0: forward then backward sweep of one
// subdomain per workgroup, the subdomain's y and x in LDS (3 values per
// row, by slot), then the level bounds of the subdomain (2 ints per level).
// MODE (kry::FusedMode): the forward right-hand side is r, or the p or s
// update of a BiCGStab iteration, preceded by the tests of that iteration
// (every workgroup evaluates them on the same partials and returns at once
// if the iteration does not run); with the s update the workgroup's partial
// of <s, s> goes to f.part_out.
template <typename T, int NT, bool WIDE, int DEPTH, int MODE, bool LVR>
__global__ __launch_bounds__(NT) void k_apply_blocks(IluView<T> v, const int32_t* slp, int nsub,
                                                      int nlev, int max_sub, const double* r,
                                                      double* x, const int32_t* skip,
                                                      kry::Fused f) {
  __shared__ double red[NT / 64];
  __shared__ int word;
  // the skip flag or the iteration's state word (read once for the
  // workgroup) go out together with the level bounds
  // (a uniform read in every wavefront; thread 0's value is the workgroup's;
  // without a skip flag the zero word is read: no branch around the load)
  typedef const __attribute__((address_space(1))) int32_t GlobalWord;
  const int skipv = MODE == kry::kFuseNone ? *(GlobalWord*)(skip ? skip : &kZeroWord) : 0;
  const int st0 = MODE != kry::kFuseNone ? f.sc->state : 0;
  extern __shared__ unsigned char smem[];
  // [max_sub + 1][3], the last row zero; an LDS-qualified pointer keeps the
  // address arithmetic in 32 bits
  Lds<T>* zl = (Lds<T>*)reinterpret_cast<T*>(smem);
  int* lp = reinterpret_cast<int*>(smem + sizeof(T) * 3 * ((size_t)max_sub + 1));
  const int s = blockIdx.x;
  LevelBounds<LVR> lb{lp, 0, 0};
  if (LVR) {   // every wavefront: lane l holds level l
    const int lane = (int)(threadIdx.x & 63u);
    if (lane < nlev) {
      lb.b = slp[(size_t)lane * (nsub + 1) + s];
      lb.e = slp[(size_t)lane * (nsub + 1) + s + 1];
    }
  }
  for (int l = threadIdx.x; l < nlev; l += NT) {
    lp[2 * l] = slp[(size_t)l * (nsub + 1) + s];
    lp[2 * l + 1] = slp[(size_t)l * (nsub + 1) + s + 1];
  }
  if (threadIdx.x < 3) zl[3 * (size_t)max_sub + threadIdx.x] = (T)0;
  if (MODE != kry::kFuseNone && threadIdx.x == 0) word = st0;
  __syncthreads();
  if (MODE == kry::kFuseNone && skipv != 0) return;
  int state = kry::kRunning;
  if (MODE != kry::kFuseNone) {
    state = word;
    if (state != kry::kRunning) {
      if (MODE == kry::kFuseBegin && state == kry::kHalfPending && blockIdx.x == 0 &&
          threadIdx.x == 0)
        f.sc->state = kry::kDone;
      return;
    }
  }
  int nrows = 0;
  for (int l = 0; l < nlev; ++l) nrows += lp[2 * l + 1] - lp[2 * l];
  BlockRhs q{r, f, 0.0, 0.0, 0.0};
  // the iteration's tests and scalars (every workgroup on the same partials)
  auto gate = [&](BlockRhs& qq) -> bool {
    if (MODE == kry::kFuseBegin)
      return kry::begin_iteration<NT>(*f.sc, state, f.part_a, f.part_b, f.n_part, red, qq.beta,
                                      qq.omega);
    if (MODE == kry::kFuseS)
      return kry::alpha_step<NT>(*f.sc, state, f.part_a, f.n_part, red, qq.alpha);
    return true;
  };
  auto open = [](BlockRhs&) { return true; };
  double ss = 0.0;
  if (!block_sweep<T, NT, true, WIDE, DEPTH, MODE>(v, q, zl, x, lb, nlev, nrows, max_sub, ss,
                                                   gate))
    return;
  if (MODE == kry::kFuseS) {
    const double tot = block_sum<NT>(ss, red);
    if (threadIdx.x == 0) f.part_out[blockIdx.x] = tot;
  }
  block_sweep<T, NT, false, WIDE, DEPTH, MODE>(v, q, zl, x, lb, nlev, nrows, max_sub, ss, open);
}

// Both sweeps by one workgroup of NT threads through the LDS ring with
// branch-free prefetch (the right-hand side already in z, see k_gather_rhs).
template <typename T, int NT, bool WIDE, bool SKIP>
__global__ __launch_bounds__(NT) void k_apply_ring2(Topo t, IluView<T> v, double* x,
                                                     const int32_t* skip, unsigned mask) {
  if (skip && *skip != 0) return;
  extern __shared__ unsigned char smem[];
  T* ring = reinterpret_cast<T*>(smem);
  ilu::ring2_sweep<T, NT, true, WIDE, SKIP>(t, v, x, ring, mask);
  // each lane reads back in the backward sweep only z values that it wrote
  // itself in the forward sweep (same level-position mapping)
  __syncthreads();
  ilu::ring2_sweep<T, NT, false, WIDE, SKIP>(t, v, x, ring, mask);
}

template <typename T>
__global__ __launch_bounds__(kWgThreads) void k_apply_wg(Topo t, IluView<T> v, const double* r,
                                                          double* x, const int32_t* skip) {
  if (skip && *skip != 0) return;
  extern __shared__ unsigned char smem[];
  apply_levels_wg<T, kWgThreads>(t, v, r, x, reinterpret_cast<T*>(smem));
}

template <typename T>
size_t apply_lds(const opm_problem* pb) {
  return sizeof(T) * 2 * 3 * (size_t)pb->max_level;
}

size_t factor_lds(const opm_problem* pb) { return sizeof(double) * 2 * 9 * (size_t)pb->max_level; }

// one flag per (kernel, precision): slots 0-5 level-window kernels, 12-21
// (FP64) and 24-33 (FP32) ring sweeps, 34-39 block-ILU0 factorisation,
// 64-99 (FP64) and 100-135 (FP32) block-ILU0 sweeps (12 per fused mode),
// 136-153 (FP64) and 154-171 (FP32) those with level bounds in registers,
// 172-177 block-ILU0 factorisation with its loads spread over levels
bool g_lds_attr_set[178] = {};

// Dynamic LDS up to the 160 KB of a workgroup less the kernel's static LDS.
template <typename K>
int allow_lds(K kernel, int slot) {
  if (!g_lds_attr_set[slot]) {
    hipFuncAttributes at;
    OPM_TRY_HIP(hipFuncGetAttributes(&at, reinterpret_cast<const void*>(kernel)));
    OPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    160 * 1024 - (int)at.sharedSizeBytes));
    g_lds_attr_set[slot] = true;
  }
  return OPM_OK;
}

// Threads of a block-ILU0 factorisation workgroup (a row per thread) and of
// a sweep workgroup (16 rows per wavefront): the widest level of a
// subdomain rounded up to a wavefront, at most 256 (wider levels loop).
int block_threads(const opm_problem* pb) {
  return pb->max_width <= 64 ? 64 : pb->max_width <= 128 ? 128 : 256;
}
int block_sweep_threads(const opm_problem* pb) {
  const int waves = (pb->max_width + kRowsPerWave - 1) / kRowsPerWave;
  return waves <= 1 ? 64 : waves <= 2 ? 128 : 256;
}
bool block_sweep_wide(const opm_problem* pb) {
  return pb->max_width > block_sweep_threads(pb) / 64 * kRowsPerWave;
}

// The subdomain's vector (one row per slot and a zero row) and its level
// bounds.
template <typename T>
size_t block_lds(const opm_problem* pb) {
  return sizeof(T) * 3 * ((size_t)pb->max_sub + 1) + sizeof(int) * 2 * (size_t)pb->n_levels;
}

// ---------------------------------------------- plane-pipelined sweeps
// The ILU(0) of a system too large for one workgroup, on a Cartesian
// lattice: the rows of z-plane k on diagonal d = i + j form one contiguous
// range of the level schedule (level i + j + k lists its rows in natural
// order, so by plane), their lower neighbours are the same plane's diagonal
// d - 1 and plane k - 1's diagonal d.  One workgroup per plane walks its
// diagonals in order with the previous diagonal's results in an LDS ring;
// the values another plane reads go through a vector that is filled with a
// marker before the sweep (a signalling-NaN bit pattern, which no
// arithmetic result has), are written through to the device's coherence
// point and are read from there until they no longer hold the marker.  So a
// plane never waits for a whole step of its neighbour, only for the values
// it needs, and needs no counters, fences or completion waits.  The
// backward sweep mirrors the forward one downwards.  Workgroups are
// dispatched in index order and only wait on lower indices, so they cannot
// deadlock; the wait is bounded all the same, and a wait that gives up
// raises an abort word that every workgroup honours: the solve then returns
// NaN (the Krylov solver reports it) instead of hanging.  The row arithmetic
// is solve_row's, so the results equal the per-level launches' bit for bit.
constexpr int kPlaneThreads = 256;
typedef int int2v __attribute__((ext_vector_type(2)));

struct PlaneTab {
  int2v* rng;       // [nz][D] (first position, end position) of plane k on diagonal d
  int32_t* abort_w;
  void* xb;         // [3][ns] the backward sweep's results by position (T)
  int nx, ny, nz, D, W;
  unsigned spin;    // polls of a wait before it gives up (0: at once)
};

// The ILU(0) of the whole lattice only: with a block-ILU0 topology the
// positions go by (local level, subdomain, cell), so a plane's rows on one
// diagonal are not one contiguous range.
inline bool plane_capable(const opm_problem* pb) {
  return pb->n_sub == 0 && pb->box_cell && pb->cell_box && pb->nx > 0 && pb->ny > 0 &&
         pb->nz > 0 &&
         std::min(pb->nx, pb->ny) <= kPlaneThreads && pb->nz <= 4096 &&
         pb->nx + pb->ny - 1 <= 4096;
}
inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }
// sized for FP64 (the FP32 factors use half of the vector)
inline size_t plane_bytes(const opm_problem* pb) {
  if (!plane_capable(pb)) return 0;
  const size_t D = (size_t)pb->nx + pb->ny - 1;
  return al256(sizeof(int2v) * D * pb->nz) + 256 +
         al256(sizeof(double) * 3 * ilu_padded(pb->n_cells));
}
template <typename T>
PlaneTab plane_tab(const opm_problem* pb, void* ilu) {
  PlaneTab p;
  char* base = (char*)ilu + al256(view_bytes<T>(pb->n_cells));
  p.nx = pb->nx;
  p.ny = pb->ny;
  p.nz = pb->nz;
  p.D = pb->nx + pb->ny - 1;
  p.W = std::min(pb->nx, pb->ny);
  p.rng = (int2v*)base;
  base += al256(sizeof(int2v) * (size_t)p.D * p.nz);
  p.abort_w = (int32_t*)base;
  p.xb = base + 256;
  p.spin = (unsigned)g_plane_spin;
  return p;
}

__global__ __launch_bounds__(256) void k_plane_init(PlaneTab p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < p.D * p.nz) p.rng[e] = int2v{0x7fffffff, -1};
}

__global__ __launch_bounds__(256) void k_plane_fill(Topo t, const int32_t* cell_box, PlaneTab p) {
  const int pos = blockIdx.x * 256 + threadIdx.x;
  if (pos >= t.n) return;
  const int box = cell_box[t.perm[pos]];
  const int i = box % p.nx, j = (box / p.nx) % p.ny, k = box / (p.nx * p.ny);
  int* e = reinterpret_cast<int*>(p.rng + (size_t)k * p.D + i + j);
  atomicMin(e, pos);
  atomicMax(e + 1, pos + 1);
}

// the marker of a value not yet written (signalling NaNs: arithmetic
// returns quiet ones)
__device__ __forceinline__ void unset_value(double& v) {
  v = __builtin_bit_cast(double, 0x7FF4A5A5A5A5A5A5ull);
}
__device__ __forceinline__ void unset_value(float& v) { v = __builtin_bit_cast(float, 0x7FA5A5A5u); }
__device__ __forceinline__ bool is_unset(double v) {
  return __builtin_bit_cast(unsigned long long, v) == 0x7FF4A5A5A5A5A5A5ull;
}
__device__ __forceinline__ bool is_unset(float v) {
  return __builtin_bit_cast(unsigned, v) == 0x7FA5A5A5u;
}

// Before a pair of sweeps: both exchange vectors hold the marker, no abort.
template <typename T>
__global__ __launch_bounds__(256) void k_plane_reset(IluView<T> v, PlaneTab p,
                                                      const int32_t* skip) {
  if (skip && *skip != 0) return;
  T u;
  unset_value(u);
  const unsigned n = 3u * (unsigned)v.ns;
  T* xb = static_cast<T*>(p.xb);
  for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    v.z[e] = u;
    xb[e] = u;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *p.abort_w = 0;
}

__device__ __forceinline__ double coherent_load(const double* p) {
  return __builtin_bit_cast(double, __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ float coherent_load(const float* p) {
  return __builtin_bit_cast(float, __hip_atomic_load(reinterpret_cast<const unsigned*>(p),
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
// written through to the device's coherence point
__device__ __forceinline__ void coherent_store(double* p, double x) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, x),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coherent_store(float* p, float x) {
  __hip_atomic_store(reinterpret_cast<unsigned*>(p), __builtin_bit_cast(unsigned, x), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// The re-read of a value found not yet written (the slow path): the load and
// its wait in one block, so that the compiler counts no load of this loop
// among those in flight (a counted load here would make it wait for every
// prefetch issued since, at the next use of any of them).
__device__ __forceinline__ double coherent_reread(const double* p) {
  unsigned long long b;
  asm volatile("global_load_dwordx2 %0, %1, off sc1\n\ts_waitcnt vmcnt(0)" : "=v"(b) : "v"(p));
  return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ float coherent_reread(const float* p) {
  unsigned b;
  asm volatile("global_load_dword %0, %1, off sc1\n\ts_waitcnt vmcnt(0)" : "=v"(b) : "v"(p));
  return __builtin_bit_cast(float, b);
}

// A row of a plane step: its sweep data, and the value of its off-plane
// neighbour (loaded with the data; re-read at use while it holds the marker).
template <typename T>
struct PlaneJob {
  SweepJob<T> j;
  T xo[3];
  int ko;     // the off-plane neighbour's position (-1: none)
  int have;   // the lane has a row in this step
  int pos;
};

// FWD: plane k = blockIdx.x walks d = 0 .. D-1 and reads plane k - 1's
// forward results; backward: plane k = nz - 1 - blockIdx.x walks d = D-1 ..
// 0 and reads plane k + 1's backward results (every workgroup waits on a
// lower index).  The rows of steps s + 1 and s + 2 are in flight while step
// s is solved (a ring of three jobs, the loop unrolled over its period);
// every lane loads (lanes without a row at a valid position) so that the
// loads stay in straight-line code whose waits count only what they need.
template <typename T, bool FWD>
__global__ __launch_bounds__(kPlaneThreads) void k_sweep_planes(Topo t, IluView<T> v, PlaneTab p,
                                                                const double* r, double* x,
                                                                const int32_t* skip) {
  if (skip && *skip != 0) return;
  extern __shared__ unsigned char smem_planes[];
  T* ring = reinterpret_cast<T*>(smem_planes);                      // [2][W][3]
  int2v* rl = reinterpret_cast<int2v*>(ring + 2 * 3 * (size_t)p.W);   // [D] the plane's rows per step
  // fail[s % 3]: a lane of step s gave up.  Read by every wave after the
  // step's barrier; the slot of step s + 1 is cleared before it (no wave
  // still reads it: they all passed the barrier of step s - 1 after their
  // last read of step s - 2).
  __shared__ int fail[3];
  __shared__ int go;
  const int k = FWD ? (int)blockIdx.x : p.nz - 1 - (int)blockIdx.x;
  const unsigned ns = (unsigned)v.ns;
  const int tid = (int)threadIdx.x;
  // the vector the neighbouring planes exchange: forward results in z,
  // backward results in xb
  T* xch = FWD ? v.z : static_cast<T*>(p.xb);
  const int2v none = int2v{0, 0};
  for (int s = tid; s < p.D; s += kPlaneThreads) {
    int2v e = p.rng[(size_t)k * p.D + (FWD ? s : p.D - 1 - s)];
    // a diagonal of a plane holds at most W rows (the ring's capacity);
    // empty ranges are (INT_MAX, -1)
    if (e.x < e.y) e.y = min(e.y, e.x + p.W);
    rl[s] = e.x < e.y ? e : none;
  }
  if (tid == 0) {
    // a backward sweep after a forward sweep that gave up does not start
    go = FWD || __hip_atomic_load(p.abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    fail[0] = 0;
  }
  __syncthreads();
  if (go == 0) {
    // the forward sweep gave up: this plane's solution is NaN, not a stale value
    for (int s = 0; s < p.D; ++s)
      for (int q = rl[s].x + tid; q < rl[s].y; q += kPlaneThreads) {
        const int cell = t.perm[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) x[3 * cell + c] = __builtin_nan("");
      }
    return;
  }
  auto range = [&](int s) { return s < p.D ? rl[s] : none; };
  // rows rg of a step whose in-plane neighbours are the rows prg
  // the row's record (neighbour positions and cell; the blocks and D^{-1}
  // in 16-byte pieces, the values of the slot-major arrays): 25 vector
  // loads per row in FP64, 16 in FP32, so that two steps of rows stay
  // within the 63 loads a wave can have in flight
  typedef typename Vec16<T>::type V;
  constexpr unsigned kV = 16 / sizeof(T);
  const V* rec = reinterpret_cast<const V*>(FWD ? v.rec_f : v.rec_b);
  const int4v* idx = FWD ? v.idx_f : v.idx_b;
  auto fetch = [&](PlaneJob<T>& J, const int2v& rg, const int2v& prg) {
    const int cnt = rg.y - rg.x;
    J.have = tid < cnt;
    J.pos = J.have ? rg.x + tid : 0;
    const unsigned up = (unsigned)J.pos;
    SweepJob<T>& j = J.j;
    const int4v ix = idx[up];
#pragma unroll
    for (unsigned c = 0; c < (unsigned)kRecValues / kV; ++c) {
      const V w = rec[c * ns + up];
#pragma unroll
      for (unsigned l = 0; l < kV; ++l) {
        const unsigned e = c * kV + l;
        if (e < 27u)
          j.a[e] = w[l];
        else
          j.D[e - 27u] = w[l];
      }
    }
    if (!FWD) {
#pragma unroll
      for (unsigned c = 0; c < 3; ++c) j.rhs[c] = v.z[c * ns + up];
    }
    j.kp[0] = ix.x;
    j.kp[1] = ix.y;
    j.kp[2] = ix.z;
    j.cell = ix.w;
    // the off-plane neighbour: the one listed that is not on the previous
    // diagonal of this plane
    int ko = -1;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int kp = j.kp[q];
      ko = kp >= 0 && (kp < prg.x || kp >= prg.y) ? kp : ko;
    }
    J.ko = J.have ? ko : -1;
    const unsigned uo = (unsigned)max(J.ko, 0);
#pragma unroll
    for (unsigned c = 0; c < 3; ++c) J.xo[c] = coherent_load(xch + c * ns + uo);
    if (FWD) {
#pragma unroll
      for (unsigned c = 0; c < 3; ++c) j.rhs[c] = (T)r[3u * (unsigned)j.cell + c];
    }
  };
  PlaneJob<T> jobs[3];
  int2v rgs[3];
  rgs[0] = range(0);
  rgs[1] = range(1);
  rgs[2] = none;
  int2v prv = none;
  fetch(jobs[0], rgs[0], none);
  fetch(jobs[1], rgs[1], rgs[0]);
  // Step s, first part: its off-plane values (loaded with its rows two steps
  // ago), re-read into other registers while they hold the marker (bounded);
  // done before the rows of step s + 2 are requested, so that no later wait
  // for them covers those loads.
  auto check = [&](const PlaneJob<T>& J, int s, T* xo) {
    const bool unset = J.ko >= 0 && (is_unset(J.xo[0]) || is_unset(J.xo[1]) || is_unset(J.xo[2]));
    xo[0] = J.xo[0];
    xo[1] = J.xo[1];
    xo[2] = J.xo[2];
    bool gave_up = J.ko >= 0 && p.spin == 0;
    if (unset && !gave_up) {
      const unsigned uo = (unsigned)J.ko;
      for (unsigned it = 0;; ++it) {
        if (it == p.spin) {
          gave_up = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        T xr[3];
#pragma unroll
        for (unsigned c = 0; c < 3; ++c) xr[c] = coherent_reread(xch + c * ns + uo);
        if (!is_unset(xr[0]) && !is_unset(xr[1]) && !is_unset(xr[2])) {
          xo[0] = xr[0];
          xo[1] = xr[1];
          xo[2] = xr[2];
          break;
        }
        if ((it & 63) == 63 &&
            __hip_atomic_load(p.abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          gave_up = true;
          break;
        }
      }
    }
    if (gave_up) {
      __hip_atomic_store(p.abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      fail[s % 3] = 1;
    }
  };
  // Second part: the rows (every lane computes; a missing neighbour, or a
  // lane without a row, reads zeros: its blocks are zero, so each skipped
  // term adds an exact zero and the rows' results are solve_row's bits),
  // then the results to the ring and the exchange vector.
  auto solve = [&](const PlaneJob<T>& J, const T* xo, const int2v& rg, int s) {
    const SweepJob<T>& j = J.j;
    T acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = FWD ? j.rhs[c] : (T)0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int kp = j.kp[q];
      const int off = kp - prv.x;
      const bool in_ring = kp >= 0 && off >= 0 && kp < prv.y;
      const T* w = ring + (unsigned)(((s + 1) & 1) * p.W + (in_ring ? off : 0)) * 3u;
      T xv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) xv[c] = kp < 0 ? (T)0 : in_ring ? w[c] : xo[c];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T t = j.a[9 * q + 3 * a] * xv[0] + j.a[9 * q + 3 * a + 1] * xv[1] +
                    j.a[9 * q + 3 * a + 2] * xv[2];
        acc[a] = FWD ? acc[a] - t : acc[a] + t;
      }
    }
    T out[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T d = j.D[3 * a] * acc[0] + j.D[3 * a + 1] * acc[1] + j.D[3 * a + 2] * acc[2];
      out[a] = FWD ? d : j.rhs[a] - d;
    }
    if (J.have) {
      const unsigned pos = (unsigned)J.pos;
      T* w = ring + (unsigned)((s & 1) * p.W + (J.pos - rg.x)) * 3u;
#pragma unroll
      for (unsigned c = 0; c < 3; ++c) {
        w[c] = out[c];
        coherent_store(xch + c * ns + pos, out[c]);
        if (!FWD) x[3u * (unsigned)j.cell + c] = (double)out[c];
      }
    }
    if (tid == 0) fail[(s + 1) % 3] = 0;
    __syncthreads();
    prv = rg;
    return fail[s % 3] == 0;
  };
  bool ok = true;
  for (int s0 = 0; ok && s0 < p.D; s0 += 3) {
#pragma unroll
    for (int qq = 0; qq < 3; ++qq) {
      const int s = s0 + qq;
      if (s >= p.D) break;
      T xo[3];
      check(jobs[qq], s, xo);
      rgs[(qq + 2) % 3] = range(s + 2);
      fetch(jobs[(qq + 2) % 3], rgs[(qq + 2) % 3], rgs[(qq + 1) % 3]);
      if (!solve(jobs[qq], xo, rgs[qq], s)) {
        ok = false;
        break;
      }
    }
  }
  if (!FWD && !ok) {
    // a sweep that gave up: its plane's solution is NaN, not a stale value
    for (int s = 0; s < p.D; ++s)
      for (int q = rl[s].x + tid; q < rl[s].y; q += kPlaneThreads) {
        const int cell = t.perm[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) x[3 * cell + c] = __builtin_nan("");
      }
  }
}

// The pivot recursion pipelined over z-planes like the sweeps: plane k walks
// its diagonals, a row's lower neighbours being the previous diagonal of its
// plane (their D^{-1} in an LDS ring) and the same diagonal of plane k - 1,
// whose D^{-1} is read from dinv64 (filled with the marker beforehand,
// written through to the coherence point) until it no longer holds the
// marker.  The row arithmetic is finish_fac's: the per-level launches' bits.
// A wait that gives up raises the abort word and sets the status to OPM_EHIP.
// (the rows only: the padding past n keeps what the other launch shapes leave)
template <typename T>
__global__ __launch_bounds__(256) void k_plane_factor_reset(IluView<T> v, PlaneTab p, int n) {
  double u;
  unset_value(u);
  const unsigned ns = (unsigned)v.ns, total = 9u * ns;
  for (unsigned e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256)
    if (e % ns < (unsigned)n) v.dinv64[e] = u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *p.abort_w = 0;
}

template <typename T>
__global__ __launch_bounds__(kPlaneThreads) void k_factor_planes(Topo t, const double* J,
                                                                 IluView<T> v, PlaneTab p,
                                                                 int32_t* status) {
  extern __shared__ unsigned char smem_fplanes[];
  double* ring = reinterpret_cast<double*>(smem_fplanes);               // [2][W][9]
  int2v* rl = reinterpret_cast<int2v*>(ring + 2 * 9 * (size_t)p.W);   // [D]
  __shared__ int fail[3];
  const int k = (int)blockIdx.x;
  const int tid = (int)threadIdx.x;
  const unsigned ns = (unsigned)v.ns;
  const int2v none = int2v{0, 0};
  for (int s = tid; s < p.D; s += kPlaneThreads) {
    int2v e = p.rng[(size_t)k * p.D + s];
    if (e.x < e.y) e.y = min(e.y, e.x + p.W);
    rl[s] = e.x < e.y ? e : none;
  }
  if (tid == 0) fail[0] = 0;
  __syncthreads();
  int2v prv = none;
  for (int s = 0; s < p.D; ++s) {
    const int2v rg = rl[s];
    if (tid < rg.y - rg.x) {
      const int pos = rg.x + tid;
      FacJob j;
      load_fac(t, J, pos, j);
      double inv[9];
      bool gave_up = false;
      finish_fac<T>(j, pos, v,
                    [&](int kp, double* Dk) {
                      if (kp >= prv.x && kp < prv.y) {
                        const double* w = ring + (unsigned)(((s + 1) & 1) * p.W + (kp - prv.x)) * 9u;
#pragma unroll
                        for (int e = 0; e < 9; ++e) Dk[e] = w[e];
                        return;
                      }
                      for (unsigned it = 0;; ++it) {
                        bool ready = true;
#pragma unroll
                        for (unsigned e = 0; e < 9; ++e) {
                          Dk[e] = coherent_load(v.dinv64 + e * ns + (unsigned)kp);
                          ready = ready && !is_unset(Dk[e]);
                        }
                        if (ready) return;
                        if (it >= p.spin ||
                            ((it & 63) == 63 && __hip_atomic_load(p.abort_w, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                          gave_up = true;
#pragma unroll
                          for (int e = 0; e < 9; ++e) Dk[e] = 0.0;
                          return;
                        }
                        __builtin_amdgcn_s_sleep(1);
                      }
                    },
                    status, inv);
      double* w = ring + (unsigned)((s & 1) * p.W + tid) * 9u;
#pragma unroll
      for (unsigned e = 0; e < 9; ++e) {
        w[e] = inv[e];
        coherent_store(v.dinv64 + e * ns + (unsigned)pos, inv[e]);
      }
      if (gave_up) {
        __hip_atomic_store(p.abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (status) *status = OPM_EHIP;
        fail[s % 3] = 1;
      }
    }
    if (tid == 0) fail[(s + 1) % 3] = 0;
    __syncthreads();
    if (fail[s % 3] != 0) break;
    prv = rg;
  }
}

inline size_t factor_planes_lds(const PlaneTab& p) {
  return sizeof(double) * 2 * 9 * (size_t)p.W + sizeof(int2v) * (size_t)p.D;
}

template <typename T>
int factor_impl(const opm_problem* pb, const double* J, void* ilu, int32_t* status, int mode,
                hipStream_t s) {
  IluView<T> v = view<T>(pb, ilu);
  Topo t = topo_of(pb);
  if (mode == 2) {   // block ILU0: one workgroup per subdomain
    const size_t lds = sizeof(double) * 2 * 9 * (size_t)pb->max_width;
    // the recursion with its loads spread over three levels where a
    // subdomain has at most 64 levels
    const bool lvr = pb->n_levels <= 64;
    const int slot = (sizeof(T) == 8 ? 34 : 37) + (lvr ? 138 : 0);
#define OPM_FACTOR_BLOCKS(NT, SL)                                                              \
  do {                                                                                         \
    if (lvr) {                                                                                 \
      OPM_TRY(allow_lds(k_factor_blocks_pipe<T, NT>, slot + SL));                              \
      hipLaunchKernelGGL((k_factor_blocks_pipe<T, NT>), dim3(pb->n_sub), dim3(NT), lds, s, t,  \
                         J, v, pb->sub_level_ptr, pb->n_sub, pb->max_width, status);           \
    } else {                                                                                   \
      OPM_TRY(allow_lds(k_factor_blocks<T, NT>, slot + SL));                                   \
      hipLaunchKernelGGL((k_factor_blocks<T, NT>), dim3(pb->n_sub), dim3(NT), lds, s,          \
                         t, J, v, pb->sub_level_ptr, pb->n_sub, pb->max_width, status);        \
    }                                                                                          \
  } while (0)
    switch (block_threads(pb)) {
      case 64: OPM_FACTOR_BLOCKS(64, 0); break;
      case 128: OPM_FACTOR_BLOCKS(128, 1); break;
      default: OPM_FACTOR_BLOCKS(256, 2); break;
    }
#undef OPM_FACTOR_BLOCKS
    hipLaunchKernelGGL(k_pack_block_records<T>, dim3(blocks_for(pb->n_cells, kPackRows)),
                       dim3(256), 0, s, t, pb->row_ptr, J, v, pb->slot);
    OPM_TRY_HIP(hipGetLastError());
    return OPM_OK;
  }
  hipLaunchKernelGGL(k_pack<T>, dim3(blocks_for(pb->n_cells, kBlock)), dim3(kBlock), 0, s, t, J,
                     v);
  if (mode == 0) {
    if (pb->max_level <= kMaxFactorWindowRows) {
      OPM_TRY(allow_lds(k_factor_wg<T, true>, sizeof(T) == 8 ? 0 : 1));
      hipLaunchKernelGGL((k_factor_wg<T, true>), dim3(1), dim3(kFacThreads), factor_lds(pb), s, t,
                         J, v, status);
    } else {
      hipLaunchKernelGGL((k_factor_wg<T, false>), dim3(1), dim3(kFacThreads), 0, s, t, J, v,
                         status);
    }
    // the record sweep's copy of the factors (whenever a ring sweep can run)
    if (sizeof(T) * 3 * (size_t)ring_rows(pb->sweep_span, pb->max_level) <= kMaxRingBytes)
      hipLaunchKernelGGL(k_pack_records<T>, dim3(blocks_for(pb->n_cells, kBlock)), dim3(kBlock),
                         0, s, t, v);
    OPM_TRY_HIP(hipGetLastError());
    return OPM_OK;
  }
  if (plane_capable(pb)) {   // the plane table (of the pipelined factorisation and sweeps)
    const PlaneTab pt = plane_tab<T>(pb, ilu);
    hipLaunchKernelGGL(k_plane_init, dim3(blocks_for((long)pt.D * pt.nz, 256)), dim3(256), 0, s,
                       pt);
    hipLaunchKernelGGL(k_plane_fill, dim3(blocks_for(pb->n_cells, 256)), dim3(256), 0, s, t,
                       pb->cell_box, pt);
  }
  const bool planes = g_plane_sweep > 0 && plane_capable(pb) &&
                      factor_planes_lds(plane_tab<T>(pb, ilu)) <= 64 * 1024;
  if (planes) {
    const PlaneTab pt = plane_tab<T>(pb, ilu);
    hipLaunchKernelGGL(k_plane_factor_reset<T>, dim3(blocks_for(9 * (long)v.ns, 256 * 8)),
                       dim3(256), 0, s, v, pt, pb->n_cells);
    hipLaunchKernelGGL(k_factor_planes<T>, dim3(pt.nz), dim3(kPlaneThreads), factor_planes_lds(pt),
                       s, t, J, v, pt, status);
  } else {
    for (int l = 0; l < pb->n_levels; ++l) {
      const int p0 = pb->level_ptr_h[l], p1 = pb->level_ptr_h[l + 1];
      hipLaunchKernelGGL(k_factor_level<T>, dim3(blocks_for(p1 - p0, kBlock)), dim3(kBlock), 0,
                         s, t, J, v, p0, p1, status);
    }
  }
  if (plane_capable(pb))   // the row records of the sweeps
    hipLaunchKernelGGL(k_pack_records<T>, dim3(blocks_for(pb->n_cells, kBlock)), dim3(kBlock), 0,
                       s, t, v);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

// One workgroup per subdomain, both sweeps in one launch.
template <typename T, int MODE>
int apply_blocks(const opm_problem* pb, IluView<T> v, const double* r, double* x,
                 const int32_t* skip, const kry::Fused& f, hipStream_t s) {
  const size_t lds = block_lds<T>(pb);
  const int slot = (sizeof(T) == 8 ? 64 : 100) + 12 * MODE;
  // level bounds in registers where a subdomain has at most 64 levels
  const int rslot = (sizeof(T) == 8 ? 136 : 154) + 6 * MODE;
#define OPM_BLOCKS(NT, D, SL)                                                                     \
  do {                                                                                            \
    if (!block_sweep_wide(pb) && pb->n_levels <= 64) {                                            \
      OPM_TRY(allow_lds(k_apply_blocks<T, NT, false, D, MODE, true>, rslot + SL / 2));            \
      hipLaunchKernelGGL((k_apply_blocks<T, NT, false, D, MODE, true>), dim3(pb->n_sub),          \
                         dim3(NT), lds, s, v, pb->sub_level_ptr, pb->n_sub, pb->n_levels,         \
                         pb->max_sub, r, x, skip, f);                                             \
    } else if (!block_sweep_wide(pb)) {                                                           \
      OPM_TRY(allow_lds(k_apply_blocks<T, NT, false, D, MODE, false>, slot + SL));                \
      hipLaunchKernelGGL((k_apply_blocks<T, NT, false, D, MODE, false>), dim3(pb->n_sub),         \
                         dim3(NT), lds, s, v, pb->sub_level_ptr, pb->n_sub, pb->n_levels,         \
                         pb->max_sub, r, x, skip, f);                                             \
    } else {                                                                                      \
      OPM_TRY(allow_lds(k_apply_blocks<T, NT, true, D, MODE, false>, slot + SL + 1));             \
      hipLaunchKernelGGL((k_apply_blocks<T, NT, true, D, MODE, false>), dim3(pb->n_sub),          \
                         dim3(NT), lds, s, v, pb->sub_level_ptr, pb->n_sub, pb->n_levels,         \
                         pb->max_sub, r, x, skip, f);                                             \
    }                                                                                             \
  } while (0)
  // levels of data in flight: automatically two for the sweeps fused with
  // BiCGStab (at 9000 cells the Krylov time of 20 steps 68.7 -> 67.5 ms) and
  // for the others where the subdomains fill the GPU (256 or more: bound by
  // bandwidth, 64.0 against 66.6 us at 500k cells), else one (latency-bound:
  // 10.89 against 11.08 us at 9000 cells)
  const int depth = g_block_depth == 2 || (g_block_depth == 0 && (MODE != kry::kFuseNone ||
                                                                  pb->n_sub >= 256))
                        ? 2
                        : 1;
  switch (block_sweep_threads(pb) * 4 + depth) {
    case 64 * 4 + 1: OPM_BLOCKS(64, 1, 0); break;
    case 128 * 4 + 1: OPM_BLOCKS(128, 1, 2); break;
    case 256 * 4 + 1: OPM_BLOCKS(256, 1, 4); break;
    case 64 * 4 + 2: OPM_BLOCKS(64, 2, 6); break;
    case 128 * 4 + 2: OPM_BLOCKS(128, 2, 8); break;
    default: OPM_BLOCKS(256, 2, 10); break;
  }
#undef OPM_BLOCKS
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

template <typename T>
int apply_impl(const opm_problem* pb, void* ilu, const double* r, double* x, int mode,
               hipStream_t s, const int32_t* skip) {
  IluView<T> v = view<T>(pb, ilu);
  Topo t = topo_of(pb);
  if (mode == 2) return apply_blocks<T, kry::kFuseNone>(pb, v, r, x, skip, kry::Fused{}, s);
  if (mode == 0) {
    const int ring = ring_rows(pb->sweep_span, pb->max_level);
    const size_t ring_bytes = sizeof(T) * 3 * (size_t)ring;
    if (ring_bytes <= kMaxRingBytes) {   // every neighbour value in LDS
      // automatic: 512 threads with idle wavefronts skipping their loads
      // (measured fastest on the 9000-, 45000- and 108000-cell systems)
      const int kind = g_sweep_kernel == 0 ? 5 : g_sweep_kernel;
      if (kind == 1) {
        OPM_TRY(allow_lds(k_apply_ring<T>, sizeof(T) == 8 ? 4 : 5));
        hipLaunchKernelGGL(k_apply_ring<T>, dim3(1), dim3(kWgThreads), ring_bytes, s, t, v, r, x,
                           skip, (unsigned)(ring - 1));
        OPM_TRY_HIP(hipGetLastError());
        return OPM_OK;
      }
      hipLaunchKernelGGL(k_gather_rhs<T>, dim3(blocks_for(pb->n_cells, kBlock)), dim3(kBlock), 0,
                         s, pb->n_cells, pb->perm, v, r, skip);
      const unsigned mask = (unsigned)(ring - 1);
      const int slot = (sizeof(T) == 8 ? 8 : 20) + 2 * kind;
#define OPM_RING2(NT, SKIP)                                                                  \
  do {                                                                                       \
    if (pb->max_level <= NT) {                                                               \
      OPM_TRY(allow_lds(k_apply_ring2<T, NT, false, SKIP>, slot));                           \
      hipLaunchKernelGGL((k_apply_ring2<T, NT, false, SKIP>), dim3(1), dim3(NT), ring_bytes, \
                         s, t, v, x, skip, mask);                                            \
    } else {                                                                                 \
      OPM_TRY(allow_lds(k_apply_ring2<T, NT, true, SKIP>, slot + 1));                        \
      hipLaunchKernelGGL((k_apply_ring2<T, NT, true, SKIP>), dim3(1), dim3(NT), ring_bytes,  \
                         s, t, v, x, skip, mask);                                            \
    }                                                                                        \
  } while (0)
      switch (kind) {
        case 2: OPM_RING2(512, false); break;
        case 3: OPM_RING2(256, false); break;
        case 4: OPM_RING2(128, false); break;
        case 5: OPM_RING2(512, true); break;
        default: OPM_RING2(256, true); break;
      }
#undef OPM_RING2
      OPM_TRY_HIP(hipGetLastError());
      return OPM_OK;
    }
    OPM_TRY(allow_lds(k_apply_wg<T>, sizeof(T) == 8 ? 2 : 3));
    hipLaunchKernelGGL(k_apply_wg<T>, dim3(1), dim3(kWgThreads), apply_lds<T>(pb), s, t, v, r, x,
                       skip);
    OPM_TRY_HIP(hipGetLastError());
    return OPM_OK;
  }
  if (g_plane_sweep > 0 && plane_capable(pb)) {
    const PlaneTab pt = plane_tab<T>(pb, ilu);
    const size_t lds = sizeof(T) * 2 * 3 * (size_t)pt.W + sizeof(int2v) * (size_t)pt.D;
    hipLaunchKernelGGL(k_plane_reset<T>, dim3(blocks_for(3 * (long)v.ns, 256 * 8)), dim3(256), 0,
                       s, v, pt, skip);
    hipLaunchKernelGGL((k_sweep_planes<T, true>), dim3(pt.nz), dim3(kPlaneThreads), lds, s, t, v,
                       pt, r, x, skip);
    hipLaunchKernelGGL((k_sweep_planes<T, false>), dim3(pt.nz), dim3(kPlaneThreads), lds, s, t,
                       v, pt, r, x, skip);
    OPM_TRY_HIP(hipGetLastError());
    return OPM_OK;
  }
  for (int l = 0; l < pb->n_levels; ++l) {
    const int p0 = pb->level_ptr_h[l], p1 = pb->level_ptr_h[l + 1];
    hipLaunchKernelGGL(k_fwd_level<T>, dim3(blocks_for(p1 - p0, kBlock)), dim3(kBlock), 0, s, t,
                       v, p0, p1, r, skip);
  }
  for (int l = pb->n_levels - 1; l >= 0; --l) {
    const int p0 = pb->level_ptr_h[l], p1 = pb->level_ptr_h[l + 1];
    hipLaunchKernelGGL(k_bwd_level<T>, dim3(blocks_for(p1 - p0, kBlock)), dim3(kBlock), 0, s, t,
                       v, p0, p1, x, skip);
  }
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

}  // namespace

size_t ilu_bytes(const opm_problem* pb, int precision) {
  const size_t v = precision == OPM_PREC_MIXED ? view_bytes<float>(pb->n_cells)
                                               : view_bytes<double>(pb->n_cells);
  const size_t pl = plane_bytes(pb);
  return pl ? al256(v) + pl : v;
}

// Sweeps of mode 1 on a lattice: 1 plane-pipelined (default), 0 one launch
// per level (OPM_OPT_PLANE_SWEEP).
int g_plane_sweep = 1;
// Polls of a plane sweep's wait before it gives up (OPM_OPT_PLANE_SPIN).
int g_plane_spin = 1 << 18;

// Sweep shape: one workgroup when the widest level fits the LDS window and
// the system is small enough for one compute unit, else one launch per
// level; g_sweep_mode (set by opm_set_option) forces one of them.
int g_sweep_mode = -1;
// ring-sweep kernel of the one-workgroup shape: 0 automatic, 1 gather in the
// loads, 2-6 branch-free prefetch (512, 256, 128 threads; 512 and 256
// threads with idle wavefronts skipping their loads)
int g_sweep_kernel = 0;
// levels whose data the block-ILU0 sweeps keep in flight: 0 automatic, 1, 2
int g_block_depth = 0;

// A block-ILU0 topology runs one workgroup per subdomain whenever the
// subdomain's vector fits in LDS; modes 0 and 1 also serve it (same
// factors and sweeps, level by level over the whole system).
int sweep_mode(const opm_problem* pb, int precision) {
  if (g_sweep_mode == 0 || g_sweep_mode == 1) {
    if (g_sweep_mode == 0 && pb->max_level > kMaxWindowRows) return 1;
    return g_sweep_mode;
  }
  if (pb->n_sub > 0 && pb->sub_level_ptr && pb->slot &&
      (pb->n_sub > 1 || g_sweep_mode == 2) &&
      (precision == OPM_PREC_MIXED ? block_lds<float>(pb) : block_lds<double>(pb)) <=
          kMaxBlockLds)
    return 2;
  return pb->max_level <= kMaxWindowRows && pb->n_cells <= 200000 ? 0 : 1;
}

int ilu_factor(const opm_problem* pb, const double* J, void* ilu, int precision, int32_t* status,
               hipStream_t s) {
  const int mode = sweep_mode(pb, precision);
  if (precision == OPM_PREC_MIXED) return factor_impl<float>(pb, J, ilu, status, mode, s);
  return factor_impl<double>(pb, J, ilu, status, mode, s);
}

// Block-ILU0 solve whose forward right-hand side is a BiCGStab vector
// update (mode: kry::kFuseBegin or kry::kFuseS); only for sweep mode 2.
int ilu_apply_fused(const opm_problem* pb, void* ilu, int precision, int mode,
                    const kry::Fused& f, double* x, hipStream_t s) {
  if (precision == OPM_PREC_MIXED) {
    IluView<float> v = view<float>(pb, ilu);
    return mode == kry::kFuseBegin
               ? apply_blocks<float, kry::kFuseBegin>(pb, v, nullptr, x, nullptr, f, s)
               : apply_blocks<float, kry::kFuseS>(pb, v, nullptr, x, nullptr, f, s);
  }
  IluView<double> v = view<double>(pb, ilu);
  return mode == kry::kFuseBegin
             ? apply_blocks<double, kry::kFuseBegin>(pb, v, nullptr, x, nullptr, f, s)
             : apply_blocks<double, kry::kFuseS>(pb, v, nullptr, x, nullptr, f, s);
}

// skip (device, may be null): the sweeps return at once while *skip != 0.
int ilu_apply(const opm_problem* pb, void* ilu, int precision, const double* r, double* x,
              hipStream_t s, const int32_t* skip) {
  const int mode = sweep_mode(pb, precision);
  if (precision == OPM_PREC_MIXED) return apply_impl<float>(pb, ilu, r, x, mode, s, skip);
  return apply_impl<double>(pb, ilu, r, x, mode, s, skip);
}

}  // namespace opm
