// Learned Newton initial guess: a three-layer 3-D convolutional network
// (3x3x3 kernels, 16 channels, zero padding, ReLU after layers 1 and 2) maps
// the last two states, the log-permeability and the well terms of each cell
// to a predicted state change over one report step: the last change
// y_n - y_{n-1} (a skip connection, linear extrapolation) plus the network's
// correction of the saturations away from wells (the pressure keeps the
// extrapolation: an error of a few psi in the slightly compressible system
// raises the CNV far above the extrapolation's).  The paper always starts
// Newton from the previous state (sec. 2.3); here the prediction replaces
// that start only when its CNV is lower, and the convergence test is left
// as it is, so converged states do not depend on the network.
//
// Convolutions are implicit GEMMs on the BF16 matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): one wavefront owns 16
// consecutive box cells x 16 output channels and accumulates 14 products of
// 16x16x32, each reducing over the 16 input channels of two taps.
// Activations and their gradients are stored channels-last in BF16
// ([box cell][16], rounded to nearest even); weights exist as an FP32 master
// copy (updated by Adam) and as BF16 operand copies in the two layouts that
// the forward and backward-data products read.
#include <cmath>

#include "common.h"

namespace opm {

// y_guess = learned guess; if y_extrap is given it receives a pointer into
// the workspace holding the extrapolation alone (valid until the next call).
int guess_infer(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                const double* y_nm1, double* y_guess, void* work, hipStream_t s,
                const double** y_extrap = nullptr);
size_t guess_work_bytes(const opm_problem* pb, const opm_guess_net* net);

namespace {

constexpr int kCh = OPM_GUESS_CHANNELS;
constexpr int kTaps = 27;
constexpr int kLayerW = kTaps * kCh * kCh;        // W[27][cout][cin]
constexpr int kLayerParams = kLayerW + kCh;       // + bias[cout]
constexpr int kParams = 3 * kLayerParams;
constexpr int kChunk = 16;                        // tiles per wave in the weight gradient
constexpr int kReduceGroup = 32;                  // waves per stage-1 sum of the partials
static_assert(kParams == OPM_GUESS_PARAMS, "parameter count");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short short8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x32_bf16 (gfx950): D[16][16] += A[16][32] B[32][16] in
// FP32; lane l holds A[l % 16][k] and B[k][l % 16] for the eight k of lane
// group l / 16, and D[4 (l / 16) + r][l % 16].  A product sums over k, so
// any assignment of the (tap, channel) or cell pairs to k that A and B
// share gives the same sum.
__device__ __forceinline__ floatx4 mfma32(const short8& a, const short8& b, const floatx4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ unsigned short f2bf(float f) {   // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

struct Grid {
  int nx, ny, nz, nbox;
};

inline int tiles_of(const Grid& g) { return (g.nbox + 15) / 16; }
inline size_t al(size_t b) { return (b + 255) / 256 * 256; }
inline size_t act_bytes(const Grid& g) { return al(sizeof(unsigned short) * (size_t)tiles_of(g) * 16 * kCh); }
inline int waves_of(const Grid& g) { return (tiles_of(g) + kChunk - 1) / kChunk; }
inline int groups_of(const Grid& g) { return (waves_of(g) + kReduceGroup - 1) / kReduceGroup; }
// per-wave partials, then the stage-1 sums of groups of kReduceGroup waves
inline size_t partial_bytes(const Grid& g) {
  return al(sizeof(float) * (size_t)waves_of(g) * kLayerParams) +
         al(sizeof(float) * (size_t)groups_of(g) * kLayerParams);
}

// -------------------------------------------------------------- features
// Channel scales: pressures as (p - 4800 psi) / 1000 psi, saturations as
// they are, log10(k_h / 1 mD) - 2, injection rates per 10 m^3/day, the
// producer term log(1 + WI (p - p_bhp)^+ / 1 cP per 10 m^3/day).  Outputs:
// dp per 100 psi, ds_w and ds_g per 0.1 (comparable magnitudes in the loss).
constexpr double kPsi = 6894.757293168;
constexpr double kP0 = 4800.0 * kPsi;
constexpr double kPS = 1000.0 * kPsi;
constexpr double kQS = 86400.0 / 10.0;
constexpr double kMuRef = 1e-3;
constexpr double kDPS = 100.0 * kPsi;
constexpr double kDSS = 0.1;
constexpr double kMilliDarcy = 9.869233e-16;

// channels: 0-2 y_n, 3-5 the last change y_n - y_{n-1} (per 100 psi and
// per 0.1, so BF16 keeps it to 3 digits), 6 log-permeability, 7-9 injection
// of water, oil, gas, 10 producer term, 11-15 zero.  Inactive box cells stay 0.
__global__ __launch_bounds__(kBlock) void k_features(opm_problem pb, const int32_t* cell_box,
                                                      const double* yn, const double* ynm1,
                                                      const double* perm, unsigned short* feats) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= pb.n_cells) return;
  float f[kCh];
#pragma unroll
  for (int k = 0; k < kCh; ++k) f[k] = 0.f;
  const double p = yn[3 * c];
  f[0] = (float)((p - kP0) / kPS);
  f[1] = (float)yn[3 * c + 1];
  f[2] = (float)yn[3 * c + 2];
  f[3] = (float)((p - ynm1[3 * c]) / kDPS);
  f[4] = (float)((yn[3 * c + 1] - ynm1[3 * c + 1]) / kDSS);
  f[5] = (float)((yn[3 * c + 2] - ynm1[3 * c + 2]) / kDSS);
  f[6] = (float)(log10(perm[c] / kMilliDarcy) - 2.0);
  double inj[3] = {0.0, 0.0, 0.0}, prod = 0.0;
  for (int t = pb.cell_conn_ptr[c]; t < pb.cell_conn_ptr[c + 1]; ++t) {
    const int k = pb.cell_conn[t];
    if (pb.conn_kind[k] == OPM_WELL_RATE_INJ) {
      const int ph = pb.conn_phase[k];
#pragma unroll
      for (int a = 0; a < 3; ++a)   // conn_rate is an outflux: negative for injection
        if (a == ph) inj[a] -= pb.conn_rate[k];
    } else {
      const double dd = p - pb.conn_bhp[k];
      if (dd > 0.0) prod += pb.conn_wi[k] * dd;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) f[7 + a] = (float)(inj[a] * kQS);
  f[10] = (float)log1p(prod / kMuRef * kQS);
  unsigned short* o = feats + (size_t)cell_box[c] * kCh;
#pragma unroll
  for (int k = 0; k < kCh; ++k) o[k] = f2bf(f[k]);
}

__global__ __launch_bounds__(kBlock) void k_zero_u16(unsigned short* p, size_t count) {
  for (size_t k = blockIdx.x * (size_t)kBlock + threadIdx.x; k < count;
       k += (size_t)gridDim.x * kBlock)
    p[k] = 0;
}

// A box cell is near a well when it or one of its 26 box neighbours carries a
// non-zero well channel (7-10) in the feature box: the learned correction is
// neither trained nor applied there.
__device__ __forceinline__ bool near_well(const Grid& g, const unsigned short* feats, int b) {
  const int i = b % g.nx, j = (b / g.nx) % g.ny, k = b / (g.nx * g.ny);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int ii = i + dx, jj = j + dy, kk = k + dz;
        if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) continue;
        const unsigned short* f = feats + (size_t)(ii + g.nx * (jj + g.ny * kk)) * kCh;
        // +0 and -0 both count as zero
        if ((f[7] | f[8] | f[9] | f[10]) & 0x7fffu) return true;
      }
  return false;
}

// ---------------------------------------------------- convolution (MFMA)
// Tap t covers the offset (t % 3 - 1, t / 3 % 3 - 1, t / 9 - 1) in (x, y, z).
//
// conv_tile: one 16x16x32 product per pair of taps: A rows are the 16 cells
// of the tile, A columns the 16 input channels of the cell at each of the
// two tap offsets (mirrored when FLIP); B the two taps' weights wt[t] as
// [n][k] rows of 16.  Lane group kb takes tap t + kb / 2 and channels
// 8 (kb % 2) .. + 7 in both operands; the 27th tap pairs with zeros.
template <bool FLIP>
__device__ __forceinline__ floatx4 conv_tile(const Grid& g, const unsigned short* in,
                                             const unsigned short* wt, int tile, int lane) {
  const int m = lane & 15, kb = lane >> 4;
  const int half = kb >> 1, c8 = (kb & 1) * 8;
  const int cell = tile * 16 + m;
  const bool valid = cell < g.nbox;
  const int ci = cell % g.nx, cj = (cell / g.nx) % g.ny, ck = cell / (g.nx * g.ny);
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t2 = 0; t2 < kTaps; t2 += 2) {
    const int t = t2 + half;
    int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    if (FLIP) {
      dx = -dx;
      dy = -dy;
      dz = -dz;
    }
    const int ii = ci + dx, jj = cj + dy, kk = ck + dz;
    short8 a = {0, 0, 0, 0, 0, 0, 0, 0};
    short8 b = {0, 0, 0, 0, 0, 0, 0, 0};
    if (t < kTaps) {
      if (valid && ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz) {
        const unsigned nb = (unsigned)(ii + g.nx * (jj + g.ny * kk));
        a = *reinterpret_cast<const short8*>(in + nb * kCh + c8);
      }
      b = *reinterpret_cast<const short8*>(wt + (t * kCh + m) * kCh + c8);
    }
    acc = mfma32(a, b, acc);
  }
  return acc;
}

// out = conv(in) + bias, then ReLU and BF16 (RELU) or FP32 as it is.
template <bool RELU>
__global__ __launch_bounds__(256) void k_conv_fwd(Grid g, const unsigned short* in,
                                                  const unsigned short* wt, const float* bias,
                                                  unsigned short* out_bf, float* out_f,
                                                  int ntiles) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;   // whole wavefront: MFMA needs all lanes
  const floatx4 acc = conv_tile<false>(g, in, wt, tile, lane);
  const int ch = lane & 15;
  const float b = bias[ch];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int cell = tile * 16 + 4 * (lane >> 4) + r;
    if (cell >= g.nbox) continue;
    const float v = acc[r] + b;
    if (RELU)
      out_bf[(size_t)cell * kCh + ch] = f2bf(v > 0.f ? v : 0.f);
    else
      out_f[(size_t)cell * kCh + ch] = v;
  }
}

// d_in = conv^T(d_out), masked by the ReLU of the layer input (act_in > 0).
__global__ __launch_bounds__(256) void k_conv_bwd_data(Grid g, const unsigned short* dout,
                                                       const unsigned short* wtb,
                                                       const unsigned short* act_in,
                                                       unsigned short* din, int ntiles) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;
  const floatx4 acc = conv_tile<true>(g, dout, wtb, tile, lane);
  const int ch = lane & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int cell = tile * 16 + 4 * (lane >> 4) + r;
    if (cell >= g.nbox) continue;
    const float a = bf2f(act_in[(size_t)cell * kCh + ch]);
    din[(size_t)cell * kCh + ch] = f2bf(a > 0.f ? acc[r] : 0.f);
  }
}

// Weight-gradient partials of one wave over kChunk tiles:
// dW[t][cout][cin] = sum_cells in[cell + off_t][cin] d_out[cell][cout] as
// 16x16x32 products whose reduction runs over 32 cells, two tiles (A =
// in^T with rows cin, B = d_out with columns cout; lane group kb takes
// cells 8 kb .. 8 kb + 7 of the pair in both operands); bias[cout] =
// sum_cells d_out[cell][cout].  Tile pairs are the outer loop: a lane's
// eight cells and their d_out values are found once per pair and the 27 tap
// accumulators stay in registers.
__global__ __launch_bounds__(256) void k_conv_bwd_weight(Grid g, const unsigned short* in,
                                                         const unsigned short* dout, int ntiles,
                                                         float* partials) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int t0 = wave * kChunk;
  if (t0 >= ntiles) return;   // whole wavefront: MFMA needs all lanes
  const int t1 = min(t0 + kChunk, ntiles);
  const int m = lane & 15, kb = lane >> 4;
  floatx4 acc[kTaps];
#pragma unroll
  for (int t = 0; t < kTaps; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int tile = t0; tile < t1; tile += 2) {
    int ci[8], cj[8], ck[8];
    bool ok[8];
    short8 b = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int cell = tile * 16 + 8 * kb + r;
      ok[r] = cell < g.nbox && cell < t1 * 16;
      const int c = ok[r] ? cell : 0;
      ci[r] = c % g.nx;
      cj[r] = (c / g.nx) % g.ny;
      ck[r] = c / (g.nx * g.ny);
      const unsigned short dv = ok[r] ? dout[(unsigned)c * kCh + m] : (unsigned short)0;
      b[r] = (short)dv;
      bsum += bf2f(dv);
    }
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
      short8 a = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int ii = ci[r] + dx, jj = cj[r] + dy, kk = ck[r] + dz;
        if (ok[r] && ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz)
          a[r] = (short)in[(unsigned)(ii + g.nx * (jj + g.ny * kk)) * kCh + m];
      }
      acc[t] = mfma32(a, b, acc[t]);
    }
  }
  float* P = partials + (size_t)wave * kLayerParams;
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) P[(t * kCh + m) * kCh + 4 * kb + r] = acc[t][r];
  // lanes m, m+16, m+32, m+48 hold the four cell groups of channel m
  bsum += __shfl_xor(bsum, 16, 64);
  bsum += __shfl_xor(bsum, 32, 64);
  if (kb == 0) P[kLayerW + m] = bsum;
}

// Sum of the per-wave partials in two fixed-order stages: stage 1 adds
// groups of kReduceGroup waves (grid: parameter blocks x groups), stage 2
// adds the groups (deterministic).

__global__ __launch_bounds__(256) void k_reduce_stage1(const float* partials, int nwaves,
                                                       float* stage) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kLayerParams) return;
  const int w0 = blockIdx.y * kReduceGroup, w1 = min(w0 + kReduceGroup, nwaves);
  float s = 0.f;
  for (int w = w0; w < w1; ++w) s += partials[(size_t)w * kLayerParams + e];
  stage[(size_t)blockIdx.y * kLayerParams + e] = s;
}

__global__ __launch_bounds__(256) void k_reduce_partials(const float* stage, int ngroups,
                                                         float* grad) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kLayerParams) return;
  float s = 0.f;
  for (int gr = 0; gr < ngroups; ++gr) s += stage[(size_t)gr * kLayerParams + e];
  grad[e] = s;
}

// -------------------------------------------------------------- training
// Squared error of the two saturation outputs against the scaled correction
// of the step to the extrapolated one, (y_next - y_n) - (y_n - y_{n-1})
// (ds / 0.1), summed over active cells away from wells and divided by
// 2 n_cells; d_out = dL/d out in BF16 (channels 1-2; channel 0, the unused
// pressure output, and cells near wells get zero).
__global__ __launch_bounds__(kBlock) void k_loss(Grid g, int n, const int32_t* cell_box,
                                                 const unsigned short* feats, const float* out,
                                                 const double* yn, const double* ynm1,
                                                 const double* ynext, unsigned short* dout,
                                                 double* partials) {
  __shared__ double sh[kBlock / kWave];
  const int c = blockIdx.x * kBlock + threadIdx.x;
  double se = 0.0;
  if (c < n && !near_well(g, feats, cell_box[c])) {
    const size_t b = (size_t)cell_box[c];
    double tgt[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      tgt[k] = ((ynext[3 * c + k] - yn[3 * c + k]) - (yn[3 * c + k] - ynm1[3 * c + k])) /
               (k == 0 ? kDPS : kDSS);
    dout[b * kCh] = 0;   // the pressure output is neither trained nor used
#pragma unroll
    for (int k = 1; k < 3; ++k) {
      const double e = (double)out[b * kCh + k] - tgt[k];
      se += e * e;
      dout[b * kCh + k] = f2bf((float)(2.0 * e / (2.0 * n)));
    }
  }
  const double s = block_sum<kBlock>(se, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_loss_final(const double* partials, int nblk, int n,
                                                       double* loss) {
  __shared__ double sh[kBlock / kWave];
  double v = 0.0;
  for (int k = threadIdx.x; k < nblk; k += kBlock) v += partials[k];
  v = block_sum<kBlock>(v, sh);
  if (threadIdx.x == 0) *loss = v / (2.0 * n);
}

// Adam (Kingma and Ba) on the FP32 master parameters; step is 1-based.
__global__ __launch_bounds__(256) void k_adam(float* w, const float* grad, float* m1, float* m2,
                                              int count, float lr, float b1, float b2, float eps,
                                              int step) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const float gr = grad[e];
  const float a = b1 * m1[e] + (1.f - b1) * gr;
  const float b = b2 * m2[e] + (1.f - b2) * gr * gr;
  m1[e] = a;
  m2[e] = b;
  const float ah = a / (1.f - powf(b1, (float)step));
  const float bh = b / (1.f - powf(b2, (float)step));
  w[e] -= lr * ah / (sqrtf(bh) + eps);
}

// BF16 operand copies of the master weights: forward wf[l][t][cout][cin],
// backward-data wb[l][t][cin][cout].
__global__ __launch_bounds__(256) void k_pack_weights(const float* master, unsigned short* wf,
                                                      unsigned short* wb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= 3 * kLayerW) return;
  const int layer = e / kLayerW, r = e % kLayerW;
  const int t = r / (kCh * kCh), co = (r / kCh) % kCh, ci = r % kCh;
  const unsigned short v = f2bf(master[(size_t)layer * kLayerParams + r]);
  wf[(size_t)layer * kLayerW + r] = v;
  wb[(size_t)layer * kLayerW + (t * kCh + ci) * kCh + co] = v;
}

// y_guess = y_n + (y_n - y_{n-1}) + the correction of the two saturations
// (the skip connection is applied in FP64; the pressure keeps the
// extrapolation, output 0 is unused); the correction is used only away from
// wells and only if all three outputs are finite, and not at all when out is
// null (the extrapolation alone); saturations clamped to [0, 1] with
// s_w + s_g <= 1 (s_g reduced first).
__global__ __launch_bounds__(kBlock) void k_guess_apply(Grid g, int n, const int32_t* cell_box,
                                                        const unsigned short* feats,
                                                        const double* yn, const double* ynm1,
                                                        const float* out, double* yg) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  const size_t b = (size_t)cell_box[c];
  float o0 = 0.f, o1 = 0.f, o2 = 0.f;
  bool ok = false;
  if (out) {
    o0 = out[b * kCh];
    o1 = out[b * kCh + 1];
    o2 = out[b * kCh + 2];
    ok = isfinite(o0) && isfinite(o1) && isfinite(o2) && !near_well(g, feats, (int)b);
  }
  const double p = yn[3 * c] + (yn[3 * c] - ynm1[3 * c]);
  double sw = yn[3 * c + 1] + (yn[3 * c + 1] - ynm1[3 * c + 1]) + (ok ? kDSS * (double)o1 : 0.0);
  double sg = yn[3 * c + 2] + (yn[3 * c + 2] - ynm1[3 * c + 2]) + (ok ? kDSS * (double)o2 : 0.0);
  sw = fmin(fmax(sw, 0.0), 1.0);
  sg = fmin(fmax(sg, 0.0), 1.0);
  if (sw + sg > 1.0) sg = 1.0 - sw;
  yg[3 * c] = p;
  yg[3 * c + 1] = sw;
  yg[3 * c + 2] = sg;
}

// ------------------------------------------------------------ host side
bool valid_grid(int nx, int ny, int nz) {
  return nx > 0 && ny > 0 && nz > 0 && (long)nx * ny * nz * kCh < (1L << 31);
}

void conv_launch(const Grid& g, const unsigned short* in, const unsigned short* wf,
                 const float* bias, bool relu, unsigned short* out_bf, float* out_f,
                 hipStream_t s) {
  const int nt = tiles_of(g);
  if (relu)
    hipLaunchKernelGGL(k_conv_fwd<true>, dim3((nt + 3) / 4), dim3(256), 0, s, g, in, wf, bias,
                       out_bf, nullptr, nt);
  else
    hipLaunchKernelGGL(k_conv_fwd<false>, dim3((nt + 3) / 4), dim3(256), 0, s, g, in, wf, bias,
                       nullptr, out_f, nt);
}

void backward_launch(const Grid& g, const unsigned short* in, const unsigned short* dout,
                     const unsigned short* wb, const unsigned short* act_in, unsigned short* din,
                     float* grad, float* partials, hipStream_t s) {
  const int nt = tiles_of(g), nw = waves_of(g), ng = groups_of(g);
  float* stage = partials + al(sizeof(float) * (size_t)nw * kLayerParams) / sizeof(float);
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3((nw + 3) / 4), dim3(256), 0, s, g, in, dout, nt,
                     partials);
  hipLaunchKernelGGL(k_reduce_stage1, dim3((kLayerParams + 255) / 256, ng), dim3(256), 0, s,
                     partials, nw, stage);
  hipLaunchKernelGGL(k_reduce_partials, dim3((kLayerParams + 255) / 256), dim3(256), 0, s, stage,
                     ng, grad);
  if (din)
    hipLaunchKernelGGL(k_conv_bwd_data, dim3((nt + 3) / 4), dim3(256), 0, s, g, dout, wb, act_in,
                       din, nt);
}

// Workspace of infer / train: activations a0 (features), a1, a2, output,
// gradients d3, d2, d1, weight partials, gradient, loss partials, guess.
struct Bufs {
  unsigned short *a0, *a1, *a2, *d3, *d2, *d1;
  float* out;
  float* partials;
  float* grad;
  double* lpart;
  double* yg;
};

size_t bufs_bytes(const Grid& g, int n) {
  return 6 * act_bytes(g) + al(sizeof(float) * (size_t)tiles_of(g) * 16 * kCh) +
         partial_bytes(g) + al(sizeof(float) * kParams) +
         al(sizeof(double) * (blocks_for(n, kBlock) + 1)) + al(sizeof(double) * 3 * (size_t)n);
}

Bufs carve(const Grid& g, int n, void* work) {
  char* c = (char*)work;
  Bufs b;
  unsigned short** acts[6] = {&b.a0, &b.a1, &b.a2, &b.d3, &b.d2, &b.d1};
  for (auto* p : acts) {
    *p = (unsigned short*)c;
    c += act_bytes(g);
  }
  b.out = (float*)c;
  c += al(sizeof(float) * (size_t)tiles_of(g) * 16 * kCh);
  b.partials = (float*)c;
  c += partial_bytes(g);
  b.grad = (float*)c;
  c += al(sizeof(float) * kParams);
  b.lpart = (double*)c;
  c += al(sizeof(double) * (blocks_for(n, kBlock) + 1));
  b.yg = (double*)c;
  return b;
}

bool valid_net(const opm_problem* pb, const opm_guess_net* net) {
  return pb && net && pb->n_cells > 0 && valid_grid(net->nx, net->ny, net->nz) &&
         pb->n_cells <= net->nx * net->ny * net->nz && net->cell_box && net->perm_h &&
         net->master && net->wbf16 && pb->cell_conn_ptr &&
         (pb->n_conns == 0 || (pb->cell_conn && pb->conn_kind && pb->conn_phase &&
                               pb->conn_wi && pb->conn_rate && pb->conn_bhp));
}

int features(const opm_problem* pb, const opm_guess_net* net, const Grid& g, const double* yn,
             const double* ynm1, unsigned short* a0, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u16, dim3(256), dim3(kBlock), 0, s, a0,
                     (size_t)tiles_of(g) * 16 * kCh);
  hipLaunchKernelGGL(k_features, dim3(blocks_for(pb->n_cells, kBlock)), dim3(kBlock), 0, s, *pb,
                     net->cell_box, yn, ynm1, net->perm_h, a0);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

void forward(const Grid& g, const opm_guess_net* net, const Bufs& b, hipStream_t s) {
  const unsigned short* wf = (const unsigned short*)net->wbf16;
  const float* m = net->master;
  conv_launch(g, b.a0, wf, m + kLayerW, true, b.a1, nullptr, s);
  conv_launch(g, b.a1, wf + kLayerW, m + kLayerParams + kLayerW, true, b.a2, nullptr, s);
  conv_launch(g, b.a2, wf + 2 * kLayerW, m + 2 * kLayerParams + kLayerW, false, nullptr, b.out,
              s);
}

}  // namespace

size_t guess_work_bytes(const opm_problem* pb, const opm_guess_net* net) {
  Grid g{net->nx, net->ny, net->nz, net->nx * net->ny * net->nz};
  return bufs_bytes(g, pb->n_cells);
}

int guess_infer(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                const double* y_nm1, double* y_guess, void* work, hipStream_t s,
                const double** y_extrap) {
  Grid g{net->nx, net->ny, net->nz, net->nx * net->ny * net->nz};
  Bufs b = carve(g, pb->n_cells, work);
  OPM_TRY(features(pb, net, g, y_n, y_nm1, b.a0, s));
  forward(g, net, b, s);
  const int blocks = blocks_for(pb->n_cells, kBlock);
  hipLaunchKernelGGL(k_guess_apply, dim3(blocks), dim3(kBlock), 0, s, g, pb->n_cells,
                     net->cell_box, b.a0, y_n, y_nm1, b.out, y_guess);
  if (y_extrap) {   // the skip path alone, into the workspace
    hipLaunchKernelGGL(k_guess_apply, dim3(blocks), dim3(kBlock), 0, s, g, pb->n_cells,
                       net->cell_box, b.a0, y_n, y_nm1, (const float*)nullptr, b.yg);
    *y_extrap = b.yg;
  }
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

}  // namespace opm

using namespace opm;

extern "C" {

size_t opm_guess_conv_backward_bytes(int32_t nx, int32_t ny, int32_t nz) {
  if (!valid_grid(nx, ny, nz)) return 0;
  return partial_bytes(Grid{nx, ny, nz, nx * ny * nz});
}

int opm_guess_pack_weights(const float* master, void* wbf16, void* stream) {
  if (!master || !wbf16) return OPM_EINVAL;
  unsigned short* wf = (unsigned short*)wbf16;
  hipLaunchKernelGGL(k_pack_weights, dim3((3 * kLayerW + 255) / 256), dim3(256), 0,
                     as_stream(stream), master, wf, wf + 3 * kLayerW);
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int opm_guess_conv(int32_t nx, int32_t ny, int32_t nz, const void* in, const void* w_fwd,
                   const float* bias, int32_t relu, void* out_bf16, float* out_f32,
                   void* stream) {
  if (!valid_grid(nx, ny, nz) || !in || !w_fwd || !bias || (relu ? !out_bf16 : !out_f32))
    return OPM_EINVAL;
  Grid g{nx, ny, nz, nx * ny * nz};
  conv_launch(g, (const unsigned short*)in, (const unsigned short*)w_fwd, bias, relu != 0,
              (unsigned short*)out_bf16, out_f32, as_stream(stream));
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

int opm_guess_conv_backward(int32_t nx, int32_t ny, int32_t nz, const void* in, const void* dout,
                            const void* w_bwd, const void* act_in, void* din, float* grad,
                            void* work, size_t work_bytes, void* stream) {
  if (!valid_grid(nx, ny, nz) || !in || !dout || !grad || !work) return OPM_EINVAL;
  if (din && (!w_bwd || !act_in)) return OPM_EINVAL;
  Grid g{nx, ny, nz, nx * ny * nz};
  if (work_bytes < partial_bytes(g)) return OPM_EINVAL;
  backward_launch(g, (const unsigned short*)in, (const unsigned short*)dout,
                  (const unsigned short*)w_bwd, (const unsigned short*)act_in,
                  (unsigned short*)din, grad, (float*)work, as_stream(stream));
  OPM_TRY_HIP(hipGetLastError());
  return OPM_OK;
}

size_t opm_guess_work_bytes(const opm_problem* pb, const opm_guess_net* net) {
  if (!valid_net(pb, net)) return 0;
  return guess_work_bytes(pb, net);
}

int opm_guess_features(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                       const double* y_nm1, void* feats, void* stream) {
  if (!valid_net(pb, net) || !y_n || !y_nm1 || !feats) return OPM_EINVAL;
  Grid g{net->nx, net->ny, net->nz, net->nx * net->ny * net->nz};
  return features(pb, net, g, y_n, y_nm1, (unsigned short*)feats, as_stream(stream));
}

int opm_guess_infer(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                    const double* y_nm1, double* y_guess, void* work, void* stream) {
  if (!valid_net(pb, net) || !y_n || !y_nm1 || !y_guess || !work) return OPM_EINVAL;
  return guess_infer(pb, net, y_n, y_nm1, y_guess, work, as_stream(stream));
}

int opm_guess_train_step(const opm_problem* pb, const opm_guess_net* net, const double* y_n,
                         const double* y_nm1, const double* y_next, float* adam_m, float* adam_v,
                         int32_t step, float lr, double* loss, void* work, void* stream) {
  if (!valid_net(pb, net) || !y_n || !y_nm1 || !y_next || !adam_m || !adam_v || step < 1 ||
      !(lr > 0.f) || !loss || !work)
    return OPM_EINVAL;
  hipStream_t s = as_stream(stream);
  Grid g{net->nx, net->ny, net->nz, net->nx * net->ny * net->nz};
  Bufs b = carve(g, pb->n_cells, work);
  const unsigned short* wb = (const unsigned short*)net->wbf16 + 3 * kLayerW;
  OPM_TRY(features(pb, net, g, y_n, y_nm1, b.a0, s));
  forward(g, net, b, s);
  hipLaunchKernelGGL(k_zero_u16, dim3(256), dim3(kBlock), 0, s, b.d3,
                     (size_t)tiles_of(g) * 16 * kCh);
  const int nblk = blocks_for(pb->n_cells, kBlock);
  hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(kBlock), 0, s, g, pb->n_cells, net->cell_box, b.a0,
                     b.out, y_n, y_nm1, y_next, b.d3, b.lpart);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kBlock), 0, s, b.lpart, nblk, pb->n_cells, loss);
  const unsigned short* layer_in[3] = {b.a0, b.a1, b.a2};
  unsigned short* layer_d[3] = {b.d1, b.d2, b.d3};
  for (int l = 2; l >= 0; --l)
    backward_launch(g, layer_in[l], layer_d[l], wb + (size_t)l * kLayerW, layer_in[l],
                    l > 0 ? layer_d[l - 1] : nullptr, b.grad + (size_t)l * kLayerParams,
                    b.partials, s);
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, net->master, b.grad,
                     adam_m, adam_v, kParams, lr, 0.9f, 0.999f, 1e-8f, step);
  OPM_TRY_HIP(hipGetLastError());
  return opm_guess_pack_weights(net->master, net->wbf16, stream);
}

}  // extern "C"
