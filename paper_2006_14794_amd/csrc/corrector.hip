// Learned corrector: maps the dyadic-order-0 solve of a pair to its order-3
// terminal value (the network is this library's own; the paper has none).
//
//   features   one wave per pair runs the order-0 explicit scheme of Section
//              3.1 (eq. (explicit_finite_diff) with lambda = 0) and reduces
//              every 4 x 4 block of coarse cells to eight moments of the
//              grid on the fly: the grid itself never reaches memory.
//   conv       3 x 3 / stride 2 / pad 1 layers on the matrix cores
//              (v_mfma_f32_32x32x16_bf16: bf16 weights and activations,
//              float32 accumulation), bias and ReLU fused; NHWC bf16
//              activations (every consumer reads them as bf16).
//   fused      inference: one workgroup per pair runs all four layers and
//              the head with the feature map, layer 1's output and each
//              layer's weights in LDS.
//   backward   float32 VALU: input gradients by gathering the (at most four)
//              taps that reach an input pixel, weight gradients as
//              per-workgroup partial sums over LDS-staged positions reduced
//              in a fixed order (deterministic).
//   head       dense 512 -> 2; loss, Adam, channel statistics, and the
//              fallback decision with device-side compaction of the pairs
//              that need the plain order-3 solve.
#include <hip/hip_bf16.h>
#include <math.h>

#include "corrector.h"
#include "sweep_fwd_kernel.h"

namespace sk {
namespace corr {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
using bf16 = __bf16;

// ---------------------------------------------------------------- features --
template <int D>
__global__ __launch_bounds__(256) void features_kernel(const FeatArgs a) {
  constexpr int DP = (D + 3) & ~3;
  const int lane = threadIdx.x & 63;
  const int64_t pair = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (pair >= a.npairs) return;  // uniform per wave
  const int m = a.m, n = a.n;
  bf16* __restrict__ fo = a.feats + pair * (int64_t)kFeatFloats;
  float mu[kFeatChannels], rs[kFeatChannels];
#pragma unroll
  for (int c = 0; c < kFeatChannels; ++c) {
    mu[c] = a.norm ? a.norm[c] : 0.0f;
    rs[c] = a.norm ? a.norm[kFeatChannels + c] : 1.0f;
  }
  // block (P, Q) of this lane's strip: moments f[0..5] plus coordinates,
  // normalised in float32 and stored as eight bf16 (16 bytes).  The
  // coordinates P / 63 and Q / 63 (P, Q in 0 .. 63) are the correctly rounded
  // float quotients, formed as one double product with 1/63 rounded once to
  // float: the binary expansion of a multiple of 1/63 repeats 000001, so it is
  // never within the product's error of a float rounding midpoint (checked
  // for all 64 values against the float division).
  auto coord = [](int P) { return (float)((double)P * (1.0 / 63.0)); };
  auto put = [&](int P, int Q, const float (&f)[6]) {
    const float v[kFeatChannels] = {f[0], f[1], f[2], f[3], f[4], f[5], coord(P), coord(Q)};
    bf16x8 o;
#pragma unroll
    for (int c = 0; c < kFeatChannels; ++c) o[c] = (bf16)((v[c] - mu[c]) * rs[c]);
    *reinterpret_cast<bf16x8*>(fo + ((int64_t)P * kBlocks + Q) * kFeatChannels) = o;
  };
  const float zero6[6] = {0, 0, 0, 0, 0, 0};
  if (m <= 0 || n <= 0) {  // a one-point path: k = 1 and no cells
    for (int Q = 0; Q < kBlocks; ++Q) put(lane, Q, zero6);
    if (lane == 0) a.k0[pair] = 1.0f;
    return;
  }
  // lane l owns coarse cell rows 4l .. 4l + 3 (rows >= m are outside the grid:
  // zero increments, masked out of the moments)
  const int p0 = 4 * lane;
  float dx[4][D];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float t[DP];
    if (p0 + r < m) {
      fwd::load_row<DP>(a.incx + (pair * m + p0 + r) * DP, t);
    } else {
#pragma unroll
      for (int k = 0; k < DP; ++k) t[k] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) dx[r][k] = t[k];
  }
  // The scheme in double (the plain order-0 solve's arithmetic); the moments
  // in float32 from one float copy of every node.  The y increment row that
  // lane l needs at step t (row t - l) is the one lane l-1 used at step t-1:
  // rows travel down the wave by DPP, and only row t itself is loaded, by a
  // broadcast read (the same LDS address in every lane) one step ahead.
  double u[4] = {1.0, 1.0, 1.0, 1.0};  // nodes K[p0 + r + 1][q] left of column q
  float uf[4] = {1.0f, 1.0f, 1.0f, 1.0f};
  double pub = 1.0;                    // this lane's bottom node after its last column
  double up_last = 1.0;                // K[p0][q]: the upper-left node of row 0
  float up_last_f = 1.0f;
  float f[6] = {0, 0, 0, 0, 0, 0};
  float hf[6] = {0, 0, 0, 0, 0, 0};  // the last full block this lane ended
  int hq = -1;                       // its block column, -1: none pending
  const float* __restrict__ ybase = a.incy + pair * (int64_t)n * DP;
  // The rows reach the wave through LDS in blocks of 16: the wave loads
  // block b (DP / 4 floats per lane, zero past the path) at step 16 (b - 1),
  // writes it into half b mod 2 of its staging area at step 16 (b - 1) + 12,
  // and reads row 16 b first at step 16 b - 1; that half's previous block was
  // last read at step 16 (b - 1) - 2.  The loads so run 12 steps ahead of
  // their use instead of one.
  constexpr int PER = DP / 4;
  __shared__ float ystage[4][2][16 * DP];
  float (&stage)[2][16 * DP] = ystage[threadIdx.x >> 6];
  float pend[PER];
  auto issue = [&](int b) {  // block b's floats of this lane, into pend
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = lane * PER + i;
      const int q = 16 * b + e / DP;
      pend[i] = q < n ? ybase[(int64_t)16 * b * DP + e] : 0.0f;
    }
  };
  auto commit = [&](int b) {
#pragma unroll
    for (int i = 0; i < PER; ++i) stage[b & 1][lane * PER + i] = pend[i];
    __builtin_amdgcn_wave_barrier();
  };
  auto fetch = [&](int q, float (&row)[DP]) {  // row q of the stream, from LDS
#pragma unroll
    for (int k = 0; k < DP; ++k) row[k] = stage[(q >> 4) & 1][(q & 15) * DP + k];
  };
  float dy[DP];
#pragma unroll
  for (int k = 0; k < DP; ++k) dy[k] = 0.0f;
  auto step = [&](int t, const float (&fresh)[DP], float (&next)[DP]) {
    const int q = t - lane;
    fetch(t + 1, next);
#pragma unroll
    for (int k = 0; k < D; ++k)
      dy[k] = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fresh[k]),
                                                         __float_as_int(dy[k]), 0x138, 0xF, 0xF,
                                                         false));
    // lane l-1 finished column q at the previous step: its bottom node there
    // is K[p0][q + 1]; lane 0 reads the boundary row (value 1)
    const double up = fwd::from_prev_lane(pub, 1.0);
    if (q < 0 || q >= n) return;
    const float upf = (float)up;
    double nv[4];
    float nvf[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float c = 0.0f;
#pragma unroll
      for (int k = 0; k < D; ++k) c = __builtin_fmaf(dx[r][k], dy[k], c);
      const double A = u[r];
      const double B = (r == 0) ? up : nv[r - 1];
      const double C = (r == 0) ? up_last : u[r - 1];
      nv[r] = __builtin_fma(__builtin_fma((double)c, 0.5, 1.0), A + B, -C);
      nvf[r] = (float)nv[r];
      if (p0 + r < m) {
        const float Af = uf[r];
        const float Bf = (r == 0) ? upf : nvf[r - 1];
        const float Cf = (r == 0) ? up_last_f : uf[r - 1];
        const float s = Af + Bf, c2 = c * c;
        f[0] += c;
        f[1] = __builtin_fmaf(c2 * 0.5f, s, f[1]);
        f[2] = __builtin_fmaf(c, s, f[2]);
        f[3] += Cf - 1.0f;
        f[4] = __builtin_fmaf(c2, Cf, f[4]);
        f[5] = __builtin_fmaf(c, Bf - Af, f[5]);
      }
    }
    up_last = up;
    up_last_f = upf;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      u[r] = nv[r];
      uf[r] = nvf[r];
    }
    pub = nv[3];
    // a full block ends at column q = 4Q + 3: its moments move to the held
    // registers (selects, no branch: a quarter of the lanes end a block at
    // every step, as the lanes are one column apart)
    const bool done = (q & 3) == 3;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      hf[k] = done ? f[k] : hf[k];
      f[k] = done ? 0.0f : f[k];
    }
    hq = done ? q >> 2 : hq;
  };
  // the held blocks are written by the whole wave every fourth step: a lane
  // ends at most one full block per four steps, so none is overwritten first
  auto flush = [&]() {
    if (hq >= 0) put(lane, hq, hf);
    hq = -1;
  };
  issue(0);
  commit(0);
  issue(1);
  commit(1);
  float dyA[DP], dyB[DP];
  fetch(0, dyA);
  const int nsteps = n + 63;
  for (int t = 0; t < nsteps; t += 4) {
    if ((t & 15) == 0 && t > 0) issue((t >> 4) + 1);
    if ((t & 15) == 12 && t > 12) commit((t >> 4) + 1);
    step(t, dyA, dyB);
    step(t + 1, dyB, dyA);
    step(t + 2, dyA, dyB);
    step(t + 3, dyB, dyA);
    flush();
  }
  flush();
  // the last block, when n is not a multiple of 4, ends partial
  if (n & 3) put(lane, n >> 2, f);
  // k = K[m - 1][n - 1]: the last node of row m - 1, held by its lane
  if (lane == (m - 1) >> 2) a.k0[pair] = (float)u[(m - 1) & 3];
  for (int Q = (n + 3) >> 2; Q < kBlocks; ++Q) put(lane, Q, zero6);
}

template <int D>
void* features_fn() {
  return reinterpret_cast<void*>(&features_kernel<D>);
}

// ------------------------------------------------------------- conv tile --
__device__ __forceinline__ bf16x8 load8(const bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}
__device__ __forceinline__ bf16x8 load8(const float* p) {
  const float4 x0 = reinterpret_cast<const float4*>(p)[0];
  const float4 x1 = reinterpret_cast<const float4*>(p)[1];
  bf16x8 r;
  r[0] = (bf16)x0.x; r[1] = (bf16)x0.y; r[2] = (bf16)x0.z; r[3] = (bf16)x0.w;
  r[4] = (bf16)x1.x; r[5] = (bf16)x1.y; r[6] = (bf16)x1.z; r[7] = (bf16)x1.w;
  return r;
}

__device__ __forceinline__ float bf16r(float v) { return (float)(bf16)v; }

// Tile t of one pair's layer: 32 output positions (raster order, t*32 ..) x
// 32 output channels in acc.  Lane l supplies position (l mod 32) of the A
// tile and output channel (l mod 32) of the B tile; its half (l / 32)
// selects 8 of the 16 reduction indices of an instruction: for Cin = 32 one
// tap's channels c0 + 8 half .. + 8, for Cin = 8 tap 2 s + half of
// instruction s (a tenth tap is zero).  `in` is the pair's [HI][HI][Cin]
// bf16 map and `w` the layer's [32][9][Cin] weights (bf16, or float32
// rounded on load), either in global memory or in LDS.
template <int CIN, int HI, class TW>
__device__ __forceinline__ void conv_tile(const bf16* in, const TW* w, int t, int lane,
                                          f32x16& acc) {
  constexpr int HO = HI / 2, PPP = HO * HO;
  const int row = lane & 31, half = lane >> 5;
  const int pos = t * 32 + row;
  const bool valid = pos < PPP;
  const int ho = pos / HO, wo = pos - (pos / HO) * HO;
  auto a_op = [&](int tap, int c0) -> bf16x8 {
    const int kh = tap / 3, kw = tap - (tap / 3) * 3;
    const int hi = 2 * ho - 1 + kh, wi = 2 * wo - 1 + kw;
    if (valid && tap < 9 && hi >= 0 && hi < HI && wi >= 0 && wi < HI)
      return load8(in + ((hi * HI + wi) * CIN + c0));
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = (bf16)0.0f;
    return z;
  };
  auto b_op = [&](int tap, int c0) -> bf16x8 {
    if (tap < 9) return load8(w + ((row * 9 + tap) * CIN + c0));
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = (bf16)0.0f;
    return z;
  };
  if constexpr (CIN == 8) {
#pragma unroll
    for (int s = 0; s < 5; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_op(2 * s + half, 0), b_op(2 * s + half, 0),
                                                    acc, 0, 0, 0);
  } else {
    static_assert(CIN == 32, "layers have 8 or 32 input channels");
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
      for (int c0 = 0; c0 < 32; c0 += 16)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_op(tap, c0 + 8 * half),
                                                      b_op(tap, c0 + 8 * half), acc, 0, 0, 0);
    }
  }
}

// bias + ReLU, rounded to bf16: out[pos][co] of the tile's valid positions
template <int PPP>
__device__ __forceinline__ void store_tile(const f32x16& acc, float bias, bf16* out, int t,
                                           int lane) {
  const int half = lane >> 5, co = lane & 31;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int p = t * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
    if (p < PPP) out[p * kCout + co] = (bf16)fmaxf(acc[r] + bias, 0.0f);
  }
}

// Training / standalone forward of one layer: wave w = (pair, tile).
template <int CIN, int HI>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const ConvArgs a) {
  constexpr int HO = HI / 2, PPP = HO * HO, TPP = (PPP + 31) / 32;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wave >= a.n * TPP) return;
  const int64_t pn = wave / TPP;
  const int t = (int)(wave - pn * TPP);
  f32x16 acc = {};
  conv_tile<CIN, HI>(a.in + pn * (int64_t)(HI * HI * CIN), a.w, t, lane, acc);
  store_tile<PPP>(acc, a.b[lane & 31], a.out + pn * (int64_t)(PPP * kCout), t, lane);
}

// ------------------------------------------------------ fused inference --
// Persistent workgroups of 8 waves, one pair at a time: the feature map,
// layer 1's output and the current layer's weights stay in LDS; layer 2's
// output reuses the feature map's space and layers 3-4 that of layer 1; only
// the two outputs leave the chip.  While a pair is evaluated, waves 4-7 hold
// the next pair's feature map in registers (loaded at the start, written to
// LDS once layer 3 has read the feature map's space), and waves 0-3 stage the
// weights: a wave's global loads complete in order, so the waves that wait on
// weight loads must not be the ones with the feature loads in flight.
constexpr int kNetThreads = 512;
constexpr int kLdsF = kFeatFloats;              // feature map, later layer 2
constexpr int kLdsA1 = 32 * 32 * kCout;         // layer 1 output, later layers 3-4
constexpr int kLdsW = kCout * 9 * 32;           // one layer's weights
constexpr int kStageThreads = 256;              // waves 0-3
constexpr int kFeat16 = kFeatFloats / 8;        // 16-byte chunks of a feature map
constexpr int kPre = kFeat16 / (kNetThreads - kStageThreads);  // per thread of waves 4-7
static_assert(kPre * (kNetThreads - kStageThreads) == kFeat16, "feature map split");
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // stays in registers

template <int CIN>
__device__ __forceinline__ void stage_weights(bf16* W, const bf16* src, int tid) {
  constexpr int N16 = kCout * 9 * CIN / 8;  // 16-byte chunks
  if (tid >= kStageThreads) return;
  for (int i = tid; i < N16; i += kStageThreads)
    reinterpret_cast<uint4*>(W)[i] = reinterpret_cast<const uint4*>(src)[i];
}

__global__ __launch_bounds__(kNetThreads) void net_fused_kernel(const NetArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 lds[kLdsF + kLdsA1 + kLdsW];
  bf16* F = lds;
  bf16* A1 = lds + kLdsF;
  bf16* W = lds + kLdsF + kLdsA1;
  bf16* A2 = F;                 // 16 x 16 x 32
  bf16* A3 = A1;                // 8 x 8 x 32
  bf16* A4 = A1 + 8 * 8 * 32;   // 4 x 4 x 32
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // the biases of the four layers (the same for every pair)
  float bias[4];
  bias[0] = a.params[param_offset(0) + kCout * 9 * 8 + (lane & 31)];
#pragma unroll
  for (int l = 1; l < 4; ++l) bias[l] = a.params[param_offset(l) + kCout * 9 * 32 + (lane & 31)];
  if ((int64_t)blockIdx.x < a.n) {
    const uint4* src = reinterpret_cast<const uint4*>(a.feats + blockIdx.x * (int64_t)kFeatFloats);
    for (int i = tid; i < kFeat16; i += kNetThreads) reinterpret_cast<uint4*>(F)[i] = src[i];
  }
  for (int64_t pn = blockIdx.x; pn < a.n; pn += gridDim.x) {
    const int64_t nx = pn + gridDim.x;
    const bool pre = wid >= 4 && nx < a.n;
    u32x4 next[kPre];
    if (pre) {
      const u32x4* src = reinterpret_cast<const u32x4*>(a.feats + nx * (int64_t)kFeatFloats);
#pragma unroll
      for (int j = 0; j < kPre; ++j)
        next[j] = src[(tid - kStageThreads) + j * (kNetThreads - kStageThreads)];
    }
    stage_weights<8>(W, a.wb + param_offset(0), tid);
    __syncthreads();
    for (int t = wid; t < 32; t += 8) {  // layer 1: 64 x 64 x 8 -> 32 x 32 x 32
      f32x16 acc = {};
      conv_tile<8, 64>(F, W, t, lane, acc);
      store_tile<32 * 32>(acc, bias[0], A1, t, lane);
    }
    __syncthreads();
    stage_weights<32>(W, a.wb + param_offset(1), tid);
    __syncthreads();
    {
      f32x16 acc = {};
      conv_tile<32, 32>(A1, W, wid, lane, acc);
      store_tile<16 * 16>(acc, bias[1], A2, wid, lane);
    }
    __syncthreads();
    stage_weights<32>(W, a.wb + param_offset(2), tid);
    __syncthreads();
    if (wid < 2) {
      f32x16 acc = {};
      conv_tile<32, 16>(A2, W, wid, lane, acc);
      store_tile<8 * 8>(acc, bias[2], A3, wid, lane);
    }
    __syncthreads();
    // the feature map's space is free: the next pair's map goes in
    if (pre) {
#pragma unroll
      for (int j = 0; j < kPre; ++j)
        reinterpret_cast<u32x4*>(F)[(tid - kStageThreads) + j * (kNetThreads - kStageThreads)] =
            next[j];
    }
    stage_weights<32>(W, a.wb + param_offset(3), tid);
    __syncthreads();
    if (wid == 0) {
      f32x16 acc = {};
      conv_tile<32, 8>(A3, W, 0, lane, acc);
      store_tile<4 * 4>(acc, bias[3], A4, 0, lane);
    }
    __syncthreads();
    if (wid == 0) {  // head, in the order of head_fwd_kernel
      const float* __restrict__ wh = a.params + kHeadOffset;
      float s0 = 0.0f, s1 = 0.0f;
      for (int k = lane; k < kHeadIn; k += 64) {
        const float x = (float)A4[k];
        s0 = __builtin_fmaf(x, wh[k], s0);
        s1 = __builtin_fmaf(x, wh[kHeadIn + k], s1);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
      }
      // every lane of the wave holds the same sums (the butterfly adds the
      // same two operands in every lane) and stores them
      a.y[2 * pn] = s0 + wh[2 * kHeadIn];
      a.y[2 * pn + 1] = s1 + wh[2 * kHeadIn + 1];
    }
    // the next pair's layer 1 overwrites layers 3-4 only after the barrier
    // that follows its weight staging, which wave 0 reaches after the head
  }
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ x, int64_t n,
                                                      bf16* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (bf16)x[i];
}

// ---------------------------------------------------------- conv backward --
// Gradient of the pre-activation at output element e: dout where the ReLU
// passed (out > 0), else 0.
__device__ __forceinline__ float dpre(const bf16* out, const float* dout, int64_t e) {
  return (float)out[e] > 0.0f ? dout[e] : 0.0f;
}

template <int CIN, int HI>
__global__ __launch_bounds__(256) void conv_dx_kernel(const ConvBwdArgs a) {
  constexpr int HO = HI / 2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n * HI * HI * CIN) return;
  const int ci = (int)(e % CIN);
  const int64_t pix = e / CIN;
  const int wi = (int)(pix % HI), hi = (int)((pix / HI) % HI);
  const int64_t pn = pix / (HI * HI);
  float s = 0.0f;
#pragma unroll
  for (int kh = 0; kh < 3; ++kh) {
    const int th = hi + 1 - kh;  // = 2 ho
    if (th < 0 || (th & 1) || (th >> 1) >= HO) continue;
#pragma unroll
    for (int kw = 0; kw < 3; ++kw) {
      const int tw = wi + 1 - kw;
      if (tw < 0 || (tw & 1) || (tw >> 1) >= HO) continue;
      const int64_t o = ((pn * HO + (th >> 1)) * HO + (tw >> 1)) * kCout;
      const float* __restrict__ wp = a.w + (kh * 3 + kw) * CIN + ci;
#pragma unroll 8
      for (int co = 0; co < kCout; ++co)
        s = __builtin_fmaf(dpre(a.out, a.dout, o + co), bf16r(wp[co * 9 * CIN]), s);
    }
  }
  a.din[e] = s;
}

// Partial weight and bias gradients of one workgroup's positions:
// partial[block][E + 32], E = 32 x 9 x Cin (weight order), then the biases.
template <int CIN, int HI>
__global__ __launch_bounds__(256) void conv_dw_kernel(const ConvBwdArgs a) {
  constexpr int HO = HI / 2, PPP = HO * HO;
  constexpr int KT = 9 * CIN, E = kCout * KT, PER = (E + 255) / 256, CH = 16;
  __shared__ float sd[CH][kCout];
  __shared__ float sp[CH][KT];
  const int tid = threadIdx.x;
  const int64_t T = a.n * PPP;
  const int64_t begin = (int64_t)blockIdx.x * a.per_block;
  const int64_t end = begin + a.per_block < T ? begin + a.per_block : T;
  float acc[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) acc[j] = 0.0f;
  float db = 0.0f;
  for (int64_t c0 = begin; c0 < end; c0 += CH) {
    __syncthreads();
    for (int e2 = tid; e2 < CH * kCout; e2 += 256) {
      const int64_t p = c0 + e2 / kCout;
      sd[e2 / kCout][e2 % kCout] = p < end ? dpre(a.out, a.dout, p * kCout + e2 % kCout) : 0.0f;
    }
    for (int e2 = tid; e2 < CH * KT; e2 += 256) {
      const int pp = e2 / KT, r = e2 - (e2 / KT) * KT;
      const int tap = r / CIN, ci = r - (r / CIN) * CIN;
      const int64_t p = c0 + pp;
      float v = 0.0f;
      if (p < end) {
        const int64_t pn = p / PPP;
        const int rem = (int)(p - pn * PPP);
        const int hi = 2 * (rem / HO) - 1 + tap / 3, wi = 2 * (rem % HO) - 1 + tap % 3;
        if (hi >= 0 && hi < HI && wi >= 0 && wi < HI)
          v = (float)a.in[((pn * HI + hi) * HI + wi) * CIN + ci];
      }
      sp[pp][r] = v;
    }
    __syncthreads();
#pragma unroll 1
    for (int pp = 0; pp < CH; ++pp) {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int e = tid + 256 * j;
        if (E % 256 == 0 || e < E) acc[j] = __builtin_fmaf(sd[pp][e / KT], sp[pp][e % KT], acc[j]);
      }
      if (tid < kCout) db += sd[pp][tid];
    }
  }
  float* __restrict__ part = a.partial + (int64_t)blockIdx.x * (E + kCout);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int e = tid + 256 * j;
    if (e < E) part[e] = acc[j];
  }
  if (tid < kCout) part[E + tid] = db;
}

// grads[e] = sum over blocks (in block order) of partial[block][e]
__global__ __launch_bounds__(256) void reduce_partials_kernel(const float* __restrict__ partial,
                                                              int nblocks, int width,
                                                              float* __restrict__ grads) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= width) return;
  float s = 0.0f;
  for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * width + e];
  grads[e] = s;
}

// ------------------------------------------------------------------- head --
__global__ __launch_bounds__(256) void head_fwd_kernel(const bf16* __restrict__ act4,
                                                       const float* __restrict__ wh,
                                                       const float* __restrict__ bh, int64_t n,
                                                       float* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t pn = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pn >= n) return;
  const bf16* __restrict__ x = act4 + pn * kHeadIn;
  float s0 = 0.0f, s1 = 0.0f;
  for (int k = lane; k < kHeadIn; k += 64) {
    const float xv = (float)x[k];
    s0 = __builtin_fmaf(xv, wh[k], s0);
    s1 = __builtin_fmaf(xv, wh[kHeadIn + k], s1);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
  }
  if (lane == 0) {
    y[2 * pn] = s0 + bh[0];
    y[2 * pn + 1] = s1 + bh[1];
  }
}

__global__ __launch_bounds__(256) void head_dx_kernel(const float* __restrict__ dy,
                                                      const float* __restrict__ wh, int64_t n,
                                                      float* __restrict__ dact4) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kHeadIn) return;
  const int64_t pn = e / kHeadIn;
  const int k = (int)(e - pn * kHeadIn);
  dact4[e] = __builtin_fmaf(dy[2 * pn], wh[k], dy[2 * pn + 1] * wh[kHeadIn + k]);
}

// grads of the head: [2][512] weights then [2] biases, summed over pairs in order
__global__ __launch_bounds__(256) void head_dw_kernel(const float* __restrict__ dy,
                                                      const bf16* __restrict__ act4, int64_t n,
                                                      float* __restrict__ g) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * kHeadIn + 2) return;
  float s = 0.0f;
  if (e < 2 * kHeadIn) {
    const int o = e / kHeadIn, k = e - (e / kHeadIn) * kHeadIn;
    for (int64_t pn = 0; pn < n; ++pn)
      s = __builtin_fmaf(dy[2 * pn + o], (float)act4[pn * kHeadIn + k], s);
  } else {
    const int o = e - 2 * kHeadIn;
    for (int64_t pn = 0; pn < n; ++pn) s += dy[2 * pn + o];
  }
  g[e] = s;
}

// ------------------------------------------------------------ loss, Adam --
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ y,
                                                   const float* __restrict__ k_target,
                                                   const float* __restrict__ k0,
                                                   const float* __restrict__ tnorm, int64_t n,
                                                   float* __restrict__ loss,
                                                   float* __restrict__ dy) {
  __shared__ double red[256];
  const float mu = tnorm[0], rsig = 1.0f / tnorm[1];
  const float inv_n = 1.0f / (float)n;
  double part = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float t = (k_target[i] - k0[i] - mu) * rsig;
    const float r = y[2 * i] - t, s = y[2 * i + 1];
    const float e = expf(-2.0f * s);
    part += (double)(r * r) + 0.5 * (double)(r * r * e) + (double)s;
    dy[2 * i] = 2.0f * r * inv_n;
    dy[2 * i + 1] = (1.0f - r * r * e) * inv_n;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(red[0] / (double)n);
}

__global__ void tick_kernel(int32_t* step) {
  if (threadIdx.x == 0) step[0] = step[0] + 1;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t n, const int32_t* __restrict__ step,
                                                   float lr, float b1, float b2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = (double)step[0];
  const float c1 = (float)(1.0 / (1.0 - pow((double)b1, t)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)b2, t)));
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// --------------------------------------------------------- channel stats --
constexpr int kStatBlocks = 256;

// pass 0: per-block sums of v = x (- sub); pass 1: of (v - mean)^2 (mean from ws)
template <class T>
__global__ __launch_bounds__(256) void stats_partial_kernel(const T* __restrict__ x,
                                                            const float* __restrict__ sub,
                                                            int64_t rows, int C, int pass,
                                                            double* __restrict__ ws) {
  __shared__ double red[256][kMaxStatChannels];
  double s[kMaxStatChannels];
  double mean[kMaxStatChannels];
  for (int c = 0; c < kMaxStatChannels; ++c) {
    s[c] = 0.0;
    mean[c] = (pass && c < C) ? ws[2 * kStatBlocks * kMaxStatChannels + c] : 0.0;
  }
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows;
       r += (int64_t)kStatBlocks * 256) {
    for (int c = 0; c < C; ++c) {
      const double xv = sub ? (double)x[r * C + c] - (double)sub[r * C + c] : (double)x[r * C + c];
      const double v = xv - mean[c];
      s[c] += pass ? v * v : v;
    }
  }
  for (int c = 0; c < kMaxStatChannels; ++c) red[threadIdx.x][c] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < kMaxStatChannels; ++c) red[threadIdx.x][c] += red[threadIdx.x + w][c];
    __syncthreads();
  }
  if ((int)threadIdx.x < C)
    ws[(pass * kStatBlocks + blockIdx.x) * kMaxStatChannels + threadIdx.x] = red[0][threadIdx.x];
}

__global__ void stats_final_kernel(int64_t rows, int C, int pass, double* __restrict__ ws,
                                   float* __restrict__ mean, float* __restrict__ rstd) {
  const int c = threadIdx.x;
  if (c >= C) return;
  double s = 0.0;
  for (int b = 0; b < kStatBlocks; ++b) s += ws[(pass * kStatBlocks + b) * kMaxStatChannels + c];
  const double v = s / (double)rows;
  if (pass == 0) {
    ws[2 * kStatBlocks * kMaxStatChannels + c] = v;
    mean[c] = (float)v;
  } else {
    rstd[c] = v > 0.0 ? (float)(1.0 / sqrt(v)) : 1.0f;
  }
}

// ---------------------------------------------------------------- decide --
__global__ __launch_bounds__(256) void decide_kernel(const DecideArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < a.n;
  bool fb = false;
  if (in) {
    const float mu = a.tnorm[0], sigma = a.tnorm[1];
    const float y0 = a.y[2 * i], y1 = a.y[2 * i + 1];
    const float k = a.k0[i] + mu + sigma * y0;
    const float err = sigma * expf(y1);
    // relative: kappa e <= tol |k_hat| accepts (NaN falls back)
    fb = !(a.kappa * err <= a.tol * fabsf(k));
    a.out[i] = k;
    if (a.err) a.err[i] = err;
    if (a.fallback) a.fallback[i] = fb ? 1 : 0;
  }
  // wave-aggregated compaction: one vector atomic per wave
  const unsigned long long mask = __ballot(fb);
  if (mask == 0) return;
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == __ffsll((long long)mask) - 1) base = atomicAdd(a.count, __popcll(mask));
  base = __shfl(base, __ffsll((long long)mask) - 1, 64);
  if (fb) {
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    a.order[base + rank] = (int32_t)i;
  }
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

template <int CIN, int HI>
struct Layer {
  static hipError_t fwd(const ConvArgs& a, hipStream_t s) {
    constexpr int64_t TPP = ((HI / 2) * (HI / 2) + 31) / 32;
    const int64_t waves = a.n * TPP;
    if (waves == 0) return hipSuccess;
    hipLaunchKernelGGL((conv_fwd_kernel<CIN, HI>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0,
                       s, a);
    return hipGetLastError();
  }
  static hipError_t dx(const ConvBwdArgs& a, hipStream_t s) {
    const int64_t total = a.n * HI * HI * CIN;
    hipLaunchKernelGGL((conv_dx_kernel<CIN, HI>), dim3((unsigned)((total + 255) / 256)), dim3(256),
                       0, s, a);
    return hipGetLastError();
  }
  static hipError_t dw(const ConvBwdArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((conv_dw_kernel<CIN, HI>), dim3((unsigned)a.nblocks), dim3(256), 0, s, a);
    return hipGetLastError();
  }
};

}  // namespace

// ------------------------------------------------------------- launchers --
hipError_t launch_features(const FeatArgs& a, int d, hipStream_t s) {
  if (a.npairs == 0) return hipSuccess;
  void* f = nullptr;
  switch (d) {
    case 1: f = features_fn<1>(); break;
    case 2: f = features_fn<2>(); break;
    case 3: f = features_fn<3>(); break;
    case 4: f = features_fn<4>(); break;
    case 5: f = features_fn<5>(); break;
    case 6: f = features_fn<6>(); break;
    case 7: f = features_fn<7>(); break;
    case 8: f = features_fn<8>(); break;
    case 9: f = features_fn<9>(); break;
    case 10: f = features_fn<10>(); break;
    case 11: f = features_fn<11>(); break;
    case 12: f = features_fn<12>(); break;
    case 13: f = features_fn<13>(); break;
    case 14: f = features_fn<14>(); break;
    case 15: f = features_fn<15>(); break;
    case 16: f = features_fn<16>(); break;
    default: return hipErrorInvalidValue;
  }
  const int64_t blocks = (a.npairs + 3) / 4;
  hipLaunchKernelGGL(reinterpret_cast<void (*)(const FeatArgs)>(f), dim3((unsigned)blocks),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_conv_fwd(int layer, const ConvArgs& a, hipStream_t s) {
  switch (layer) {
    case 0: return Layer<8, 64>::fwd(a, s);
    case 1: return Layer<32, 32>::fwd(a, s);
    case 2: return Layer<32, 16>::fwd(a, s);
    case 3: return Layer<32, 8>::fwd(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_conv_dx(int layer, const ConvBwdArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  switch (layer) {
    case 1: return Layer<32, 32>::dx(a, s);
    case 2: return Layer<32, 16>::dx(a, s);
    case 3: return Layer<32, 8>::dx(a, s);
    default: return hipErrorInvalidValue;  // layer 0: the features need no gradient
  }
}

hipError_t launch_conv_dw(int layer, const ConvBwdArgs& a, float* grads, hipStream_t s) {
  const int cin = kLayerCin[layer];
  const int width = kCout * 9 * cin + kCout;
  if (a.n == 0 || a.nblocks == 0) {
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((width + 255) / 256)), dim3(256), 0,
                       s, a.partial, 0, width, grads);
    return hipGetLastError();
  }
  hipError_t e;
  switch (layer) {
    case 0: e = Layer<8, 64>::dw(a, s); break;
    case 1: e = Layer<32, 32>::dw(a, s); break;
    case 2: e = Layer<32, 16>::dw(a, s); break;
    case 3: e = Layer<32, 8>::dw(a, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((width + 255) / 256)), dim3(256), 0, s,
                     a.partial, a.nblocks, width, grads);
  return hipGetLastError();
}

hipError_t launch_head_fwd(const bf16* act4, const float* wh, const float* bh, int64_t n,
                           float* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, act4, wh, bh,
                     n, y);
  return hipGetLastError();
}

hipError_t launch_head_bwd(const float* dy, const bf16* act4, const float* wh, int64_t n,
                           float* dact4, float* g_head, hipStream_t s) {
  if (n > 0) {
    hipLaunchKernelGGL(head_dx_kernel, dim3((unsigned)((n * kHeadIn + 255) / 256)), dim3(256), 0, s,
                       dy, wh, n, dact4);
  }
  hipLaunchKernelGGL(head_dw_kernel, dim3((2 * kHeadIn + 2 + 255) / 256), dim3(256), 0, s, dy, act4,
                     n, g_head);
  return hipGetLastError();
}

hipError_t launch_loss(const float* y, const float* k_target, const float* k0, const float* tnorm,
                       int64_t n, float* loss, float* dy, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, y, k_target, k0, tnorm, n, loss, dy);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int32_t* step,
                       float lr, float b1, float b2, float eps, hipStream_t s) {
  hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, s, step);
  if (n > 0)
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v,
                       n, (const int32_t*)step, lr, b1, b2, eps);
  return hipGetLastError();
}

hipError_t launch_channel_stats(const void* x, bool x_bf16, const float* sub, int64_t rows, int C,
                                float* mean, float* rstd, double* ws, hipStream_t s) {
  for (int pass = 0; pass < 2; ++pass) {
    if (x_bf16)
      hipLaunchKernelGGL(stats_partial_kernel<bf16>, dim3(kStatBlocks), dim3(256), 0, s,
                         static_cast<const bf16*>(x), sub, rows, C, pass, ws);
    else
      hipLaunchKernelGGL(stats_partial_kernel<float>, dim3(kStatBlocks), dim3(256), 0, s,
                         static_cast<const float*>(x), sub, rows, C, pass, ws);
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(64), 0, s, rows, C, pass, ws, mean, rstd);
  }
  return hipGetLastError();
}

hipError_t launch_net_fused(const NetArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  // one persistent workgroup per compute unit (the LDS holds one)
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorInvalidDevice;
  const int64_t blocks = a.n < (int64_t)cus ? a.n : (int64_t)(cus > 0 ? cus : 1);
  hipLaunchKernelGGL(net_fused_kernel, dim3((unsigned)blocks), dim3(kNetThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, int64_t n, bf16* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, y);
  return hipGetLastError();
}

hipError_t launch_decide(const DecideArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, a.count, 4);
  if (a.n > 0)
    hipLaunchKernelGGL(decide_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace corr
}  // namespace sk
