// Internal declarations of the learned corrector (corrector.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {
namespace corr {

using bf16 = __bf16;

constexpr int kBlocks = 64;          // feature map side: 64 blocks of 4 x 4 coarse cells
constexpr int kFeatChannels = 8;
constexpr int kFeatFloats = kBlocks * kBlocks * kFeatChannels;
constexpr int kCout = 32;            // channels of every conv layer
constexpr int kHeadIn = 4 * 4 * kCout;
constexpr int kMaxStatChannels = 8;
constexpr int kLayers = 4;
constexpr int kLayerCin[kLayers] = {8, 32, 32, 32};
constexpr int kLayerHi[kLayers] = {64, 32, 16, 8};

constexpr int64_t layer_params(int l) { return (int64_t)kCout * 9 * kLayerCin[l] + kCout; }
// flat parameter vector: per layer [32][3][3][Cin] weights then [32] biases,
// then the head's [2][512] weights and [2] biases
constexpr int64_t param_offset(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += layer_params(i);
  return o;
}
constexpr int64_t kHeadOffset = param_offset(kLayers);
constexpr int64_t kParams = kHeadOffset + 2 * kHeadIn + 2;
// activations per pair: the outputs of the four layers, layer-major
constexpr int64_t act_floats(int l) {
  return (int64_t)(kLayerHi[l] / 2) * (kLayerHi[l] / 2) * kCout;
}
constexpr int64_t kActFloats = act_floats(0) + act_floats(1) + act_floats(2) + act_floats(3);
constexpr int64_t act_offset(int l) {  // per pair; multiply by the batch size
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += act_floats(i);
  return o;
}
// channel statistics scratch: two passes of per-block partials and the mean
constexpr size_t kStatsWorkspaceBytes = (2 * 256 + 1) * kMaxStatChannels * sizeof(double);

struct FeatArgs {
  const float* incx;   // dense increments (padded pitch), uniform batches, not scaled
  const float* incy;
  int32_t m, n;        // coarse increments per x / y path, <= 256
  int64_t npairs;
  const float* norm;   // [16]: mean[8], 1/std[8] (nullptr: raw moments)
  bf16* feats;         // [npairs][64][64][8]
  float* k0;           // [npairs]: order-0 terminal value
};

struct ConvArgs {
  const bf16* in;      // [n][HI][HI][Cin]
  const float* w;      // [32][3][3][Cin] (rounded to bf16 on load)
  const float* b;      // [32]
  bf16* out;           // [n][HI/2][HI/2][32], after ReLU
  int64_t n;
};

struct NetArgs {
  const bf16* feats;   // [n][64][64][8]
  const bf16* wb;      // bf16 copy of the conv part of the parameters (same offsets)
  const float* params; // biases and the head
  int64_t n;
  float* y;            // [n][2]
};

struct ConvBwdArgs {
  const bf16* in;      // layer input
  const float* w;
  const bf16* out;     // layer output (after ReLU): the ReLU mask
  const float* dout;   // gradient with respect to the output
  float* din;          // gradient with respect to the input
  float* partial;      // [nblocks][32 * 9 * Cin + 32]
  int64_t n;
  int nblocks;
  int64_t per_block;   // output positions per workgroup (a multiple of 16)
};

struct DecideArgs {
  const float* k0;
  const float* y;      // [n][2] network outputs
  const float* tnorm;  // [2]: mu, sigma of the order-3 minus order-0 difference
  float kappa, tol;
  int64_t n;
  float* out;          // corrected values
  float* err;          // predicted errors (nullable)
  int32_t* fallback;   // 0/1 per pair (nullable)
  int32_t* order;      // [n]: compacted ids of the pairs that fall back
  int32_t* count;      // [4]: count, 0, queue head, 0 (zeroed by the launcher)
};

hipError_t launch_features(const FeatArgs& a, int d, hipStream_t s);
hipError_t launch_conv_fwd(int layer, const ConvArgs& a, hipStream_t s);
hipError_t launch_conv_dx(int layer, const ConvBwdArgs& a, hipStream_t s);
hipError_t launch_conv_dw(int layer, const ConvBwdArgs& a, float* grads, hipStream_t s);
hipError_t launch_head_fwd(const bf16* act4, const float* wh, const float* bh, int64_t n,
                           float* y, hipStream_t s);
hipError_t launch_head_bwd(const float* dy, const bf16* act4, const float* wh, int64_t n,
                           float* dact4, float* g_head, hipStream_t s);
hipError_t launch_net_fused(const NetArgs& a, hipStream_t s);
hipError_t launch_to_bf16(const float* x, int64_t n, bf16* y, hipStream_t s);
hipError_t launch_loss(const float* y, const float* k_target, const float* k0, const float* tnorm,
                       int64_t n, float* loss, float* dy, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int32_t* step,
                       float lr, float b1, float b2, float eps, hipStream_t s);
hipError_t launch_channel_stats(const void* x, bool x_bf16, const float* sub, int64_t rows, int C,
                                float* mean, float* rstd, double* ws, hipStream_t s);
hipError_t launch_decide(const DecideArgs& a, hipStream_t s);

}  // namespace corr
}  // namespace sk
