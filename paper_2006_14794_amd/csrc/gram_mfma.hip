// Coarse increment Gram G0[p][q] = <x_{p+1} - x_p, y_{q+1} - y_q> (Section
// 3.1, piecewise-linear case) of every pair of two uniform batches with 17 to
// 64 channels, on the matrix cores.  (At 16 channels or fewer the contraction
// is too short to pay for them and the row kernel of gram_rows.hip writes G0.)
//
// A workgroup owns 64 whole rows of one pair's G0.  It stages the points of
// those rows and of 128-column chunks of the other path in LDS (up to 64
// channels), each of its four waves takes one 32-column strip of the chunk,
// and a wave accumulates the strip's two 32 x 32 tiles (rows 0-31 and 32-63
// of the block) in sixteen float32 registers per lane each, forming each y
// operand once for both:
//   float32 inputs: v_mfma_f32_32x32x2_f32, two channels per instruction;
//   bf16 / fp16 inputs: v_mfma_f32_32x32x16_{bf16,f16}, sixteen channels per
//   instruction (increments rounded to nearest even, products and sums in
//   float32).
// Operands are the increments themselves, formed from the staged points.
// Lane l supplies row (l mod 32) of the x tile and column (l mod 32) of the y
// tile; its half (l / 32) selects the channel slice.  Accumulator register r
// of lane l holds row 8 (r / 4) + 4 (l / 32) + (r mod 4), column l mod 32,
// and is stored from there: each store instruction writes 32 consecutive
// floats of two rows.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"

namespace sk {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kChunk = 128;    // columns per output chunk: one 32-column tile per wave
constexpr int kMaxDim = kGramMfmaMaxDim;  // channels staged in LDS

template <int PREC>  // 0: float32, 1: bf16, 2: fp16
__global__ __launch_bounds__(256) void gram_mfma_kernel(const GramArgs a) {
  // staged points, row stride ds = d | 1 (odd: a tile's 32 rows or columns,
  // one per lane, fall in distinct LDS banks)
  __shared__ float xs[65 * (kMaxDim + 1)];            // 65 points: 64 increments
  __shared__ float ys[(kChunk + 1) * (kMaxDim + 1)];  // a chunk's 129 points
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t pair = blockIdx.x;
  const int64_t ia = a.gram ? pair / a.ny : pair;
  const int64_t ib = a.gram ? pair - ia * a.ny : pair;
  const int32_t m = a.x_len - 1, n = a.y_len - 1, d = a.d;
  const int32_t p0 = blockIdx.y * 64;  // 64 whole rows of the pair
  const int32_t rows = m - p0 < 64 ? m - p0 : 64;
  const float* __restrict__ xp = a.x + (ia * (int64_t)a.x_len + p0) * d;
  const float* __restrict__ yq = a.y + ib * (int64_t)a.y_len * d;
  const int64_t ld = a.ld;  // row stride of G0, >= n
  float* __restrict__ g = a.g0 + pair * (int64_t)m * ld + (int64_t)p0 * ld;
  const int32_t ds = d | 1;
  // staging: thread t copies channel t mod d of every (256 / d)-th point, so
  // consecutive threads read consecutive floats
  const int32_t st_ch = (int32_t)threadIdx.x % d, st_r0 = (int32_t)threadIdx.x / d,
                st_step = 256 / d;
  const bool stager = st_r0 < st_step;
  if (stager)
    for (int32_t r = st_r0; r <= rows; r += st_step) xs[r * ds + st_ch] = xp[r * d + st_ch];
  const int32_t row = lane & 31, half = lane >> 5;
  auto xinc = [&](int rt, int k) -> float {  // row tile rt (0, 1)
    const int r = rt * 32 + row;
    return (r < rows && k < d) ? xs[(r + 1) * ds + k] - xs[r * ds + k] : 0.0f;
  };
  for (int32_t c0 = 0; c0 < n; c0 += kChunk) {
    const int32_t cw = n - c0 < kChunk ? n - c0 : kChunk;
    __syncthreads();  // xs ready / the previous chunk's ys consumed
    if (stager)
      for (int32_t r = st_r0; r <= cw; r += st_step)
        ys[r * ds + st_ch] = yq[(int64_t)(c0 + r) * d + st_ch];
    __syncthreads();
    for (int32_t t0 = wid * 32; t0 < cw; t0 += 128) {
      auto yinc = [&](int k) -> float {
        const int c = t0 + row;
        return (c < cw && k < d) ? ys[(c + 1) * ds + k] - ys[c * ds + k] : 0.0f;
      };
      f32x16 acc0 = {}, acc1 = {};
      if constexpr (PREC == 0) {
        for (int k0 = 0; k0 < d; k0 += 2) {
          const float B = yinc(k0 + half);
          acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(xinc(0, k0 + half), B, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(xinc(1, k0 + half), B, acc1, 0, 0, 0);
        }
      } else {
        for (int k0 = 0; k0 < d; k0 += 16) {
          if constexpr (PREC == 1) {
            bf16x8 A0, A1, B;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              A0[j] = (__bf16)xinc(0, k0 + half * 8 + j);
              A1[j] = (__bf16)xinc(1, k0 + half * 8 + j);
              B[j] = (__bf16)yinc(k0 + half * 8 + j);
            }
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A0, B, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, B, acc1, 0, 0, 0);
          } else {
            f16x8 A0, A1, B;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              A0[j] = (_Float16)xinc(0, k0 + half * 8 + j);
              A1[j] = (_Float16)xinc(1, k0 + half * 8 + j);
              B[j] = (_Float16)yinc(k0 + half * 8 + j);
            }
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(A0, B, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(A1, B, acc1, 0, 0, 0);
          }
        }
      }
      // straight from the accumulators: lanes 0-31 write 32 consecutive
      // floats of one row, lanes 32-63 of another (the L2 merges the
      // workgroup's rows into whole lines before they reach HBM)
      const int32_t c = t0 + row;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int32_t R = 8 * (r >> 2) + 4 * half + (r & 3);
        if (R < rows && c < cw) g[(int64_t)R * ld + c0 + c] = acc0[r];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int32_t R = 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (R < rows && c < cw) g[(int64_t)R * ld + c0 + c] = acc1[r];
      }
    }
  }
}

}  // namespace

hipError_t launch_gram_mfma(const GramArgs& a, int precision, hipStream_t stream) {
  const int32_t m = a.x_len - 1, n = a.y_len - 1;
  const int64_t pairs = a.gram ? a.nx * a.ny : a.nx;
  if (m <= 0 || n <= 0 || pairs == 0) return hipSuccess;
  if (a.ld < n || a.d < 1 || a.d > kMaxDim) return hipErrorInvalidValue;
  const int64_t row_blocks = (m + 63) / 64;
  if (row_blocks > 65535 || pairs > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)pairs, (unsigned)row_blocks, 1);
  if (precision == kRoundBf16)
    hipLaunchKernelGGL(gram_mfma_kernel<1>, grid, dim3(256), 0, stream, a);
  else if (precision == kRoundF16)
    hipLaunchKernelGGL(gram_mfma_kernel<2>, grid, dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(gram_mfma_kernel<0>, grid, dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace sk
