// Coarse increment Gram G0[p][q] = <x_{p+1} - x_p, y_{q+1} - y_q> (Section
// 3.1, piecewise-linear case) of every pair of two uniform batches, on the
// vector ALUs, written row after row.
//
// At d <= 16 channels the contraction is 2d flops per 4-byte output, far
// below the matrix cores' ridge: the kernel is bound by its HBM writes, and
// the order of those writes sets their rate.  A workgroup owns 64 consecutive
// rows of one pair (up to 256 columns; wider rows are split into 256-column
// chunks over consecutive workgroups).  It stages the chunk's y points in LDS
// once; each of its four waves then holds the y increments of columns
// l + 64 j (lane l, j < 4) in registers and writes every fourth row (rows
// r0 + w, r0 + w + 4, ...), so the four waves advance through the block's
// rows together and their stores fill one contiguous region front to back.
// Each store instruction writes 64 consecutive floats.  A wave's x
// increments (the same for every lane) are formed into its slice of LDS
// before its first store: in the row loop they are LDS reads, which wait on
// their own counter, whereas a global load there would also wait for every
// store the wave has issued.  Products and sums are float32, channel by
// channel in order; with 16-bit inputs both increments are first rounded to
// bfloat16 / half (round to nearest even), so each product is exact in
// float32.
//
// On the 128 x 128 Gram of 256-point paths (d = 9, 4.26 GB of G0) it takes
// 0.86 ms against 1.36 ms for 32 x 32 MFMA tiles stored from the
// accumulators.  Measured alternatives: 64 whole rows per wave with per-wave y
// loads 0.98 ms; the y chunk shared by the workgroup with 16, 32 or 64
// consecutive rows per wave 0.89, 0.94, 0.99 ms; interleaved with 4, 8, 32 or
// 64 rows per wave 1.18, 1.00, 0.89, 1.08 ms.

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"

namespace sk {
namespace {

constexpr int kCols = 256;        // columns per wave: four per lane
constexpr int kRowsPerWave = 16;  // every fourth row of a 64-row block
// LDS row stride of the staged y points: odd, so that the lanes' rows (one
// column per lane) fall in distinct banks
template <int D>
constexpr int kYStride = D | 1;

template <int PREC>  // 0: float32, 1: bf16, 2: fp16
__device__ __forceinline__ float round_input(float v) {
  if constexpr (PREC == 1) return (float)(__bf16)v;
  if constexpr (PREC == 2) return (float)(_Float16)v;
  return v;
}

template <int PREC, int D>
__global__ __launch_bounds__(256) void gram_rows_kernel(const GramArgs a, int32_t row_groups,
                                                         int32_t col_chunks) {
  __shared__ float ys[(kCols + 1) * kYStride<D>];   // the chunk's points
  __shared__ float xs_all[4][kRowsPerWave * D];      // each wave's x increments
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // workgroup -> (pair, 64-row block, column chunk), column chunks adjacent
  const int64_t b = blockIdx.x;
  const int64_t per_pair = (int64_t)col_chunks * row_groups;
  const int64_t pair = b / per_pair;
  const int32_t rest = (int32_t)(b - pair * per_pair);
  const int32_t rg = rest / col_chunks, cc = rest - rg * col_chunks;
  const int64_t ia = a.gram ? pair / a.ny : pair;
  const int64_t ib = a.gram ? pair - ia * a.ny : pair;
  const int32_t m = a.x_len - 1, n = a.y_len - 1;
  const int32_t cbase = cc * kCols;
  const int32_t cw = n - cbase < kCols ? n - cbase : kCols;

  const float* __restrict__ yq = a.y + (ib * (int64_t)a.y_len + cbase) * D;
  for (int32_t e = threadIdx.x; e < (cw + 1) * D; e += 256) {
    const int32_t r = e / D;
    ys[r * kYStride<D> + (e - r * D)] = yq[e];
  }
  __syncthreads();  // the only barrier: waves without rows may leave after it

  // the wave's rows: p0 + 4 i for i < nr
  const int32_t p0 = rg * 4 * kRowsPerWave + wid;
  if (p0 >= m) return;
  int32_t nr = (m - p0 + 3) / 4;
  if (nr > kRowsPerWave) nr = kRowsPerWave;

  float dy[4][D];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int32_t c = lane + 64 * j;
    const bool ok = c < cw;
#pragma unroll
    for (int k = 0; k < D; ++k)
      dy[j][k] = ok ? round_input<PREC>(ys[(c + 1) * kYStride<D> + k] - ys[c * kYStride<D> + k])
                    : 0.0f;
  }

  // the wave's x increments, [i][k]
  float* xs = xs_all[wid];
  const float* __restrict__ xb = a.x + (ia * (int64_t)a.x_len + p0) * D;
  for (int32_t e = lane; e < nr * D; e += 64) {
    const int32_t i = e / D, k = e - i * D;
    const int32_t o = 4 * i * D + k;
    xs[e] = round_input<PREC>(xb[o + D] - xb[o]);
  }
  __builtin_amdgcn_wave_barrier();

  float* __restrict__ g = a.g0 + (pair * (int64_t)m + p0) * a.ld + cbase;
  for (int32_t i = 0; i < nr; ++i) {
    float dx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) dx[k] = xs[i * D + k];
    float* __restrict__ row = g + (int64_t)(4 * i) * a.ld;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float acc = dx[0] * dy[j][0];
#pragma unroll
      for (int k = 1; k < D; ++k) acc = __builtin_fmaf(dx[k], dy[j][k], acc);
      const int32_t c = lane + 64 * j;
      if (c < cw) row[c] = acc;
    }
  }
}

template <int PREC, int D>
void launch_d(const GramArgs& a, dim3 grid, int32_t row_groups, int32_t col_chunks,
              hipStream_t stream) {
  hipLaunchKernelGGL((gram_rows_kernel<PREC, D>), grid, dim3(256), 0, stream, a, row_groups,
                     col_chunks);
}

template <int PREC>
hipError_t launch_prec(const GramArgs& a, dim3 grid, int32_t row_groups, int32_t col_chunks,
                       hipStream_t stream) {
  switch (a.d) {
#define SK_GRAM_ROWS_D(N) \
  case N: launch_d<PREC, N>(a, grid, row_groups, col_chunks, stream); break;
    SK_GRAM_ROWS_D(1) SK_GRAM_ROWS_D(2) SK_GRAM_ROWS_D(3) SK_GRAM_ROWS_D(4)
    SK_GRAM_ROWS_D(5) SK_GRAM_ROWS_D(6) SK_GRAM_ROWS_D(7) SK_GRAM_ROWS_D(8)
    SK_GRAM_ROWS_D(9) SK_GRAM_ROWS_D(10) SK_GRAM_ROWS_D(11) SK_GRAM_ROWS_D(12)
    SK_GRAM_ROWS_D(13) SK_GRAM_ROWS_D(14) SK_GRAM_ROWS_D(15) SK_GRAM_ROWS_D(16)
#undef SK_GRAM_ROWS_D
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gram_rows(const GramArgs& a, int precision, hipStream_t stream) {
  const int32_t m = a.x_len - 1, n = a.y_len - 1;
  const int64_t pairs = a.gram ? a.nx * a.ny : a.nx;
  if (m <= 0 || n <= 0 || pairs == 0) return hipSuccess;
  if (a.ld < n || a.d < 1 || a.d > kGramRowsMaxDim) return hipErrorInvalidValue;
  const int32_t row_groups = (m + 4 * kRowsPerWave - 1) / (4 * kRowsPerWave);
  const int32_t col_chunks = (n + kCols - 1) / kCols;
  const int64_t blocks = pairs * col_chunks * row_groups;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks, 1, 1);
  if (precision == kRoundBf16) return launch_prec<1>(a, grid, row_groups, col_chunks, stream);
  if (precision == kRoundF16) return launch_prec<2>(a, grid, row_groups, col_chunks, stream);
  return launch_prec<0>(a, grid, row_groups, col_chunks, stream);
}

}  // namespace sk
