// Sweep of the explicit (or implicit) scheme driven by precomputed coarse
// coefficients, for any number of channels.
//
// The fused sweeps (sweep_fwd_kernel.h) keep each lane's x increments in
// registers, which bounds the channels they take.  For wider paths the
// coarse increment Gram (Section 3.1: G0[p][q] = <dx_p, dy_q>) is formed
// first, a dense contraction over the channels on the matrix cores, and
// written in the order the sweep consumes it:
//   * coef_kernel<PREC> computes 32 x 32 tiles of G0 with v_mfma_f32_32x32x2_f32
//     (float32 increments) or v_mfma_f32_32x32x16_{bf16,f16} (16-bit inputs,
//     float32 sums), staging 32 channels of 32 rows and 128 columns in LDS per
//     step, and stores each value, scaled by the fine-cell factor
//     2^-(2 lambda + 1) (times 1 / rep^2 on a refined batch), at the step and
//     lane where the sweep uses it: wave-step t = g + lane of the run's column
//     stream g, slot (lane, coarse row of the strip).  One step of one wave
//     then reads 64 x CR consecutive floats.
//   * coef_sweep_kernel<R, LAM, IMPL> is the one-wave sweep with the
//     inner products replaced by those loads (prefetched two steps ahead).
// Dyadic orders beyond 3 (a batch refined rep times): G0 of coarse cell
// (p, q) fills the rep x rep refined cells (p rep + i, q rep + j).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"
#include "sweep_fwd_kernel.h"

namespace sk {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kKC = 32;    // channels staged per step
constexpr int kCols = 128; // columns per workgroup (four 32-column tiles)

using fwd::cell_block;
using fwd::first_row;
using fwd::from_prev_lane;
using fwd::implicit_factors;
using fwd::n_inc;
using fwd::store_out;
using fwd::wave_run;

// Lane of the one-wave strip layout that owns refined coarse row p of an
// m-row grid, and the row's index within the lane's CR rows: strips are
// aligned to the bottom, lane l holding rows [m - (64 - l) CR, m - (63 - l) CR).
__device__ __forceinline__ int strip_lane(int32_t m, int32_t p, int32_t cr) {
  return 64 - (m - p + cr - 1) / cr;
}

template <int PREC>  // 0: float32, 1: bf16, 2: fp16
__global__ __launch_bounds__(256) void coef_kernel(const CoefArgs a) {
  __shared__ float xs[32][kKC + 1];
  __shared__ float ys[kCols][kKC + 1];
  const int64_t slot = blockIdx.x;
  const int64_t wl = slot / a.run;
  const int32_t j = (int32_t)(slot - wl * a.run);
  const int64_t w = a.wave0 + wl;
  // the pair of this slot, enumerated as the sweep's wave_run does
  int64_t ia, b;
  if (a.mode == 0) {
    if (j > 0) return;
    ia = w;
    b = w;
  } else {
    ia = w / a.runs_per_row;
    int64_t b0 = (w - ia * a.runs_per_row) * a.run;
    const int64_t b1 = b0 + a.run < a.ny ? b0 + a.run : a.ny;
    if (a.mode == 2 && b0 < ia) b0 = ia;
    b = b0 + j;
    if (b >= b1) return;
  }
  // refined counts (the sweep's) and the unrefined ones of the increments
  const int32_t mr = n_inc(a.x_n, a.x_len, ia), nr = n_inc(a.y_n, a.y_len, b);
  if (mr <= 0 || nr <= 0 || ((int64_t)mr << a.lam) > 64 * (int64_t)a.R) return;
  const int32_t rep = a.rep;
  const int32_t m = mr / rep, n = nr / rep;
  const int32_t p_base = blockIdx.y * 32, q_base = blockIdx.z * kCols;
  if (p_base >= m || q_base >= n) return;
  const int64_t xrow = a.x_start ? a.x_start[ia] / rep : ia * (int64_t)m;
  const int64_t yrow = a.y_start ? a.y_start[b] / rep : b * (int64_t)n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row = lane & 31, half = lane >> 5;

  f32x16 acc = {};
  for (int k0 = 0; k0 < a.d; k0 += kKC) {
    __syncthreads();  // the previous step's tiles are consumed
    for (int e = threadIdx.x; e < 32 * kKC; e += blockDim.x) {
      const int r = e / kKC, k = e - r * kKC;
      xs[r][k] = (p_base + r < m && k0 + k < a.d)
                     ? a.incx[(xrow + p_base + r) * a.dpad + k0 + k]
                     : 0.0f;
    }
    for (int e = threadIdx.x; e < kCols * kKC; e += blockDim.x) {
      const int c = e / kKC, k = e - c * kKC;
      ys[c][k] = (q_base + c < n && k0 + k < a.d)
                     ? a.incy[(yrow + q_base + c) * a.dpad + k0 + k]
                     : 0.0f;
    }
    __syncthreads();
    const int col = wid * 32 + row;
    if constexpr (PREC == 0) {
#pragma unroll
      for (int kk = 0; kk < kKC; kk += 2)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xs[row][kk + half], ys[col][kk + half], acc,
                                                    0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < kKC; kk += 16) {
        if constexpr (PREC == 1) {
          bf16x8 A, B;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            A[t] = (__bf16)xs[row][kk + half * 8 + t];
            B[t] = (__bf16)ys[col][kk + half * 8 + t];
          }
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc, 0, 0, 0);
        } else {
          f16x8 A, B;
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            A[t] = (_Float16)xs[row][kk + half * 8 + t];
            B[t] = (_Float16)ys[col][kk + half * 8 + t];
          }
          acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, B, acc, 0, 0, 0);
        }
      }
    }
  }

  // accumulator register r of this lane: row 8 (r / 4) + 4 half + (r mod 4),
  // column row (the MFMA output layout)
  const int32_t cr = a.R >> a.lam;
  const int32_t q = q_base + wid * 32 + row;
  if (q >= n) return;
  float* __restrict__ base = a.coef + wl * a.coef_stride;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int32_t p = p_base + 8 * (r >> 2) + 4 * half + (r & 3);
    if (p >= m) continue;
    const float v = acc[r] * a.scale;
    for (int32_t i = 0; i < rep; ++i) {
      const int32_t pr = p * rep + i;
      const int l2 = strip_lane(mr, pr, cr);
      const int32_t c = pr - (mr - (64 - l2) * cr);
      for (int32_t jj = 0; jj < rep; ++jj) {
        const int64_t t = (int64_t)j * nr + (int64_t)q * rep + jj + l2;
        base[(t * 64 + l2) * cr + c] = v;
      }
    }
  }
}

// The one-wave sweep of sweep_fwd_kernel.h with the coarse coefficients read
// from the layout coef_kernel writes.  R >= 2^LAM: every coarse row belongs to
// one lane.  Rows above the grid (virtual rows of the top strip) take
// coefficient 0 without reading.
template <int R, int LAM, bool IMPL>
__global__ __launch_bounds__(256) void coef_sweep_kernel(const SweepArgs a) {
  constexpr int S = 1 << LAM;
  constexpr int CR = R >> LAM;
  static_assert(CR >= 1, "a coarse row must not span lanes");

  const int lane = threadIdx.x & 63;
  const int64_t w = a.wave0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= a.wave0 + a.n_waves) return;
  int64_t ia, b0, b1, total;
  int32_t m;
  if (!wave_run(a, w, lane, 64 * R, LAM, ia, b0, b1, m, total)) return;
  const int32_t p0 = m - (64 - lane) * CR;  // negative rows are virtual
  const int32_t total32 = (int32_t)total;
  const int32_t cn = n_inc(a.y_n, a.y_len, b0);
  int32_t g = -lane;
  int32_t q = 0;
  // wave-step t of this lane's slot: cp + t 64 CR
  const float* __restrict__ cp = a.coef + (w - a.wave0) * a.coef_stride + lane * CR;

  double u[R];
#pragma unroll
  for (int r = 0; r < R; ++r) u[r] = 1.0;
  double pub[S], up[S];
#pragma unroll
  for (int cc = 0; cc < S; ++cc) {
    pub[cc] = 1.0;
    up[cc] = 1.0;
  }
  double up_last = 1.0;
  bool real[CR];
#pragma unroll
  for (int c = 0; c < CR; ++c) real[c] = p0 + c >= 0;

  float cA[CR], cB[CR], cC[CR];
#pragma unroll
  for (int c = 0; c < CR; ++c) {
    cA[c] = cp[c];
    cB[c] = cp[64 * CR + c];
  }
  const int32_t nsteps = (int32_t)sweep_steps(total);
  auto step = [&](float (&cur)[CR], float (&refill)[CR]) {
#pragma unroll
    for (int c = 0; c < CR; ++c) refill[c] = cp[2 * 64 * CR + c];
#pragma unroll
    for (int cc = 0; cc < S; ++cc) up[cc] = from_prev_lane(pub[cc], up[cc]);
    if ((uint32_t)g < (uint32_t)total32) {
      double gk[CR], h[CR];
#pragma unroll
      for (int c = 0; c < CR; ++c) h[c] = real[c] ? (double)cur[c] : 0.0;
      if constexpr (IMPL) {
        implicit_factors<CR>(h, gk);
      } else {
#pragma unroll
        for (int c = 0; c < CR; ++c) gk[c] = 1.0 + h[c];
      }
      double v[R][S];
      float sv[1];
      cell_block<R, LAM, CR, false>(v, sv, u, up, up_last, gk);
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[r][S - 1];
#pragma unroll
      for (int cc = 0; cc < S; ++cc) pub[cc] = v[R - 1][cc];
      up_last = up[S - 1];
      if (++q == cn) {
        if (lane == 63) {
          const int64_t cb = b0 + g / cn;
          store_out(a, ia, cb, (a.mode == 2 && a.no_diag && cb == ia) ? 0.0f : (float)u[R - 1]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = 1.0;
        up_last = 1.0;
        q = 0;
      }
    }
    ++g;
    cp += 64 * CR;
  };
  for (int32_t t = 0; t < nsteps; t += 3) {
    step(cA, cC);
    step(cB, cA);
    step(cC, cB);
  }
}

using SweepFn = void (*)(const SweepArgs);

template <int R, int LAM>
SweepFn pick_impl(bool implicit) {
  if constexpr ((R >> LAM) >= 1)
    return implicit ? &coef_sweep_kernel<R, LAM, true> : &coef_sweep_kernel<R, LAM, false>;
  else
    return nullptr;
}

template <int R>
SweepFn pick_lam(int lam, bool implicit) {
  switch (lam) {
    case 0: return pick_impl<R, 0>(implicit);
    case 1: return pick_impl<R, 1>(implicit);
    case 2: return pick_impl<R, 2>(implicit);
    case 3: return pick_impl<R, 3>(implicit);
    default: return nullptr;
  }
}

SweepFn coef_sweep_fn(int R, int lam, bool implicit) {
  switch (R) {
    case 1: return pick_lam<1>(lam, implicit);
    case 2: return pick_lam<2>(lam, implicit);
    case 4: return pick_lam<4>(lam, implicit);
    case 8: return pick_lam<8>(lam, implicit);
    case 16: return pick_lam<16>(lam, implicit);
    case 32: return pick_lam<32>(lam, implicit);
    default: return nullptr;
  }
}

}  // namespace

int coef_rows_per_lane(int64_t fine_rows, int lam) {
  for (int R = 1; R <= kMaxRowsPerLane; R *= 2)
    if (R >= (1 << lam) && 64 * (int64_t)R >= fine_rows) return R;
  return 0;
}

int64_t coef_wave_floats(int64_t total_cols, int R, int lam) {
  // the sweep's steps plus its two-step prefetch
  return (sweep_steps(total_cols) + 2) * 64 * (int64_t)(R >> lam);
}

hipError_t launch_coef(const CoefArgs& a, int precision, int64_t max_m, int64_t max_n,
                       hipStream_t stream) {
  if (a.n_waves == 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  const int64_t slots = a.n_waves * a.run;
  const int64_t rb = (max_m + 31) / 32, cb = (max_n + kCols - 1) / kCols;
  if (slots > 0x7FFFFFFF || rb > 65535 || cb > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)slots, (unsigned)rb, (unsigned)cb);
  if (precision == kRoundBf16)
    hipLaunchKernelGGL(coef_kernel<1>, grid, dim3(256), 0, stream, a);
  else if (precision == kRoundF16)
    hipLaunchKernelGGL(coef_kernel<2>, grid, dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(coef_kernel<0>, grid, dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_coef_sweep(const SweepArgs& a, int lam, int R, bool implicit,
                             hipStream_t stream, int wpb) {
  const SweepFn f = coef_sweep_fn(R, lam, implicit);
  if (!f) return hipErrorInvalidValue;
  if (a.n_waves == 0) return hipSuccess;
  if (wpb != 1 && wpb != 2) wpb = 4;
  const int64_t blocks = (a.n_waves + wpb - 1) / wpb;
  hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(64 * wpb), 0, stream, a);
  return hipGetLastError();
}

}  // namespace sk
