// Argument block and stream geometry of the forward sweeps (the one-wave Gram
// sweep and the lifted sweep), kept apart from the other internal
// declarations so that the sweep kernels compile from this file, their own
// headers and nothing else of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

// Work description of one forward sweep launch.
struct SweepArgs {
  const float* incx;        // dense increments of the x side, pre-scaled by 2^-(2 lam + 1)
                            // (lifted sweep: dense node rows of x, not scaled)
  const float* incy;        // dense increments of the y side (lifted sweep: node rows of y)
  const int32_t* x_n;       // ragged plans (nullptr for a uniform batch)
  const int64_t* x_start;
  const int32_t* y_n;
  const int64_t* y_start;
  int32_t x_len, y_len;     // points per path of a uniform batch
  int64_t nx, ny;           // paths per batch
  int32_t mode;             // 0: pairs (x_k, y_k); 1: Gram; 2: Gram upper triangle, mirrored
  int32_t no_diag;          // mode 2: diagonal written as 0
  int32_t implicit;         // 1: the implicit scheme's cell factor (2 + h) / (2 - h)
  double lift_inv;          // lifted sweep: 1 / (2 sigma^2) of the Gaussian static kernel
  double lift_scale;        // lifted sweep: 2^-(2 lam + 1), the coefficient's fine-cell factor
  int32_t run;              // pairs streamed through one wave (Gram with uniform y)
  int64_t runs_per_row;     // ceil(ny / run)
  int32_t tri;       // mode 2: waves enumerate only the runs of the upper triangle
                     // (tri_runs): 1 with the diagonal, 2 without it
  int64_t n_waves;
  float* out;               // nullptr: terminal values not written
  int64_t out_ld;           // ny for the Gram
  // waves [wave0, wave0 + n_waves) of the run enumeration are launched
  int64_t wave0;
  // coefficient sweep: per launched wave, coef_stride floats of pre-scaled
  // coarse coefficients in step order ([step][lane][coarse row of the strip])
  const float* coef;
  int64_t coef_stride;
};

// Rows before and after the data of every dense increment buffer: a wave
// streams rows g - lane for lanes 0..63 and prefetches two rows ahead, so it
// reads rows -63 .. total + 66 of a run (steps are rounded up to a multiple
// of three).
constexpr int64_t kStreamPad = 128;

// Steps of a wave that streams `total` coarse columns (a multiple of three:
// the y-row prefetch rotates three buffers).
__host__ __device__ inline int64_t sweep_steps(int64_t total) {
  return ((total + 63 + 2) / 3) * 3;
}

// The upper triangle of a symmetric Gram by runs: row i (x_i) takes the y
// columns from i + s on (s = 0 with the diagonal, 1 without it) in runs that
// start at multiples of `run`, the one holding column i + s clipped to start
// there, so it holds runs_per_row - floor((i + s) / run) runs (rows
// i < nx - s; without the diagonal the last row has none).  Waves enumerated
// over these alone (no wave without a pair) are spread evenly over the
// compute units; tri_runs(i) counts the runs of rows 0 .. i-1:
//   i runs_per_row - sum_{j < i + s} floor(j / run).
__host__ __device__ inline int64_t tri_runs(int64_t i, int64_t runs_per_row, int64_t run,
                                            int64_t s = 0) {
  const int64_t x = i + s, q = x / run, r = x - q * run;
  return i * runs_per_row - (run * q * (q - 1) / 2 + q * r);
}

}  // namespace sk
