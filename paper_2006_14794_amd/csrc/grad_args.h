// Argument block and scratch geometry of the Gram gradient kernel
// (grad_kernel.h), kept apart so that the kernel compiles from this file, the
// forward sweep's header and nothing else of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

// Work description of one gradient launch.  A task is a run of pairs
// (x_ia, y_b), b in [b0, b1), sharing the x path (uniform y batches), or one
// pair taken from `order` (ragged batches).
struct GradArgs {
  const float* incx;        // dense x increments, pre-scaled by 2^-(2 lam + 1)
  const float* incy;        // dense y increments
  const int32_t* x_n;       // ragged plans (nullptr for a uniform batch)
  const int64_t* x_start;
  const int32_t* y_n;
  const int64_t* y_start;
  int32_t x_len, y_len;     // points per path as swept (upper bounds when ragged)
  int64_t nx, ny;
  int32_t mode;             // 1: every pair; 2: upper triangle of a symmetric Gram
  int32_t no_diag;          // mode 2: the diagonal is the constant 0 (no gradient)
  int32_t run;              // pairs per task of a uniform y batch
  int64_t runs_per_row;     // tasks per x path (ny when `order` is set)
  int32_t n_tasks;
  const int32_t* order;     // ragged: task t is pair order[t] = a ny + b; nullptr: runs
  int32_t* counter;         // queue head, zeroed before the launch
  const float* dK;          // [nx][ny] upstream weights
  float* K;                 // [nx][ny] forward values (nullptr: not written)
  double* scratch;          // per wave slot: slot_stride doubles (grad_slot_layout)
  int64_t slot_stride;
  int32_t nb_max;           // row bands of the tallest x path
  int32_t nseg_max;         // segments of the longest task
  int64_t cols_max;         // coarse columns of the longest task
  double* part_x;           // [nx][runs_per_row][mrows][dim]: x-side increment gradients
  double* part_y;           // [nx][ny][nrows][dim]: y-side increment gradients
  int32_t mrows, nrows;     // x_len - 1, y_len - 1
};

// Fine rows per lane of the gradient kernel: bands of 64 R rows.
constexpr int kGradRows = 4;

// Forward steps per segment: the adjoint recomputes a segment from its
// checkpoint and keeps the segment's R 2^lam cell sums per step on chip, the
// first grad_lds_steps steps in LDS (64 floats per lane: 16 KB per wave) and
// the rest in registers (32 floats per lane; half that at order 0, whose
// increments and gradient accumulators take more registers).
__host__ __device__ constexpr int grad_reg_steps(int lam, int d) {
  const int rs = kGradRows << lam;
  // order 0 keeps four coarse rows per lane (increments, accumulators)
  const int floats = 32 / (lam == 0 ? 2 : 1) + 0 * d;
  const int c = floats / rs;
  return c < 1 ? 1 : c;
}
__host__ __device__ constexpr int grad_lds_steps(int lam) {
  const int c = 64 / (kGradRows << lam);
  return c < 1 ? 1 : c;
}
__host__ __device__ constexpr int grad_segment(int lam, int d) {
  return grad_reg_steps(lam, d) + grad_lds_steps(lam);
}

// Doubles of the wave state saved per lane at a checkpoint: the lane's first
// R - 1 values at its last fine column, its bottom row at the 2^lam fine
// columns of its last step (whose last entry is the R-th value, unless that
// column ended a pair and the values restarted at 1), and the upper-left
// neighbour of its next block.
__host__ __device__ constexpr int grad_state_doubles(int lam) {
  return kGradRows + (1 << lam);
}

// Scratch of one wave slot, in doubles:
//   checkpoints  [nb_max][nseg_max - 1][state][64 lanes]   (segment 0 starts from the boundary)
//   hand_f       [nb_max - 1][cols_max << lam]             forward: bottom rows of the bands
//   hand_a       [2][cols_max + 1][2^lam + 1]              adjoint: a values of a band's top
//                                                         row and its first coarse row's
//                                                         coefficient, for the band above
struct GradSlot {
  int64_t ckpt, hand_f, hand_a, stride;
};
__host__ __device__ inline GradSlot grad_slot_layout(int lam, int nb_max, int nseg_max,
                                                     int64_t cols_max) {
  GradSlot s{};
  const int64_t S = int64_t(1) << lam;
  s.ckpt = 0;
  s.hand_f = (int64_t)nb_max * (nseg_max - 1) * grad_state_doubles(lam) * 64;
  s.hand_a = s.hand_f + (int64_t)(nb_max - 1) * cols_max * S;
  s.stride = s.hand_a + 2 * (cols_max + 1) * (S + 1);
  s.stride = (s.stride + 31) & ~int64_t(31);  // 256-byte aligned slots
  return s;
}

}  // namespace sk
