// Launchers of the adjoint sweep (sweep_bwd_kernel.h) and the reduction of
// increment gradients into point gradients.
#include "internal.h"

namespace sk {
namespace {

// Increment gradients -> point gradients of one batch, with the deterministic
// reductions over runs (x side) and over the other batch (y side):
//   dinc[k][p] = scale * sum_j part_x[k runs + j][p]            (row side)
//              + sum_{a} part_y[a][k][p]                          (column side)
//   dpts[k][i] = dinc[k][i-1] - dinc[k][i]   (x_i enters x_i - x_{i-1} and x_{i+1} - x_i)
__global__ __launch_bounds__(256) void point_grad_kernel(
    const float* __restrict__ part_x, int64_t runs_per_row, float scale,
    const float* __restrict__ part_y, int64_t part_y_rows, int64_t part_y_ld, int32_t col_upper,
    float yscale, int32_t rep, int64_t n_paths, int32_t len, int32_t d,
    float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = n_paths * len * d;
  if (e >= total) return;
  const int c = (int)(e % d);
  const int64_t i = (e / d) % len;
  const int64_t k = e / ((int64_t)d * len);
  const int32_t ninc = len - 1;
  const int64_t nrows = (int64_t)ninc * rep;  // rows per path of the partial gradients
  auto inc = [&](int64_t p) -> float {
    if (p < 0 || p >= ninc) return 0.0f;
    float accx = 0.0f, accy = 0.0f;
    for (int64_t r = p * rep; r < (p + 1) * rep; ++r) {
      if (part_x)
        for (int64_t j = 0; j < runs_per_row; ++j)
          accx += part_x[((k * runs_per_row + j) * nrows + r) * d + c];
      if (part_y) {
        const int64_t aend = col_upper ? k + 1 : part_y_rows;
        for (int64_t a2 = 0; a2 < aend; ++a2)
          accy += part_y[((a2 * part_y_ld + k) * nrows + r) * d + c];
      }
    }
    return accx * scale + accy * yscale;
  };
  out[e] = inc(i - 1) - inc(i);
}

}  // namespace

hipError_t launch_adjoint(const BwdArgs& a, int lam, int R, int d, hipStream_t stream,
                          int wpb) {
  auto f = reinterpret_cast<void (*)(const BwdArgs)>(sweep_fn(kKernelAdjoint, lam, R, d));
  if (!f) return hipErrorInvalidValue;
  if (a.n_waves == 0) return hipSuccess;
  if (wpb != 1 && wpb != 2) wpb = 4;  // the kernel is bounded to 256 threads
  const int64_t blocks = (a.n_waves + wpb - 1) / wpb;
  hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(64 * wpb), 0, stream, a);
  return hipGetLastError();
}

bool adjoint_supported(int R, int lam, int d) {
  return sweep_fn(kKernelAdjoint, lam, R, d) != nullptr;
}

hipError_t launch_point_grad(const float* part_x, int64_t runs_per_row, float scale,
                             const float* part_y, int64_t part_y_rows, int64_t part_y_ld,
                             bool col_upper, float yscale, int32_t rep, int64_t n_paths,
                             int32_t len, int32_t d, float* out, hipStream_t stream) {
  const int64_t total = n_paths * len * d;
  if (total == 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(point_grad_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, part_x,
                     runs_per_row, scale, part_y, part_y_rows, part_y_ld, col_upper ? 1 : 0,
                     yscale, rep, n_paths, len, d, out);
  return hipGetLastError();
}

}  // namespace sk
