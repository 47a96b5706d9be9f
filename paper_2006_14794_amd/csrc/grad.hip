// Launchers of the Gram gradient kernel (grad_kernel.h) and the reduction of
// its increment gradients into point gradients.
#include "internal.h"

namespace sk {

void* grad_fn_l0_(int d, bool ys);
void* grad_fn_l1_(int d, bool ys);
void* grad_fn_l2_(int d, bool ys);
void* grad_fn_l3_(int d, bool ys);

void* grad_fn(int lam, int d, bool ys) {
  switch (lam) {
    case 0: return grad_fn_l0_(d, ys);
    case 1: return grad_fn_l1_(d, ys);
    case 2: return grad_fn_l2_(d, ys);
    case 3: return grad_fn_l3_(d, ys);
    default: return nullptr;
  }
}

namespace {

__global__ void zero_i32_kernel(int32_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// Point gradients of one batch from the increment gradients of a Gram
// gradient launch, in double, each sum in a fixed order (deterministic):
//   dinc[k][p] = xscale sum_j part_x[k][j][rows of p]          (x side, j < runs)
//              + yscale sum_a part_y[a][k][rows of p]           (y side)
//   dP[k][i]  = dinc[k][i - 1] - dinc[k][i]   (x_i enters x_i - x_{i-1} and x_{i+1} - x_i)
// The rows of increment p are p rep .. p rep + rep - 1 (a batch split rep
// times for orders above the compiled ones).  col_upper: the y side of a
// symmetric Gram, only a <= k is stored.  One thread per point row i and
// channel: it forms dinc for its own increment (the one starting at x_i) and
// takes dinc[k][i - 1] from the thread of row i - 1 through LDS (the block's
// first row computes that one itself), so each sum is formed once; ragged
// batches find a row's path by bisection of the offsets, and a row that lies
// in no valid path gets NaN.  With accumulate the gradient is added to the
// output (float32 sum of the stored value and the double one).
__global__ __launch_bounds__(256) void grad_points_kernel(const GradPointArgs a) {
  __shared__ double own[256];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = a.offsets ? a.offsets[a.n_paths] : a.n_paths * (int64_t)a.len;
  const bool in_range = e < a.rows_bound * a.d && e / a.d < rows;
  const int64_t i = e / a.d;
  const int c = (int)(e - i * a.d);
  int64_t k = 0, il = 0;
  int32_t ninc = 0;
  bool valid = in_range;
  if (in_range && a.offsets) {
    int64_t lo = 0, hi = a.n_paths - 1;  // last k with offsets[k] <= i
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (a.offsets[mid] <= i) lo = mid; else hi = mid - 1;
    }
    k = lo;
    il = i - a.offsets[k];
    ninc = a.plan_n[k];  // of the batch as swept: rep times the path's increments
    if (ninc < 0 || il < 0 || i >= a.offsets[k + 1])
      valid = false;
    else
      ninc /= a.rep;
  } else if (in_range) {
    k = i / a.len;
    il = i - k * a.len;
    ninc = a.len - 1;
  }
  auto inc = [&](int64_t p) -> double {
    if (p < 0 || p >= ninc) return 0.0;
    double accx = 0.0, accy = 0.0;
    for (int64_t r = p * a.rep; r < (p + 1) * a.rep; ++r) {
      if (a.part_x) {
#pragma unroll 8
        for (int64_t j = 0; j < a.runs_per_row; ++j)
          accx += a.part_x[((k * a.runs_per_row + j) * a.mrows + r) * a.d + c];
      }
      if (a.part_y) {
        const int64_t aend = a.col_upper ? k + 1 : a.py_rows;
#pragma unroll 8
        for (int64_t a2 = 0; a2 < aend; ++a2)
          accy += a.part_y[((a2 * a.py_ld + k) * a.nrows + r) * a.d + c];
      }
    }
    return accx * a.xscale + accy * a.yscale;
  };
  const double mine = valid ? inc(il) : 0.0;
  own[threadIdx.x] = mine;
  __syncthreads();
  if (!in_range) return;
  if (!valid) {
    a.out[e] = __builtin_nanf("");
    return;
  }
  // dinc[k][il - 1]: row i - 1's own sum (same path when il > 0), held by
  // thread e - d of this block, else formed here
  double prev = 0.0;
  if (il > 0) prev = (int)threadIdx.x >= a.d ? own[threadIdx.x - a.d] : inc(il - 1);
  const double g = prev - mine;
  a.out[e] = a.accumulate ? (float)((double)a.out[e] + g) : (float)g;
}


}  // namespace

bool grad_supported(int lam, int d) { return grad_fn(lam, d, true) != nullptr; }

hipError_t launch_grad(const GradArgs& a, int lam, int d, bool ys, int64_t slots,
                       hipStream_t stream) {
  auto f = reinterpret_cast<void (*)(const GradArgs)>(grad_fn(lam, d, ys));
  if (!f) return hipErrorInvalidValue;
  if (a.n_tasks <= 0 || slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, stream, a.counter, 1);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  // one wave per workgroup: slot = workgroup; every slot's scratch is its own,
  // so any number of them may be resident at once
  hipLaunchKernelGGL(f, dim3((unsigned)slots), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_grad_points(const GradPointArgs& a, hipStream_t stream) {
  const int64_t total = a.rows_bound * a.d;
  if (total == 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(grad_points_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace sk
