// Unbiased signature-kernel MMD^2 (the estimator mentioned at the end of
// Section 3.1.1): the U-statistic
//   MMD^2 = sum_{a != b} Kxx[a][b] / (n (n - 1)) + sum_{a != b} Kyy[a][b] / (m (m - 1))
//           - 2 sum_{a, b} Kxy[a][b] / (n m),
// reduced in a fixed order by one workgroup, plus the helpers its gradient
// needs (constant upstream weights, sum of two gradients).
#include "internal.h"

namespace sk {
namespace {

// Kxx and Kyy carry zeros on their diagonals (unbiased Grams).
__global__ __launch_bounds__(1024) void mmd2_reduce_kernel(
    const float* __restrict__ kxx, int64_t n, const float* __restrict__ kyy, int64_t m,
    const float* __restrict__ kxy, float* __restrict__ out) {
  __shared__ double part[3][16];
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < n * n; i += blockDim.x) s[0] += kxx[i];
  for (int64_t i = threadIdx.x; i < m * m; i += blockDim.x) s[1] += kyy[i];
  for (int64_t i = threadIdx.x; i < n * m; i += blockDim.x) s[2] += kxy[i];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    for (int o = 32; o > 0; o >>= 1) s[j] += __shfl_down(s[j], o, 64);
    if (lane == 0) part[j][wid] = s[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < 3; ++j)
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t[j] += part[j][w];
    const double v = t[0] / ((double)n * (double)(n - 1)) +
                     t[1] / ((double)m * (double)(m - 1)) -
                     2.0 * t[2] / ((double)n * (double)m);
    out[0] = (float)v;
  }
}

__global__ __launch_bounds__(256) void add_kernel(float* __restrict__ dst,
                                                  const float* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

__global__ __launch_bounds__(256) void zero_diag_kernel(float* __restrict__ k, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) k[i * n + i] = 0.0f;
}

}  // namespace

hipError_t launch_zero_diag(float* k, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                     k, n);
  return hipGetLastError();
}

hipError_t launch_mmd2_reduce(const float* kxx, int64_t n, const float* kyy, int64_t m,
                              const float* kxy, float* out, hipStream_t stream) {
  hipLaunchKernelGGL(mmd2_reduce_kernel, dim3(1), dim3(1024), 0, stream, kxx, n, kyy, m, kxy,
                     out);
  return hipGetLastError();
}

hipError_t launch_add(float* dst, const float* src, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, dst, src, n);
  return hipGetLastError();
}

}  // namespace sk
