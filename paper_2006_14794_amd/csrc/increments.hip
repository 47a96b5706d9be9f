// Increments of piecewise-linear paths (Section 3.1: on each coarse cell the
// PDE coefficient is the inner product of the two segment increments), laid
// out densely: the increments of consecutive paths are consecutive rows, so a
// sweep that streams several y paths reads one contiguous row range.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"

namespace sk {
namespace {

// Ragged batch plan: validate every path and prefix-sum the increment counts.
// One workgroup of 1024 threads walks the paths in chunks with a running carry.
__global__ __launch_bounds__(1024) void plan_kernel(const int64_t* __restrict__ off,
                                                    int32_t len, int64_t n_paths,
                                                    int32_t* __restrict__ n_out,
                                                    int64_t* __restrict__ start_out) {
  __shared__ int64_t warp_sums[16];
  __shared__ int64_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // the points buffer holds off[n_paths] rows; offsets that do not start at 0
  // break the contract for every path
  const int64_t end = off[n_paths];
  const bool first_ok = off[0] == 0;
  for (int64_t base = 0; base < n_paths; base += 1024) {
    const int64_t k = base + threadIdx.x;
    int32_t n = 0;
    if (k < n_paths) {
      const int64_t s = off[k], e = off[k + 1], L = e - s;
      const bool ok = first_ok && s >= 0 && L >= 1 && L <= len && e <= end;
      n = ok ? (int32_t)(L - 1) : -1;
      n_out[k] = n;
    }
    // inclusive scan of max(n, 0) within the wave, then across waves
    int64_t v = n > 0 ? n : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t t = __shfl_up(v, o, 64);
      if (lane >= o) v += t;
    }
    if (lane == 63) warp_sums[wid] = v;
    __syncthreads();
    int64_t before = carry_s;
    for (int w = 0; w < wid; ++w) before += warp_sums[w];
    const int64_t own = n > 0 ? n : 0;
    if (k < n_paths) start_out[k] = before + v - own;
    __syncthreads();
    if (threadIdx.x == 1023) carry_s = before + v;
    __syncthreads();
  }
}

// The increments of one batch (the two batches of a call go in one launch).
struct IncJob {
  const float* pts;
  const int64_t* off;        // ragged offsets, or null
  const int32_t* plan_n;     // ragged plan
  const int64_t* plan_start;
  int32_t len;
  int64_t n_paths;
  int32_t d, dpad;
  float scale;               // includes 1 / rep
  int32_t rounding, rep;
  float* incr;
};

// Path k of a job: one workgroup writes its dense rows [start, start + n).
__device__ __forceinline__ void increments_one(const IncJob& j, int64_t k) {
  const float* __restrict__ pts = j.pts;
  const int64_t* __restrict__ off = j.off;
  const int32_t len = j.len, d = j.d, dpad = j.dpad, rounding = j.rounding, rep = j.rep;
  const float scale = j.scale;
  float* __restrict__ incr = j.incr;
  int64_t pstart, dstart;
  int32_t n;
  if (off) {
    n = j.plan_n[k];
    if (n <= 0) return;
    pstart = off[k];
    dstart = j.plan_start[k] * rep;
  } else {
    n = len - 1;
    pstart = k * (int64_t)len;
    dstart = k * (int64_t)n * rep;
  }
  // increment p fills rows p rep .. p rep + rep - 1 (refinement beyond the
  // sweep's compiled orders: rep equal sub-increments of a straight segment).
  // Element (row, c) of the block's rows, stepped by the block size without
  // divisions; rep is a power of two.
  const int64_t nrows = (int64_t)n * rep;
  const int rs = __builtin_ctz((unsigned)rep);
  const int32_t drow = (int32_t)blockDim.x / dpad, dc = (int32_t)blockDim.x - drow * dpad;
  int64_t row = (int32_t)threadIdx.x / dpad;
  int32_t c = (int32_t)threadIdx.x - (int32_t)row * dpad;
  while (row < nrows) {
    const int64_t p = row >> rs;
    float v = 0.0f;
    if (c < d) {
      const float a = pts[(pstart + p + 1) * d + c];
      const float b = pts[(pstart + p) * d + c];
      v = a - b;
      // 16-bit inputs of the inner products (round to nearest even); the
      // products and their sums stay float32
      if (rounding == kRoundBf16) v = __bfloat162float(__float2bfloat16(v));
      if (rounding == kRoundF16) v = __half2float(__float2half(v));
      v *= scale;  // power-of-two scale (including 1 / rep): exact
    }
    incr[(dstart + row) * dpad + c] = v;
    row += drow;
    c += dc;
    if (c >= dpad) {
      c -= dpad;
      ++row;
    }
  }
}

// Workgroups [0, jx.n_paths) take the paths of jx, the rest those of jy.
__global__ __launch_bounds__(256) void increments_kernel(const IncJob jx, const IncJob jy) {
  const int64_t b = blockIdx.x;
  if (b < jx.n_paths)
    increments_one(jx, b);
  else
    increments_one(jy, b - jx.n_paths);
}

// The same for d a multiple of 4 (then the padded row is the point row and
// both are 16-byte aligned): four channels per thread with 16-byte loads and
// stores, the same arithmetic per element.
__device__ __forceinline__ float increment_value(float a, float b, int32_t rounding,
                                                 float scale) {
  float v = a - b;
  if (rounding == kRoundBf16) v = __bfloat162float(__float2bfloat16(v));
  if (rounding == kRoundF16) v = __half2float(__float2half(v));
  return v * scale;
}

__device__ __forceinline__ void increments4_one(const IncJob& j, int64_t k) {
  const float* __restrict__ pts = j.pts;
  const int64_t* __restrict__ off = j.off;
  const int32_t len = j.len, d = j.d, rounding = j.rounding, rep = j.rep;
  const float scale = j.scale;
  float* __restrict__ incr = j.incr;
  int64_t pstart, dstart;
  int32_t n;
  if (off) {
    n = j.plan_n[k];
    if (n <= 0) return;
    pstart = off[k];
    dstart = j.plan_start[k] * rep;
  } else {
    n = len - 1;
    pstart = k * (int64_t)len;
    dstart = k * (int64_t)n * rep;
  }
  const int64_t nrows = (int64_t)n * rep;
  const int rs = __builtin_ctz((unsigned)rep);
  const int32_t q = d >> 2;  // float4 per row
  const int32_t drow = (int32_t)blockDim.x / q, dc = (int32_t)blockDim.x - drow * q;
  int64_t row = (int32_t)threadIdx.x / q;
  int32_t c = (int32_t)threadIdx.x - (int32_t)row * q;
  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(pts + pstart * d);
  float4* __restrict__ o4 = reinterpret_cast<float4*>(incr + dstart * d);
  while (row < nrows) {
    const int64_t p = row >> rs;
    const float4 a = p4[(p + 1) * q + c], b = p4[p * q + c];
    float4 v;
    v.x = increment_value(a.x, b.x, rounding, scale);
    v.y = increment_value(a.y, b.y, rounding, scale);
    v.z = increment_value(a.z, b.z, rounding, scale);
    v.w = increment_value(a.w, b.w, rounding, scale);
    o4[row * q + c] = v;
    row += drow;
    c += dc;
    if (c >= q) {
      c -= q;
      ++row;
    }
  }
}

__global__ __launch_bounds__(256) void increments4_kernel(const IncJob jx, const IncJob jy) {
  const int64_t b = blockIdx.x;
  if (b < jx.n_paths)
    increments4_one(jx, b);
  else
    increments4_one(jy, b - jx.n_paths);
}

// Plans of a batch refined rep times: n -> n rep (broken paths keep n < 0),
// start -> start rep.
__global__ __launch_bounds__(256) void scale_plan_kernel(int32_t* __restrict__ n,
                                                         int64_t* __restrict__ start,
                                                         int64_t n_paths, int32_t rep) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_paths) return;
  if (n[k] > 0) n[k] *= rep;
  start[k] *= rep;
}

// One workgroup per path: its points as dense padded rows [start + k, start
// + k + n + 1) (uniform: [k len, (k + 1) len)), channels beyond d zero.
__global__ __launch_bounds__(256) void nodes_kernel(
    const float* __restrict__ pts, const int64_t* __restrict__ off,
    const int32_t* __restrict__ plan_n, const int64_t* __restrict__ plan_start, int32_t len,
    int64_t n_paths, int32_t d, int32_t dpad, float* __restrict__ nodes) {
  const int64_t k = blockIdx.x;
  if (k >= n_paths) return;
  int64_t pstart, dstart;
  int32_t n;
  if (off) {
    n = plan_n[k];
    if (n < 0) return;
    pstart = off[k];
    dstart = plan_start[k] + k;
  } else {
    n = len - 1;
    pstart = k * (int64_t)len;
    dstart = k * (int64_t)len;
  }
  const int64_t rows = (int64_t)n + 1;
  const int32_t drow = (int32_t)blockDim.x / dpad, dc = (int32_t)blockDim.x - drow * dpad;
  int64_t p = (int32_t)threadIdx.x / dpad;
  int32_t c = (int32_t)threadIdx.x - (int32_t)p * dpad;
  while (p < rows) {
    nodes[(dstart + p) * dpad + c] = c < d ? pts[(pstart + p) * d + c] : 0.0f;
    p += drow;
    c += dc;
    if (c >= dpad) {
      c -= dpad;
      ++p;
    }
  }
}

__global__ __launch_bounds__(256) void fill_u64_kernel(uint64_t* __restrict__ p, int64_t n,
                                                       uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void fill_kernel(float* __restrict__ p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_plan(const Batch& b, PathPlan plan, hipStream_t stream) {
  if (b.n_paths == 0 || !b.offsets) return hipSuccess;
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, stream, b.offsets, b.len, b.n_paths,
                     plan.n, plan.start);
  return hipGetLastError();
}

namespace {
IncJob make_job(const Batch& b, const PathPlan* plan, float scale, int dpad, float* incr,
                int rounding, int rep) {
  IncJob j{};
  j.pts = b.points;
  j.off = b.offsets;
  j.plan_n = plan ? plan->n : nullptr;
  j.plan_start = plan ? plan->start : nullptr;
  j.len = b.len;
  // a uniform batch of one-point paths has no increments
  j.n_paths = (!b.offsets && b.len < 2) ? 0 : b.n_paths;
  j.d = b.dim;
  j.dpad = dpad;
  j.scale = scale / (float)rep;
  j.rounding = rounding;
  j.rep = rep;
  j.incr = incr;
  return j;
}

// d a multiple of 4 with 16-byte aligned points and rows (or nothing to do)
bool four_wide(const IncJob& j) {
  return j.n_paths == 0 ||
         (j.d % 4 == 0 && j.dpad == j.d && reinterpret_cast<uintptr_t>(j.pts) % 16 == 0 &&
          reinterpret_cast<uintptr_t>(j.incr) % 16 == 0);
}
}  // namespace

hipError_t launch_increments_xy(const Batch& bx, const PathPlan* planx, float scalex,
                                const Batch& by, const PathPlan* plany, float scaley, int dpad,
                                float* incx, float* incy, hipStream_t stream, int rounding,
                                int rep) {
  const IncJob jx = make_job(bx, planx, scalex, dpad, incx, rounding, rep);
  const IncJob jy = make_job(by, plany, scaley, dpad, incy, rounding, rep);
  const int64_t blocks = jx.n_paths + jy.n_paths;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (four_wide(jx) && four_wide(jy))
    hipLaunchKernelGGL(increments4_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, jx, jy);
  else
    hipLaunchKernelGGL(increments_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, jx, jy);
  return hipGetLastError();
}

hipError_t launch_scale_plan(PathPlan plan, int64_t n_paths, int rep, hipStream_t stream) {
  if (n_paths == 0 || rep == 1) return hipSuccess;
  const int64_t blocks = (n_paths + 255) / 256;
  hipLaunchKernelGGL(scale_plan_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, plan.n,
                     plan.start, n_paths, rep);
  return hipGetLastError();
}

hipError_t launch_nodes(const Batch& b, const PathPlan* plan, int dpad, float* nodes,
                        hipStream_t stream) {
  if (b.n_paths == 0) return hipSuccess;
  hipLaunchKernelGGL(nodes_kernel, dim3((unsigned)b.n_paths), dim3(256), 0, stream, b.points,
                     b.offsets, plan ? plan->n : nullptr, plan ? plan->start : nullptr, b.len,
                     b.n_paths, b.dim, dpad, nodes);
  return hipGetLastError();
}

}  // namespace sk
