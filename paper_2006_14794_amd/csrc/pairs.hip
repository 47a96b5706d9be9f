// Planning and launch of independent pairs (pair_kernel.h): every pair is
// classified by the rows it needs (shorter path, refined), the pairs of each
// class are ordered longest first, and persistent waves take them from a
// device queue.
#include "internal.h"

namespace sk {
namespace {

constexpr int kBuckets = 1024;  // cost buckets per class

__device__ __forceinline__ int32_t incs(const int32_t* plan, int32_t len, int64_t k) {
  return plan ? plan[k] : len - 1;
}

// One workgroup.  Output: order[0 .. c_hi) = long-row class, order[c_hi ..
// c_hi + c_lo) = short-row class, each roughly by decreasing estimated cost
// (a counting sort into kBuckets equal cost ranges per class; the order
// within a bucket is whatever the atomics give, which only affects
// scheduling); counts {c_hi, c_lo}; both queue counters zeroed.
__global__ __launch_bounds__(1024) void pair_plan_kernel(
    const int32_t* __restrict__ x_n, int32_t x_len, const int32_t* __restrict__ y_n,
    int32_t y_len, int32_t npairs, int32_t lam, int32_t rows_lo, int32_t rows_hi,
    int64_t gram_ny, int32_t* __restrict__ order, int32_t* __restrict__ counts,
    int32_t* __restrict__ counters) {
  __shared__ int32_t hist[2 * kBuckets];  // bucket 0 .. kBuckets-1: long class
  __shared__ int32_t cnt[2];
  __shared__ unsigned long long cmax[2];
  __shared__ int32_t wsum[16];
  for (int i = threadIdx.x; i < 2 * kBuckets; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x < 2) {
    cnt[threadIdx.x] = 0;
    cmax[threadIdx.x] = 0;
  }
  __syncthreads();
  // rows per lane are powers of two: bands by a shift (no 64-bit division)
  const int sh_lo = 6 + (rows_lo > 0 ? __builtin_ctz((unsigned)rows_lo) : 0);
  const int sh_hi = 6 + __builtin_ctz((unsigned)(rows_hi > 0 ? rows_hi : 1));
  auto classify = [&](int32_t k, unsigned long long& cost) -> int {
    const uint32_t ny = (uint32_t)gram_ny;  // npairs < 2^31
    const int64_t ix = ny ? (uint32_t)k / ny : k, iy = ny ? k - ix * (int64_t)ny : k;
    const int32_t mx = incs(x_n, x_len, ix), my = incs(y_n, y_len, iy);
    if (mx <= 0 || my <= 0) {
      cost = 0;
      // trivial or broken: instant; the short class, or the end of the long
      // one when there is no short class (rows_lo = 0)
      return rows_lo > 0 ? 0 : 1;
    }
    const int64_t mn = mx < my ? mx : my, mxn = mx < my ? my : mx;
    const int64_t M = mn << lam;
    const int cls = M <= 64 * (int64_t)rows_lo ? 0 : 1;
    const int sh = cls ? sh_hi : sh_lo;
    const int64_t bands = (M + (int64_t(1) << sh) - 1) >> sh;
    cost = (unsigned long long)(bands * (mxn + 63));
    if (cost > (1ull << 45) - 1) cost = (1ull << 45) - 1;
    return cls;
  };
  // a batch of equal lengths: every pair has the same cost and class, so the
  // identity order is already sorted
  if (!x_n && !y_n) {
    unsigned long long cost;
    const int cls = npairs > 0 ? classify(0, cost) : 1;
    for (int64_t k = threadIdx.x; k < npairs; k += blockDim.x) order[k] = (int32_t)k;
    if (threadIdx.x == 0) {
      counts[0] = cls ? npairs : 0;
      counts[1] = cls ? 0 : npairs;
      counters[0] = 0;
      counters[1] = 0;
    }
    return;
  }
  // bucket of a pair: long class first, each class by decreasing cost; the
  // cost ranges are the leading bits of the cost below the class maximum's
  // next power of two (a shift, no 64-bit division)
  auto bucket = [&](int cls, unsigned long long cost) -> int {
    const int len = 64 - __clzll((long long)cmax[cls]);  // bits of the maximum
    const int q = len > 10 ? (int)(cost >> (len - 10)) : (int)(cost << (10 - len));
    return (cls ? 0 : kBuckets) + (kBuckets - 1 - q);  // q in 0 .. kBuckets-1
  };
  // Every pass runs all lanes (k past npairs: not counted) and takes one LDS
  // atomic per wave where the wave's pairs agree (a batch of equal lengths
  // puts every pair in one bucket), one per lane otherwise.
  const int lane = threadIdx.x & 63;
  auto wave_add = [&](int32_t* ctr, bool ok, int b) -> int32_t {  // ctr[b] += 1 per ok lane
    const unsigned long long act = __ballot(ok);
    if (act == 0) return 0;
    const int first = __ffsll(act) - 1;
    const int b0 = __shfl(b, first, 64);
    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0));
    if (__ballot(ok && b == b0) == act) {
      int32_t base = 0;
      if (lane == first) base = atomicAdd(&ctr[b0], __popcll(act));
      return __shfl(base, first, 64) + rank;
    }
    return ok ? atomicAdd(&ctr[b], 1) : 0;
  };
  for (int64_t base = 0; base < npairs; base += blockDim.x) {  // 64-bit: npairs < 2^31
    const bool ok = base + threadIdx.x < npairs;
    const int32_t k = ok ? (int32_t)(base + threadIdx.x) : 0;
    unsigned long long cost = 0;
    const int cls = ok ? classify(k, cost) : 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const unsigned long long in = __ballot(ok && cls == c);
      unsigned long long m = (ok && cls == c) ? cost : 0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
      }
      if (lane == 0 && in != 0) {
        atomicAdd(&cnt[c], __popcll(in));
        atomicMax(&cmax[c], m);
      }
    }
  }
  __syncthreads();
  for (int64_t base = 0; base < npairs; base += blockDim.x) {  // 64-bit: npairs < 2^31
    const bool ok = base + threadIdx.x < npairs;
    const int32_t k = ok ? (int32_t)(base + threadIdx.x) : 0;
    unsigned long long cost = 0;
    const int cls = ok ? classify(k, cost) : 0;
    wave_add(hist, ok, ok ? bucket(cls, cost) : 0);
  }
  __syncthreads();
  // exclusive scan of the 2 kBuckets counts: two per thread, then across waves
  {
    const int t = threadIdx.x, wid = t >> 6;
    const int32_t a0 = hist[2 * t], a1 = hist[2 * t + 1];
    int32_t v = a0 + a1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t u = __shfl_up(v, o, 64);
      if (lane >= o) v += u;
    }
    if (lane == 63) wsum[wid] = v;
    __syncthreads();
    int32_t before = 0;
    for (int w = 0; w < wid; ++w) before += wsum[w];
    const int32_t start = before + v - (a0 + a1);
    hist[2 * t] = start;
    hist[2 * t + 1] = start + a0;
  }
  __syncthreads();
  for (int64_t base = 0; base < npairs; base += blockDim.x) {  // 64-bit: npairs < 2^31
    const bool ok = base + threadIdx.x < npairs;
    const int32_t k = ok ? (int32_t)(base + threadIdx.x) : 0;
    unsigned long long cost = 0;
    const int cls = ok ? classify(k, cost) : 0;
    const int32_t pos = wave_add(hist, ok, ok ? bucket(cls, cost) : 0);
    if (ok) order[pos] = k;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    counts[0] = cnt[1];
    counts[1] = cnt[0];
    counters[0] = 0;
    counters[1] = 0;
  }
}

// One workgroup: band counts of the long-class pairs (order[0 .. counts[0]))
// and their exclusive prefix sum.
__global__ __launch_bounds__(1024) void band_plan_kernel(
    const int32_t* __restrict__ x_n, int32_t x_len, const int32_t* __restrict__ y_n,
    int32_t y_len, int32_t lam, int32_t rows, int64_t gram_ny,
    const int32_t* __restrict__ order, const int32_t* __restrict__ counts,
    int32_t* __restrict__ task_base, int32_t* __restrict__ task_counter) {
  __shared__ int32_t scan[1024];
  const int32_t count = counts[0];
  // 1024 pairs at a time, carrying the running total between chunks
  int32_t carry = 0;
  for (int64_t base = 0; base < count; base += 1024) {  // 64-bit: count < 2^31
    const int32_t k = base + threadIdx.x < count ? (int32_t)(base + threadIdx.x) : count;
    int32_t nb = 0;
    if (k < count) {
      const int32_t pid = order[k];
      const int64_t ix = gram_ny ? pid / gram_ny : pid, iy = gram_ny ? pid - ix * gram_ny : pid;
      const int32_t mx = incs(x_n, x_len, ix), my = incs(y_n, y_len, iy);
      if (mx <= 0 || my <= 0) {
        nb = 1;  // one task writes its value
      } else {
        const int64_t M = (int64_t)(mx < my ? mx : my) << lam;
        nb = (int32_t)((M + 64 * (int64_t)rows - 1) / (64 * (int64_t)rows));
      }
    }
    scan[threadIdx.x] = nb;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan
      const int32_t v = (int)threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (k < count) task_base[k] = carry + scan[threadIdx.x] - nb;
    carry += scan[1023];
    __syncthreads();  // scan[] is rewritten by the next chunk
  }
  if (threadIdx.x == 0) {
    task_base[count] = carry;
    *task_counter = 0;
  }
}

// The sentinel into the part of the slot buffers that the bands write: the
// first n S doubles (n coarse columns of the pair, S fine columns each) of
// every band task but a pair's last, which hands nothing on.  One workgroup
// per pair of the band plan; tasks at or past t_max are left alone.
__global__ __launch_bounds__(256) void fill_task_slots_kernel(
    uint64_t* __restrict__ tbuf, const int32_t* __restrict__ task_base,
    const int32_t* __restrict__ order, const int32_t* __restrict__ counts,
    const int32_t* __restrict__ x_n, int32_t x_len, const int32_t* __restrict__ y_n,
    int32_t y_len, int64_t gram_ny, int32_t lam, int64_t stride, int64_t t_max, uint64_t v) {
  const int32_t count = counts[0];
  for (int64_t k = blockIdx.x; k < count; k += gridDim.x) {
    const int64_t t0 = task_base[k];
    int64_t t1 = (int64_t)task_base[k + 1] - 1;  // the pair's last task is not filled
    if (t1 > t_max) t1 = t_max;
    const int32_t pid = order[k];
    const int64_t ix = gram_ny ? pid / gram_ny : pid, iy = gram_ny ? pid - ix * gram_ny : pid;
    const int32_t mx = incs(x_n, x_len, ix), my = incs(y_n, y_len, iy);
    if (mx <= 0 || my <= 0) continue;  // a single task
    int64_t n = (int64_t)(mx > my ? mx : my) << lam;
    if (n > stride) n = stride;
    for (int64_t t = t0; t < t1; ++t) {
      uint64_t* __restrict__ p = tbuf + t * stride;
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
    }
  }
}

}  // namespace

hipError_t launch_band_plan(const PairPlanArgs& p, int rows_per_lane, int32_t* task_base,
                            int32_t* task_counter, hipStream_t stream) {
  hipLaunchKernelGGL(band_plan_kernel, dim3(1), dim3(1024), 0, stream, p.x_n, p.x_len, p.y_n,
                     p.y_len, p.lam, rows_per_lane, p.gram_ny, p.order, p.counts, task_base,
                     task_counter);
  return hipGetLastError();
}

hipError_t launch_fill_task_slots(uint64_t* tbuf, const PairPlanArgs& p,
                                  const int32_t* task_base, int64_t stride, int64_t t_max,
                                  uint64_t v, hipStream_t stream) {
  if (t_max <= 0 || p.npairs <= 0) return hipSuccess;
  const int32_t blocks = p.npairs < 8192 ? p.npairs : 8192;
  hipLaunchKernelGGL(fill_task_slots_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, tbuf,
                     task_base, p.order, p.counts, p.x_n, p.x_len, p.y_n, p.y_len, p.gram_ny,
                     p.lam, stride, t_max, v);
  return hipGetLastError();
}

hipError_t launch_pair_plan(const PairPlanArgs& p, hipStream_t stream) {
  hipLaunchKernelGGL(pair_plan_kernel, dim3(1), dim3(1024), 0, stream, p.x_n, p.x_len, p.y_n,
                     p.y_len, p.npairs, p.lam, p.rows_lo, p.rows_hi, p.gram_ny, p.order,
                     p.counts, p.counters);
  return hipGetLastError();
}

namespace {
hipError_t launch_persistent(int kind, const PairArgs& a, int lam, int R, int d,
                             int64_t max_waves, hipStream_t stream, int blocks_per_cu_wanted) {
  auto f = reinterpret_cast<void (*)(const PairArgs)>(sweep_fn(kind, lam, R, d));
  if (!f) return hipErrorInvalidValue;
  int dev = 0, cus = 0, blocks_per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorInvalidDevice;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, f, 256, 0) != hipSuccess)
    return hipErrorInvalidValue;
  if (blocks_per_cu < 1) blocks_per_cu = 1;
  if (blocks_per_cu_wanted > 0) blocks_per_cu = blocks_per_cu_wanted < 64 ? blocks_per_cu_wanted : 64;
  int64_t waves = (int64_t)cus * blocks_per_cu * 4;
  if (waves > max_waves) waves = max_waves;  // max_waves: a multiple of 4 (wave slots)
  const int64_t blocks = waves / 4 > 0 ? waves / 4 : 1;
  hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_pairs(const PairArgs& a, int lam, int R, int d, int64_t max_waves,
                        hipStream_t stream, int blocks_per_cu_wanted) {
  return launch_persistent(kKernelPair, a, lam, R, d, max_waves, stream, blocks_per_cu_wanted);
}

hipError_t launch_pair_bands(const PairArgs& a, int lam, int R, int d, int64_t max_waves,
                             hipStream_t stream, int blocks_per_cu_wanted, bool fit_top) {
  return launch_persistent(fit_top ? kKernelPairBand : kKernelPairBandFull, a, lam, R, d,
                           max_waves, stream, blocks_per_cu_wanted);
}

}  // namespace sk
