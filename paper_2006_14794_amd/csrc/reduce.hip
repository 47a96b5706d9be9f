// Moments-matching reduction of a discrete measure on paths (Section
// "Moments-matching reduction algorithm for the support of a discrete measure
// on paths"): for weights alpha and the signature-kernel Gram K of the
// support, the proximal-gradient iteration of eq. (fixed_point) for eq.
// (min_lasso),
//     beta <- A_t(beta - gamma grad L(beta)),  grad L(beta) = 2 K (beta - alpha),
// with A_t soft-thresholding at t = gamma lam (the proximal map of
// gamma lam |.|_1).
//
// The whole iteration runs in one workgroup: each iteration is a
// matrix-vector product (thread i: row i of K, summed in double) between two
// barriers, and the n-vectors (beta, beta - alpha, the gradient) live in LDS
// as doubles.  n <= 4096.
#include <math.h>

#include "internal.h"

namespace sk {
namespace {

// Two shapes of the same kernel: up to 64 atoms, one wave with K staged in
// LDS as double (barriers and reductions within the wave); beyond, 1024
// threads reading K from global memory.
template <int T, int NMAX, bool KLDS>
struct Shared {
  double beta[NMAX];
  double d[NMAX];
  double g[NMAX];
  double alpha[NMAX];
  double k[KLDS ? NMAX * NMAX : 1];
  double red[T / 64];
};

// Sum of v over the workgroup (every thread passes its part); all threads
// receive the total.
template <int T, class S>
__device__ double block_sum(double v, S& s) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if constexpr (T == 64) return v;
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s.red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < T / 64; ++w) t += s.red[w];
  return t;
}

template <int T, class S>
__device__ double block_max(double v, S& s) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if constexpr (T == 64) return v;
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s.red[wid] = v;
  __syncthreads();
  double t = s.red[0];
  for (int w = 1; w < T / 64; ++w) t = fmax(t, s.red[w]);
  return t;
}

// out[i] = sum_j K[i][j] x[j] for the rows of this thread
template <int T, bool KLDS, class S>
__device__ void matvec(const ReduceArgs& a, S& s, const double* x, double* out) {
  const int n = a.n;
  for (int i = threadIdx.x; i < n; i += T) {
    double acc = 0.0;
    if constexpr (KLDS) {
      const double* row = s.k + i * n;
      for (int j = 0; j < n; ++j) acc = fma(row[j], x[j], acc);
    } else {
      const float* __restrict__ row = a.K + (int64_t)i * a.ld;
      for (int j = 0; j < n; ++j) acc = fma((double)row[j], x[j], acc);
    }
    out[i] = acc;
  }
}

__device__ double soft(double v, double t) {
  return v > t ? v - t : (v < -t ? v + t : 0.0);
}

// `iters` iterations from the current beta; loss (optional) receives the
// objective before each iteration and after the last.
template <int T, bool KLDS, class S>
__device__ void ista_run(const ReduceArgs& a, S& s, double lam, double step, int iters,
                         double* loss) {
  const int n = a.n;
  for (int it = 0; it <= iters; ++it) {
    for (int i = threadIdx.x; i < n; i += T) s.d[i] = s.beta[i] - s.alpha[i];
    __syncthreads();
    matvec<T, KLDS>(a, s, s.d, s.g);  // g = K d
    __syncthreads();
    if (loss) {
      double part = 0.0;
      for (int i = threadIdx.x; i < n; i += T) part += s.d[i] * s.g[i] + lam * fabs(s.beta[i]);
      const double f = block_sum<T>(part, s);
      if (threadIdx.x == 0) loss[it] = f;
    }
    if (it == iters) break;
    for (int i = threadIdx.x; i < n; i += T)
      s.beta[i] = soft(s.beta[i] - step * 2.0 * s.g[i], step * lam);
    __syncthreads();
  }
}

template <int T, int NMAX, bool KLDS>
__global__ __launch_bounds__(T) void reduce_kernel(const ReduceArgs a) {
  __shared__ Shared<T, NMAX, KLDS> s;
  const int n = a.n;
  for (int i = threadIdx.x; i < n; i += T) {
    s.alpha[i] = (double)a.alpha[i];
    s.beta[i] = s.alpha[i];
  }
  if constexpr (KLDS)
    for (int e = threadIdx.x; e < n * n; e += T) s.k[e] = (double)a.K[(e / n) * a.ld + e % n];
  __syncthreads();

  // step: the caller's, else 1 / (2 lambda_max(K)) from power iteration
  // (|lambda| of largest modulus), with a 5% margin
  double step = a.step;
  if (!(step > 0.0)) {
    for (int i = threadIdx.x; i < n; i += T) s.d[i] = 1.0 + 1e-3 * (double)(i % 7);
    __syncthreads();
    double rho = 0.0;
    for (int it = 0; it < 200; ++it) {
      matvec<T, KLDS>(a, s, s.d, s.g);
      __syncthreads();
      double part = 0.0;
      for (int i = threadIdx.x; i < n; i += T) part += s.g[i] * s.g[i];
      const double nrm = sqrt(block_sum<T>(part, s));
      rho = nrm;  // |K v| with |v| = 1 after the first iteration
      for (int i = threadIdx.x; i < n; i += T) s.d[i] = nrm > 0.0 ? s.g[i] / nrm : 0.0;
      __syncthreads();
    }
    step = rho > 0.0 ? 1.0 / (2.0 * 1.05 * rho) : 1.0;
  }
  if (threadIdx.x == 0 && a.step_out) a.step_out[0] = step;

  if (a.support <= 0) {
    ista_run<T, KLDS>(a, s, a.lam, step, a.iters, a.loss);
  } else {
    // bisection on the penalty over [0, lambda_max], lambda_max = 2 max |(K alpha)_i|
    matvec<T, KLDS>(a, s, s.alpha, s.g);
    __syncthreads();
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += T) part = fmax(part, fabs(2.0 * s.g[i]));
    double lo = 0.0, hi = block_max<T>(part, s);
    bool found = false;
    double lam = hi;
    for (int r = 0; r < a.rounds; ++r) {
      lam = 0.5 * (lo + hi);
      ista_run<T, KLDS>(a, s, lam, step, a.iters, nullptr);
      double cnt = 0.0;
      for (int i = threadIdx.x; i < n; i += T) cnt += s.beta[i] != 0.0 ? 1.0 : 0.0;
      const int nnz = (int)block_sum<T>(cnt, s);
      if (nnz == a.support) {
        for (int i = threadIdx.x; i < n; i += T) a.beta[i] = s.beta[i];
        if (threadIdx.x == 0) a.lam_out[0] = lam;
        found = true;
      }
      if (nnz > a.support)
        lo = lam;
      else
        hi = lam;
      __syncthreads();
    }
    if (found) return;
    if (threadIdx.x == 0) a.lam_out[0] = lam;
  }
  for (int i = threadIdx.x; i < n; i += T) a.beta[i] = s.beta[i];
}

}  // namespace

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t stream) {
  if (a.n <= 0 || a.n > kMaxReduceN) return hipErrorInvalidValue;
  if (a.n <= 64)
    hipLaunchKernelGGL((reduce_kernel<64, 64, true>), dim3(1), dim3(64), 0, stream, a);
  else
    hipLaunchKernelGGL((reduce_kernel<1024, kMaxReduceN, false>), dim3(1), dim3(1024), 0, stream,
                       a);
  return hipGetLastError();
}

}  // namespace sk
