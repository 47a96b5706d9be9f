// Moments-matching reduction of a discrete measure on paths (Section
// "Moments-matching reduction algorithm for the support of a discrete measure
// on paths"): for weights alpha and the signature-kernel Gram K of the
// support, the proximal-gradient iteration of eq. (fixed_point) for eq.
// (min_lasso),
//     beta <- A_t(beta - gamma grad L(beta)),  grad L(beta) = 2 K (beta - alpha),
// with A_t soft-thresholding at t = gamma lam (the proximal map of
// gamma lam |.|_1).
//
// The whole iteration runs in one launch.  Up to 64 atoms: one wave, lane i
// holding row i of K and its components of the vectors in registers.  Up to
// 4096: one workgroup, each iteration a matrix-vector product (thread i: row
// i of K, summed in double) between two barriers, with the n-vectors (beta,
// beta - alpha, the gradient) in LDS as doubles.
#include <math.h>

#include "internal.h"

namespace sk {
namespace {

// Beyond 64 atoms: one workgroup of 1024 threads reading K from global
// memory, the vectors in LDS (up to 64 atoms: reduce_wave_kernel below).
template <int T, int NMAX>
struct Shared {
  double beta[NMAX];
  double d[NMAX];
  double g[NMAX];
  double alpha[NMAX];
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
template <int T>
__device__ void matvec(const ReduceArgs& a, const double* x, double* out) {
  const int n = a.n;
  for (int i = threadIdx.x; i < n; i += T) {
    double acc = 0.0;
    const float* __restrict__ row = a.K + (int64_t)i * a.ld;
    for (int j = 0; j < n; ++j) acc = fma((double)row[j], x[j], acc);
    out[i] = acc;
  }
}

__device__ double soft(double v, double t) {
  return v > t ? v - t : (v < -t ? v + t : 0.0);
}

// `iters` iterations from the current beta; loss (optional) receives the
// objective before each iteration and after the last.
template <int T, class S>
__device__ void ista_run(const ReduceArgs& a, S& s, double lam, double step, int iters,
                         double* loss) {
  const int n = a.n;
  for (int it = 0; it <= iters; ++it) {
    for (int i = threadIdx.x; i < n; i += T) s.d[i] = s.beta[i] - s.alpha[i];
    __syncthreads();
    matvec<T>(a, s.d, s.g);  // g = K d
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

template <int T, int NMAX>
__global__ __launch_bounds__(T) void reduce_kernel(const ReduceArgs a) {
  __shared__ Shared<T, NMAX> s;
  const int n = a.n;
  for (int i = threadIdx.x; i < n; i += T) {
    s.alpha[i] = (double)a.alpha[i];
    s.beta[i] = s.alpha[i];
  }
  __syncthreads();

  // step: the caller's, else 1 / (2 lambda_max(K)) from power iteration
  // (|lambda| of largest modulus), with a 5% margin
  double step = a.step;
  if (!(step > 0.0)) {
    for (int i = threadIdx.x; i < n; i += T) s.d[i] = 1.0 + 1e-3 * (double)(i % 7);
    __syncthreads();
    double rho = 0.0;
    for (int it = 0; it < 200; ++it) {
      matvec<T>(a, s.d, s.g);
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
    ista_run<T>(a, s, a.lam, step, a.iters, a.loss);
  } else {
    // bisection on the penalty over [0, lambda_max], lambda_max = 2 max |(K alpha)_i|
    matvec<T>(a, s.alpha, s.g);
    __syncthreads();
    double part = 0.0;
    for (int i = threadIdx.x; i < n; i += T) part = fmax(part, fabs(2.0 * s.g[i]));
    double lo = 0.0, hi = block_max<T>(part, s);
    bool found = false;
    double lam = hi;
    for (int r = 0; r < a.rounds; ++r) {
      lam = 0.5 * (lo + hi);
      ista_run<T>(a, s, lam, step, a.iters, nullptr);
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

// Up to 64 atoms: one wave, lane i holding row i of K (zero beyond n) and
// beta_i, alpha_i in registers.  (K d)_i is the same chain of fused
// multiply-adds over j = 0, 1, ... as in the workgroup version, with d_j
// broadcast from lane j through scalar registers (v_readlane); the padded
// columns add exact zeros, so the iterates are bitwise the same.  No LDS and
// no barriers: an iteration is a dependent chain of NB multiply-adds.
__device__ __forceinline__ double lane_value(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), j);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)b >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int NB>
__global__ __launch_bounds__(64) void reduce_wave_kernel(const ReduceArgs a) {
  const int n = a.n, i = threadIdx.x;
  const bool own = i < n;
  double krow[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) krow[j] = (own && j < n) ? (double)a.K[(int64_t)i * a.ld + j] : 0.0;
  const double alpha = own ? (double)a.alpha[i] : 0.0;
  double beta = alpha;
  auto matvec = [&](double x) -> double {  // (K x)_i, x_j held by lane j
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) acc = fma(krow[j], lane_value(x, j), acc);
    return acc;
  };
  auto ista = [&](double lam, double step, int iters, double* loss) {
    for (int it = 0; it <= iters; ++it) {
      const double d = beta - alpha;
      const double g = matvec(d);
      if (loss) {
        double part = 0.0;
        if (own) part += d * g + lam * fabs(beta);
        const double f = wave_sum(part);
        if (i == 0) loss[it] = f;
      }
      if (it == iters) break;
      if (own) beta = soft(beta - step * 2.0 * g, step * lam);
    }
  };

  // step: the caller's, else 1 / (2 lambda_max(K)) from power iteration
  // (|lambda| of largest modulus), with a 5% margin
  double step = a.step;
  if (!(step > 0.0)) {
    double d = own ? 1.0 + 1e-3 * (double)(i % 7) : 0.0;
    double rho = 0.0;
    for (int it = 0; it < 200; ++it) {
      const double g = matvec(d);
      double part = 0.0;
      if (own) part += g * g;
      const double nrm = sqrt(wave_sum(part));
      rho = nrm;  // |K v| with |v| = 1 after the first iteration
      d = own ? (nrm > 0.0 ? g / nrm : 0.0) : 0.0;
    }
    step = rho > 0.0 ? 1.0 / (2.0 * 1.05 * rho) : 1.0;
  }
  if (i == 0 && a.step_out) a.step_out[0] = step;

  if (a.support <= 0) {
    ista(a.lam, step, a.iters, a.loss);
  } else {
    // bisection on the penalty over [0, lambda_max], lambda_max = 2 max |(K alpha)_i|
    const double g = matvec(alpha);
    double part = 0.0;
    if (own) part = fmax(part, fabs(2.0 * g));
    double lo = 0.0, hi = wave_max(part);
    bool found = false;
    double lam = hi;
    for (int r = 0; r < a.rounds; ++r) {
      lam = 0.5 * (lo + hi);
      ista(lam, step, a.iters, nullptr);  // from the previous round's beta
      double cnt = 0.0;
      if (own) cnt += beta != 0.0 ? 1.0 : 0.0;
      const int nnz = (int)wave_sum(cnt);
      if (nnz == a.support) {
        if (own) a.beta[i] = beta;
        if (i == 0) a.lam_out[0] = lam;
        found = true;
      }
      if (nnz > a.support)
        lo = lam;
      else
        hi = lam;
    }
    if (found) return;
    if (i == 0) a.lam_out[0] = lam;
  }
  if (own) a.beta[i] = beta;
}

}  // namespace

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t stream) {
  if (a.n <= 0 || a.n > kMaxReduceN) return hipErrorInvalidValue;
  if (a.n <= 32)
    hipLaunchKernelGGL(reduce_wave_kernel<32>, dim3(1), dim3(64), 0, stream, a);
  else if (a.n <= 64)
    hipLaunchKernelGGL(reduce_wave_kernel<64>, dim3(1), dim3(64), 0, stream, a);
  else
    hipLaunchKernelGGL((reduce_kernel<1024, kMaxReduceN>), dim3(1), dim3(1024), 0, stream, a);
  return hipGetLastError();
}

}  // namespace sk
