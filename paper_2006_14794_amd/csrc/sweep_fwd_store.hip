// Forward sweep that also stores, for every cell, the sum of its left and
// upper nodes (the factor of the coefficient gradient) for the adjoint pass.
// Kernel: sweep_fwd_kernel.h.
#include "dispatch.h"
#include "sweep_fwd_kernel.h"

namespace sk {
namespace {

struct FwdStore {
  using Fn = void (*)(const SweepArgs);
  template <int R, int LAM, int D>
  static Fn get() {
    if constexpr (sweep_fits(R, LAM, D))
      return &fwd::sweep_kernel<R, LAM, D, true>;
    else
      return nullptr;
  }
};

}  // namespace

hipError_t launch_sweep_store(const SweepArgs& a, int lam, int R, int d, hipStream_t stream) {
  FwdStore::Fn f = pick<FwdStore>(R, lam, d);
  if (!f) return hipErrorInvalidValue;
  if (a.n_waves == 0) return hipSuccess;
  constexpr int kWavesPerBlock = 4;
  const int64_t blocks = (a.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, stream, a);
  return hipGetLastError();
}

}  // namespace sk
