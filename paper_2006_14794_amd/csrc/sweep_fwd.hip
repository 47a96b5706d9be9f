// Forward sweep launches (value only).  Kernel: sweep_fwd_kernel.h.
#include "dispatch.h"
#include "sweep_fwd_kernel.h"

namespace sk {
namespace {

struct FwdPlain {
  using Fn = void (*)(const SweepArgs);
  template <int R, int LAM, int D>
  static Fn get() {
    if constexpr (sweep_fits(R, LAM, D))
      return &fwd::sweep_kernel<R, LAM, D, false>;
    else
      return nullptr;
  }
};

}  // namespace

int choose_rows_per_lane(int64_t fine_rows, int lam, int d) {
  for (int R = 1; R <= kMaxRowsPerLane; R *= 2) {
    if (64 * (int64_t)R < fine_rows) continue;
    return pick<FwdPlain>(R, lam, d) ? R : 0;
  }
  return 0;
}

hipError_t launch_sweep(const SweepArgs& a, int lam, int R, int d, hipStream_t stream) {
  FwdPlain::Fn f = pick<FwdPlain>(R, lam, d);
  if (!f) return hipErrorInvalidValue;
  if (a.n_waves == 0) return hipSuccess;
  constexpr int kWavesPerBlock = 4;
  const int64_t blocks = (a.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0, stream, a);
  return hipGetLastError();
}

}  // namespace sk
