// Launchers of the forward sweep kernels (sweep_fwd_kernel.h) and the table of
// compiled configurations (instantiated per dyadic order in sweep_lam*.hip).
#include "internal.h"

namespace sk {

#define SK_DECL(k, l) void* sweep_fn_k##k##_l##l##_(int R, int d);
SK_DECL(0, 0) SK_DECL(0, 1) SK_DECL(0, 2) SK_DECL(0, 3)
SK_DECL(3, 0) SK_DECL(3, 1) SK_DECL(3, 2) SK_DECL(3, 3)
SK_DECL(4, 0) SK_DECL(4, 1) SK_DECL(4, 2) SK_DECL(4, 3)
SK_DECL(5, 0) SK_DECL(5, 1) SK_DECL(5, 2) SK_DECL(5, 3)
SK_DECL(6, 0) SK_DECL(6, 1) SK_DECL(6, 2) SK_DECL(6, 3)
SK_DECL(7, 0) SK_DECL(7, 1) SK_DECL(7, 2) SK_DECL(7, 3)
#undef SK_DECL

void* none_(int, int) { return nullptr; }  // kinds 1 and 2 are not compiled

void* sweep_fn(int kind, int lam, int R, int d) {
  using Pick = void* (*)(int, int);
  static const Pick table[8][4] = {
      {sweep_fn_k0_l0_, sweep_fn_k0_l1_, sweep_fn_k0_l2_, sweep_fn_k0_l3_},
      {none_, none_, none_, none_},
      {none_, none_, none_, none_},
      {sweep_fn_k3_l0_, sweep_fn_k3_l1_, sweep_fn_k3_l2_, sweep_fn_k3_l3_},
      {sweep_fn_k4_l0_, sweep_fn_k4_l1_, sweep_fn_k4_l2_, sweep_fn_k4_l3_},
      {sweep_fn_k5_l0_, sweep_fn_k5_l1_, sweep_fn_k5_l2_, sweep_fn_k5_l3_},
      {sweep_fn_k6_l0_, sweep_fn_k6_l1_, sweep_fn_k6_l2_, sweep_fn_k6_l3_},
      {sweep_fn_k7_l0_, sweep_fn_k7_l1_, sweep_fn_k7_l2_, sweep_fn_k7_l3_}};
  if (kind < 0 || kind > 7 || lam < 0 || lam > 3) return nullptr;
  return table[kind][lam](R, d);
}

int choose_rows_for(int kind, int64_t fine_rows, int lam, int d) {
  for (int R = 1; R <= kMaxRowsPerLane; R *= 2) {
    if (64 * (int64_t)R < fine_rows) continue;
    return sweep_fn(kind, lam, R, d) ? R : 0;
  }
  return 0;
}

int choose_rows_per_lane(int64_t fine_rows, int lam, int d) {
  return choose_rows_for(kKernelForward, fine_rows, lam, d);
}

namespace {
hipError_t launch_forward(int kind, const SweepArgs& a, int lam, int R, int d,
                          hipStream_t stream, int wpb) {
  auto f = reinterpret_cast<void (*)(const SweepArgs)>(sweep_fn(kind, lam, R, d));
  if (!f) return hipErrorInvalidValue;
  if (a.n_waves == 0) return hipSuccess;
  if (wpb != 1 && wpb != 2) wpb = 4;  // the kernels are bounded to 256 threads
  const int64_t blocks = (a.n_waves + wpb - 1) / wpb;
  hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(64 * wpb), 0, stream, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_sweep(const SweepArgs& a, int lam, int R, int d, hipStream_t stream,
                        int waves_per_block) {
  return launch_forward(a.implicit ? kKernelForwardImplicit : kKernelForward, a, lam, R, d,
                        stream, waves_per_block);
}

hipError_t launch_lifted(const SweepArgs& a, int lam, int R, int d, hipStream_t stream,
                         int waves_per_block) {
  return launch_forward(kKernelLifted, a, lam, R, d, stream, waves_per_block);
}

}  // namespace sk
