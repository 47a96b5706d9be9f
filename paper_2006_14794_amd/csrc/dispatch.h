// Compile-time configuration tables of the sweep kernels.  A factory F
// provides `using Fn = ...` and `template <int R, int LAM, int D> static Fn
// get()` returning the instantiation (or nullptr when the configuration is
// not compiled); pick<F>(R, lam, d) maps runtime values onto it.
#pragma once

namespace sk {

// Register budget of the one-wave sweeps: x increments (coarse rows x D
// floats) and the row state (R doubles).
constexpr bool sweep_fits(int R, int LAM, int D) {
  return ((R >> LAM) > 0 ? (R >> LAM) : 1) * D <= 96 && R <= 32;
}

// Largest power-of-two rows per lane (at most 32) that sweep_fits allows.
// The pipelined band kernel only runs when the tallest grid needs several
// bands, which happens only at this height, so it is compiled at it alone.
constexpr int max_fitting_rows(int LAM, int D) {
  int r = 0;
  for (int R = 1; R <= 32; R *= 2)
    if (sweep_fits(R, LAM, D)) r = R;
  return r;
}

// The lifted sweep keeps the x nodes (coarse rows + 1) instead of the
// increments, plus the previous column's row differences.
constexpr bool lifted_fits(int R, int LAM, int D) {
  return (((R >> LAM) > 0 ? (R >> LAM) : 1) + 1) * D <= 96 && R <= 32;
}

template <class F, int R, int LAM>
typename F::Fn pick_d(int d) {
  switch (d) {
    case 1: return F::template get<R, LAM, 1>();
    case 2: return F::template get<R, LAM, 2>();
    case 3: return F::template get<R, LAM, 3>();
    case 4: return F::template get<R, LAM, 4>();
    case 5: return F::template get<R, LAM, 5>();
    case 6: return F::template get<R, LAM, 6>();
    case 7: return F::template get<R, LAM, 7>();
    case 8: return F::template get<R, LAM, 8>();
    case 9: return F::template get<R, LAM, 9>();
    case 10: return F::template get<R, LAM, 10>();
    case 11: return F::template get<R, LAM, 11>();
    case 12: return F::template get<R, LAM, 12>();
    case 13: return F::template get<R, LAM, 13>();
    case 14: return F::template get<R, LAM, 14>();
    case 15: return F::template get<R, LAM, 15>();
    case 16: return F::template get<R, LAM, 16>();
    default: return nullptr;
  }
}

template <class F, int R>
typename F::Fn pick_lam(int lam, int d) {
  switch (lam) {
    case 0: return pick_d<F, R, 0>(d);
    case 1: return pick_d<F, R, 1>(d);
    case 2: return pick_d<F, R, 2>(d);
    case 3: return pick_d<F, R, 3>(d);
    default: return nullptr;
  }
}

template <class F>
typename F::Fn pick(int R, int lam, int d) {
  switch (R) {
    case 1: return pick_lam<F, 1>(lam, d);
    case 2: return pick_lam<F, 2>(lam, d);
    case 4: return pick_lam<F, 4>(lam, d);
    case 8: return pick_lam<F, 8>(lam, d);
    case 16: return pick_lam<F, 16>(lam, d);
    case 32: return pick_lam<F, 32>(lam, d);
    default: return nullptr;
  }
}

}  // namespace sk
