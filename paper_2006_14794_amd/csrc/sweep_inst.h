// Instantiations of one sweep kernel (SK_KIND: 0 forward, 3 persistent pairs,
// 4 lifted forward, 5 implicit forward, 6 pipelined bands with a fitted top
// band, 7 pipelined bands of one height) at one dyadic order SK_LAM.  Included
// by sweep_k{kind}_l{lam}.hip so that the configurations compile in parallel
// translation units.
#include "dispatch.h"
#if SK_KIND == 3 || SK_KIND == 6 || SK_KIND == 7
#include "pair_kernel.h"
#elif SK_KIND == 4
#include "lifted_kernel.h"
#else
#include "sweep_fwd_kernel.h"
#endif

#define SK_CAT2(a, b) a##b
#define SK_CAT(a, b) SK_CAT2(a, b)

namespace sk {
namespace {

#if SK_KIND == 0
struct FwdPlain {
  using Fn = void*;
  template <int R, int LAM, int D>
  static Fn get() {
    if constexpr (sweep_fits(R, LAM, D))
      return reinterpret_cast<void*>(&fwd::sweep_kernel<R, LAM, D, false>);
    else
      return nullptr;
  }
};
#elif SK_KIND == 3
struct Pair {
  using Fn = void*;
  template <int R, int LAM, int D>
  static Fn get() {
    if constexpr (sweep_fits(R, LAM, D))
      return reinterpret_cast<void*>(&pairk::pair_kernel<R, LAM, D>);
    else
      return nullptr;
  }
};
#elif SK_KIND == 6 || SK_KIND == 7
// fitted top band (6): ragged batches, at the largest fitting height only;
// one height (7): batches of equal lengths, at every height (few long pairs
// run lower bands, see pair_layout)
struct PairBand {
  using Fn = void*;
  template <int R, int LAM, int D>
  static Fn get() {
    if constexpr (sweep_fits(R, LAM, D) && (SK_KIND == 7 || R == max_fitting_rows(LAM, D)))
      return reinterpret_cast<void*>(&pairk::pair_band_kernel<R, LAM, D, SK_KIND == 6>);
    else
      return nullptr;
  }
};
#elif SK_KIND == 5
struct FwdImplicit {
  using Fn = void*;
  template <int R, int LAM, int D>
  static Fn get() {
    if constexpr (sweep_fits(R, LAM, D))
      return reinterpret_cast<void*>(&fwd::sweep_kernel<R, LAM, D, true>);
    else
      return nullptr;
  }
};
#elif SK_KIND == 4
struct Lifted {
  using Fn = void*;
  template <int R, int LAM, int D>
  static Fn get() {
    if constexpr (lifted_fits(R, LAM, D))
      return reinterpret_cast<void*>(&lift::lifted_sweep_kernel<R, LAM, D>);
    else
      return nullptr;
  }
};
#endif

template <class F>
void* pick_fixed_lam(int R, int d) {
  switch (R) {
    case 1: return pick_d<F, 1, SK_LAM>(d);
    case 2: return pick_d<F, 2, SK_LAM>(d);
    case 4: return pick_d<F, 4, SK_LAM>(d);
    case 8: return pick_d<F, 8, SK_LAM>(d);
    case 16: return pick_d<F, 16, SK_LAM>(d);
    case 32: return pick_d<F, 32, SK_LAM>(d);
    default: return nullptr;
  }
}

}  // namespace

#if SK_KIND == 0
void* SK_CAT(SK_CAT(sweep_fn_k0_l, SK_LAM), _)(int R, int d) { return pick_fixed_lam<FwdPlain>(R, d); }
#elif SK_KIND == 3
void* SK_CAT(SK_CAT(sweep_fn_k3_l, SK_LAM), _)(int R, int d) { return pick_fixed_lam<Pair>(R, d); }
#elif SK_KIND == 4
void* SK_CAT(SK_CAT(sweep_fn_k4_l, SK_LAM), _)(int R, int d) { return pick_fixed_lam<Lifted>(R, d); }
#elif SK_KIND == 5
void* SK_CAT(SK_CAT(sweep_fn_k5_l, SK_LAM), _)(int R, int d) { return pick_fixed_lam<FwdImplicit>(R, d); }
#elif SK_KIND == 6
void* SK_CAT(SK_CAT(sweep_fn_k6_l, SK_LAM), _)(int R, int d) { return pick_fixed_lam<PairBand>(R, d); }
#elif SK_KIND == 7
void* SK_CAT(SK_CAT(sweep_fn_k7_l, SK_LAM), _)(int R, int d) { return pick_fixed_lam<PairBand>(R, d); }
#endif

}  // namespace sk
