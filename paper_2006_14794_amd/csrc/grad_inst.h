// Instantiations of the Gram gradient kernel (grad_kernel.h) at one dyadic
// order SK_LAM, for 1 to 16 channels.  Included by grad_l{lam}.hip so that
// the orders compile in parallel translation units.
#include "grad_kernel.h"

#define SK_CAT2(a, b) a##b
#define SK_CAT(a, b) SK_CAT2(a, b)

namespace sk {
namespace {
template <int D>
void* grad_get(bool ys) {
  return ys ? reinterpret_cast<void*>(
                  &grad::grad_kernel<kGradRows, SK_LAM, D, grad_lds_steps(SK_LAM),
                                     grad_reg_steps(SK_LAM, D), true>)
            : reinterpret_cast<void*>(
                  &grad::grad_kernel<kGradRows, SK_LAM, D, grad_lds_steps(SK_LAM),
                                     grad_reg_steps(SK_LAM, D), false>);
}
}  // namespace

void* SK_CAT(SK_CAT(grad_fn_l, SK_LAM), _)(int d, bool ys) {
  switch (d) {
    case 1: return grad_get<1>(ys);
    case 2: return grad_get<2>(ys);
    case 3: return grad_get<3>(ys);
    case 4: return grad_get<4>(ys);
    case 5: return grad_get<5>(ys);
    case 6: return grad_get<6>(ys);
    case 7: return grad_get<7>(ys);
    case 8: return grad_get<8>(ys);
    case 9: return grad_get<9>(ys);
    case 10: return grad_get<10>(ys);
    case 11: return grad_get<11>(ys);
    case 12: return grad_get<12>(ys);
    case 13: return grad_get<13>(ys);
    case 14: return grad_get<14>(ys);
    case 15: return grad_get<15>(ys);
    case 16: return grad_get<16>(ys);
    default: return nullptr;
  }
}

}  // namespace sk
