// Instantiations of the Gram gradient kernel (grad_kernel.h) at one dyadic
// order SK_LAM, for 1 to 16 channels.  Included by grad_l{lam}.hip so that
// the orders compile in parallel translation units.
#include "grad_kernel.h"

#define SK_CAT2(a, b) a##b
#define SK_CAT(a, b) SK_CAT2(a, b)

namespace sk {
namespace {
template <int D>
void* grad_get() {
  return reinterpret_cast<void*>(
      &grad::grad_kernel<kGradRows, SK_LAM, D, grad_lds_steps(SK_LAM), grad_reg_steps(SK_LAM, D)>);
}
}  // namespace

void* SK_CAT(SK_CAT(grad_fn_l, SK_LAM), _)(int d) {
  switch (d) {
    case 1: return grad_get<1>();
    case 2: return grad_get<2>();
    case 3: return grad_get<3>();
    case 4: return grad_get<4>();
    case 5: return grad_get<5>();
    case 6: return grad_get<6>();
    case 7: return grad_get<7>();
    case 8: return grad_get<8>();
    case 9: return grad_get<9>();
    case 10: return grad_get<10>();
    case 11: return grad_get<11>();
    case 12: return grad_get<12>();
    case 13: return grad_get<13>();
    case 14: return grad_get<14>();
    case 15: return grad_get<15>();
    case 16: return grad_get<16>();
    default: return nullptr;
  }
}

}  // namespace sk
