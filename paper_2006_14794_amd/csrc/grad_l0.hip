// Gram gradient kernel instantiations, dyadic order 0 (see grad_inst.h).
#define SK_LAM 0
#include "grad_inst.h"
