// Gram gradient kernel instantiations, dyadic order 3 (see grad_inst.h).
#define SK_LAM 3
#include "grad_inst.h"
