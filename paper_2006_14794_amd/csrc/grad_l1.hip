// Gram gradient kernel instantiations, dyadic order 1 (see grad_inst.h).
#define SK_LAM 1
#include "grad_inst.h"
