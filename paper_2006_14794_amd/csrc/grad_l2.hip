// Gram gradient kernel instantiations, dyadic order 2 (see grad_inst.h).
#define SK_LAM 2
#include "grad_inst.h"
