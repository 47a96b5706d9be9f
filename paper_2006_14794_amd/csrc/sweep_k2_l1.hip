// Sweep kernel instantiations: adjoint, dyadic order 1 (see sweep_inst.h).
#define SK_KIND 2
#define SK_LAM 1
#include "sweep_inst.h"
