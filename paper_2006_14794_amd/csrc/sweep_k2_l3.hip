// Sweep kernel instantiations: adjoint, dyadic order 3 (see sweep_inst.h).
#define SK_KIND 2
#define SK_LAM 3
#include "sweep_inst.h"
