// Sweep kernel instantiations: adjoint, dyadic order 2 (see sweep_inst.h).
#define SK_KIND 2
#define SK_LAM 2
#include "sweep_inst.h"
