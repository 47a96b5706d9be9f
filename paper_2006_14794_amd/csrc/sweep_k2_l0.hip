// Sweep kernel instantiations: adjoint, dyadic order 0 (see sweep_inst.h).
#define SK_KIND 2
#define SK_LAM 0
#include "sweep_inst.h"
