// Sweep kernel instantiations: persistent independent pairs, dyadic order 3 (see sweep_inst.h).
#define SK_KIND 3
#define SK_LAM 3
#include "sweep_inst.h"
