// Sweep kernel instantiations: persistent independent pairs, dyadic order 2 (see sweep_inst.h).
#define SK_KIND 3
#define SK_LAM 2
#include "sweep_inst.h"
