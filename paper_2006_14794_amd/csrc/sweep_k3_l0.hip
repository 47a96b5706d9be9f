// Sweep kernel instantiations: persistent independent pairs, dyadic order 0 (see sweep_inst.h).
#define SK_KIND 3
#define SK_LAM 0
#include "sweep_inst.h"
