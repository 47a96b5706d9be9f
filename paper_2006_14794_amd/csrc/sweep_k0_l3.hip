// Sweep kernel instantiations: forward, dyadic order 3 (see sweep_inst.h).
#define SK_KIND 0
#define SK_LAM 3
#include "sweep_inst.h"
