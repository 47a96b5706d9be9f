// Sweep kernel instantiations: forward, dyadic order 2 (see sweep_inst.h).
#define SK_KIND 0
#define SK_LAM 2
#include "sweep_inst.h"
