// Sweep kernel instantiations: forward, dyadic order 0 (see sweep_inst.h).
#define SK_KIND 0
#define SK_LAM 0
#include "sweep_inst.h"
