// Sweep kernel instantiations: forward with per-cell store, dyadic order 1 (see sweep_inst.h).
#define SK_KIND 1
#define SK_LAM 1
#include "sweep_inst.h"
