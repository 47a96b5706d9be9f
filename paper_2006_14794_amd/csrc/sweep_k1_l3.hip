// Sweep kernel instantiations: forward with per-cell store, dyadic order 3 (see sweep_inst.h).
#define SK_KIND 1
#define SK_LAM 3
#include "sweep_inst.h"
