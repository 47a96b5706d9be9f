// Sweep kernel instantiations: forward with the implicit scheme's cell factor, dyadic order 1 (see sweep_inst.h).
#define SK_KIND 5
#define SK_LAM 1
#include "sweep_inst.h"
