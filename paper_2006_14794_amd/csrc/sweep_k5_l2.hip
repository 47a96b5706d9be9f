// Sweep kernel instantiations: forward with the implicit scheme's cell factor, dyadic order 2 (see sweep_inst.h).
#define SK_KIND 5
#define SK_LAM 2
#include "sweep_inst.h"
