// Sweep kernel instantiations: pipelined bands of one height, dyadic order 2
// (see sweep_inst.h).
#define SK_KIND 7
#define SK_LAM 2
#include "sweep_inst.h"
