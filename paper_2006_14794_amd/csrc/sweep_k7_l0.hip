// Sweep kernel instantiations: pipelined bands of one height, dyadic order 0
// (see sweep_inst.h).
#define SK_KIND 7
#define SK_LAM 0
#include "sweep_inst.h"
