// Sweep kernel instantiations: pipelined row bands with a fitted top band, dyadic order 3 (see sweep_inst.h).
#define SK_KIND 6
#define SK_LAM 3
#include "sweep_inst.h"
