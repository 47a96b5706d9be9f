// Sweep kernel instantiations: pipelined row bands with a fitted top band, dyadic order 2 (see sweep_inst.h).
#define SK_KIND 6
#define SK_LAM 2
#include "sweep_inst.h"
