// Sweep kernel instantiations: pipelined row bands with a fitted top band, dyadic order 0 (see sweep_inst.h).
#define SK_KIND 6
#define SK_LAM 0
#include "sweep_inst.h"
