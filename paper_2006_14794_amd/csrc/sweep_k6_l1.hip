// Sweep kernel instantiations: pipelined row bands of few long pairs, dyadic order 1 (see sweep_inst.h).
#define SK_KIND 6
#define SK_LAM 1
#include "sweep_inst.h"
