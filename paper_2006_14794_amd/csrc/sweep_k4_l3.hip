// Sweep kernel instantiations: lifted forward (Gaussian static kernel), dyadic order 3 (see sweep_inst.h).
#define SK_KIND 4
#define SK_LAM 3
#include "sweep_inst.h"
