// instantiations for models in 3 variable(s), numerator of degree 1, denominator of degree 2
#define RP_V 3
#define RP_D (1 | (2 << 4))
#include "rp_shapes.inc"
