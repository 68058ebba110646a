// instantiations for models in 1 variable(s), numerator of degree 1, denominator of degree 2
#define RP_V 1
#define RP_D (1 | (2 << 4))
#include "rp_shapes.inc"
