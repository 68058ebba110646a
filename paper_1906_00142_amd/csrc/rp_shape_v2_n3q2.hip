// instantiations for models in 2 variable(s), numerator of degree 3, denominator of degree 2
#define RP_V 2
#define RP_D (3 | (2 << 4))
#include "rp_shapes.inc"
