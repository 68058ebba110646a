// instantiations for models in 3 variable(s), numerator of degree 2, denominator of degree 3
#define RP_V 3
#define RP_D (2 | (3 << 4))
#include "rp_shapes.inc"
