// instantiations for models in 3 variable(s) of degree 2
#define RP_V 3
#define RP_D 2
#include "rp_shapes.inc"
