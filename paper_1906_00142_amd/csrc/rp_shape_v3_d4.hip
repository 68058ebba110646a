// instantiations for models in 3 variable(s) of degree 4
#define RP_V 3
#define RP_D 4
#include "rp_shapes.inc"
