// instantiations for models in 2 variable(s) of degree 3
#define RP_V 2
#define RP_D 3
#include "rp_shapes.inc"
