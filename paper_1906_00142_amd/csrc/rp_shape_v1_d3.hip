// instantiations for models in 1 variable(s) of degree 3
#define RP_V 1
#define RP_D 3
#include "rp_shapes.inc"
