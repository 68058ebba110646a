// instantiations for models in 4 variable(s) of degree 1
#define RP_V 4
#define RP_D 1
#include "rp_shapes.inc"
