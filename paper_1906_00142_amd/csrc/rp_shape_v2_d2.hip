// instantiations for models in 2 variable(s) of degree 2
#define RP_V 2
#define RP_D 2
#include "rp_shapes.inc"
