// instantiations for models in 4 variable(s) of degree 2
#define RP_V 4
#define RP_D 2
#include "rp_shapes.inc"
