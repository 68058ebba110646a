// instantiations for models in 4 variable(s) of degree 3
#define RP_V 4
#define RP_D 3
#include "rp_shapes.inc"
