// degree dispatchers for models in 2 variable(s)
#define RP_V 2
#include "rp_shapes.inc"
