// degree dispatchers for models in 3 variable(s)
#define RP_V 3
#include "rp_shapes.inc"
