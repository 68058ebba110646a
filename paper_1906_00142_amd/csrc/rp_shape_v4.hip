// degree dispatchers for models in 4 variable(s)
#define RP_V 4
#include "rp_shapes.inc"
