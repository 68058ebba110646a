// degree dispatchers for models in 1 variable(s)
#define RP_V 1
#include "rp_shapes.inc"
