// fused_nw1.hip -- fused kernel instantiations with 1 wave per workgroup.
#define FUSED_NW 1
#include "fused_nw.inc"
