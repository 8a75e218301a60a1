// fused_nw8.hip -- fused kernel instantiations with 8 waves per workgroup.
#define FUSED_NW 8
#include "fused_nw.inc"
