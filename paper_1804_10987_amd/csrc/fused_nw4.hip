// fused_nw4.hip -- fused kernel instantiations with 4 waves per workgroup.
#define FUSED_NW 4
#include "fused_nw.inc"
