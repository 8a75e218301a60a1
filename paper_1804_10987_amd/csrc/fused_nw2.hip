// fused_nw2.hip -- fused kernel instantiations with 2 waves per workgroup.
#define FUSED_NW 2
#include "fused_nw.inc"
