// fused_launch.h -- launches of the fused kernel for one waves-per-workgroup
// count NW.  Each NW is compiled in its own translation unit
// (fused_nw{1,2,4}.hip) so the instantiations build in parallel.  Internal.
#pragma once

#include "common.h"

namespace pc {

struct FusedCall {
    int K, mode;  // symbols in this launch; kFull / kPrepare / kSymbols
    int maxt;     // channel tiles per wave held in registers (0: streamed)
    bool vec;     // U == tile width and a 16-byte aligned channel
    bool split;   // PD: one subcarrier per workgroup, maxt tiles per wave
    const float2 *H, *s;
    float2 *x;
    cx<float> *ainv;  // per-instance factors (prepare / symbols modes)
    float *scale_out;
    int *status;
};

// Enqueue one launch of fused_k<UP, PREC, MAXT, VEC, NW> for problem p (UP
// from p.U, PREC from prec, MAXT = a.maxt, VEC = a.vec): one wave per system (n_sc for PD,
// n_sc * C for FD), NW waves per workgroup.
hipError_t fused_launch_nw1(const Prob &p, int prec, const FusedCall &a, hipStream_t st);
hipError_t fused_launch_nw2(const Prob &p, int prec, const FusedCall &a, hipStream_t st);
hipError_t fused_launch_nw4(const Prob &p, int prec, const FusedCall &a, hipStream_t st);

}  // namespace pc
