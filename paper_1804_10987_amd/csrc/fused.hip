// fused.hip -- single-problem launches of the fused PD / FD kernel on gfx950.
//
// One launch runs the whole per-subcarrier chain; only the precoded vectors,
// beta / weights and status are written back (the kernel body is in
// fused_kernel.h):
//
//   Gram        G_c = H_c^H H_c on MFMA over the real embedding
//               [Re h_u, Im h_u] of the columns: the 2U x 2U real Gram M
//               gives G = (M_rr + M_ii) + i (M_ri - M_ir) (local Gram,
//               Sec. III-B; PD sums the cluster Grams as a split-K reduction
//               over the waves, the on-chip form of the adder tree)
//   regularize  A = G + kappa I (PD) / A_c = G_c + kappa_c I (FD,
//               kappa_c = tau_c C kappa, Sec. III-C)
//   invert      A^-1 in registers, one wave per system (Gauss-Jordan
//               elimination; for Hermitian positive-definite A its pivots are
//               the squared diagonal of the Cholesky factor)
//   factor      t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1);
//               PD beta = sqrt(Es/rho^2 t); FD w_c = sqrt(rho_c^2/(t Es))
//   solve       Z = scale * A^-1 S for chunks of 16 symbols, on MFMA
//   precode     X_c = H_c Z on MFMA from the register-resident channel tiles
//               (Sec. III-B; FD x_c = w_c H_c A_c^-1 s, Sec. III-C), stored
//               coalesced
//
// PD: one 256-thread workgroup (4 wave64s) per subcarrier; wave w keeps the
// 32-row channel tiles t = w, w + 4, ... in registers from the Gram to the
// precode, so the channel is read from HBM exactly once.  FD: one workgroup
// per (subcarrier, group of four clusters), one cluster per wave, no
// workgroup barrier after the symbols are staged.
//
// Modes: full (Gram to precode), prepare (per-frame factors scale * A^-1 to
// device memory for the frame API and serving) and symbols (precode released
// symbols from stored factors, re-reading only the channel).
//
// MFMA precision (template PREC): FP32 (v_mfma_f32_32x32x2f32, exact FP32
// products) or split 16-bit: every operand x is written as hi + lo with
// hi = f16(x), lo = f16(x - hi) (or bf16) and a product a b is accumulated as
// ah bh + ah bl + al bh in FP32 (v_mfma_f32_32x32x16_f16 / _bf16).  Operands
// are scaled by powers of two into the FP16 range first and the FP32 results
// unscaled exactly.
#include "fused_kernel.h"

namespace pc {
namespace {

template <int UP, int ARCH, int PREC, int MAXT>
__global__ void __launch_bounds__(kThreads, (min_waves<UP, MAXT>()))
    fused_k(Prob p, int K, int mode, const float2 *__restrict__ H, const float2 *__restrict__ s,
            float2 *__restrict__ x, cx<float> *__restrict__ ainv_g, float *__restrict__ scale_out,
            int *__restrict__ status) {
    // cluster offsets read in place from the kernel-argument segment (p is the
    // first argument); indexing the by-value copy would force it to scratch
    const int *off = (const int *)((const char *)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(Prob, off));
    fused_body<UP, ARCH, PREC, MAXT>(p, off, blockIdx.x, K, mode, H, s, x, ainv_g, scale_out, status);
}

struct Call {
    int K, mode;
    const float2 *H, *s;
    float2 *x;
    cx<float> *ainv;
    float *scale_out;
    int *status;
};

template <int UP, int ARCH, int PREC, int MAXT>
hipError_t launch(const Prob &p, const Call &a, hipStream_t st) {
    const int K = a.K;
    const void *fn = (const void *)fused_k<UP, ARCH, PREC, MAXT>;
    const size_t lds = Lds<UP>::bytes(K);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const unsigned grid = (unsigned)p.n_sc * (ARCH == kPD ? 1u : (unsigned)((p.C + 3) / 4));
    hipLaunchKernelGGL((fused_k<UP, ARCH, PREC, MAXT>), dim3(grid), dim3(kThreads), lds, st, p, K, a.mode, a.H,
                       a.s, a.x, a.ainv, a.scale_out, a.status);
    return hipGetLastError();
}

template <int UP, int ARCH, int PREC>
hipError_t launch_t(int maxt, const Prob &p, const Call &a, hipStream_t st) {
    switch (maxt) {
        case 1: return launch<UP, ARCH, PREC, 1>(p, a, st);
        case 2: return launch<UP, ARCH, PREC, 2>(p, a, st);
        case 4: return launch<UP, ARCH, PREC, 4>(p, a, st);
        default:
            if constexpr (UP == 16) return launch<UP, ARCH, PREC, 8>(p, a, st);
            return hipErrorNotSupported;
    }
}

template <int UP, int ARCH>
hipError_t launch_prec(int prec, int maxt, const Prob &p, const Call &a, hipStream_t st) {
    switch (prec) {
        case kF32: return launch_t<UP, ARCH, kF32>(maxt, p, a, st);
        case kF16: return launch_t<UP, ARCH, kF16>(maxt, p, a, st);
        default: return launch_t<UP, ARCH, kBF16>(maxt, p, a, st);
    }
}

// Launches one mode over symbol slices of at most kMaxKFused.
hipError_t run_mode(const Prob &p, int precision, int mode, int K, const float2 *H, const float2 *s, float2 *x,
                    cx<float> *ainv, float *scale_out, int *status, hipStream_t st) {
    const int up = pick_up(p.U);
    const int prec = prec_of(precision);
    const int maxt = pick_maxt(p, up);
    for (int k0 = 0; k0 < K || (k0 == 0 && mode == kPrepare); k0 += kMaxKFused) {
        const int kk = mode == kPrepare ? 0 : (K - k0 < kMaxKFused ? K - k0 : kMaxKFused);
        Call a;
        a.K = kk;
        a.mode = mode;
        a.H = H;
        a.s = s ? s + (size_t)k0 * p.n_sc * p.U : nullptr;
        a.x = x ? x + (size_t)k0 * p.n_sc * p.B : nullptr;
        a.ainv = ainv;
        // factors are identical for every slice; write them once
        a.scale_out = k0 == 0 ? scale_out : nullptr;
        a.status = k0 == 0 ? status : nullptr;
        hipError_t e;
        if (up == 16)
            e = p.arch == kPD ? launch_prec<16, kPD>(prec, maxt, p, a, st) : launch_prec<16, kFD>(prec, maxt, p, a, st);
        else
            e = p.arch == kPD ? launch_prec<32, kPD>(prec, maxt, p, a, st) : launch_prec<32, kFD>(prec, maxt, p, a, st);
        if (e != hipSuccess) return e;
        if (mode == kPrepare) break;
    }
    return hipSuccess;
}

}  // namespace

bool fused_supported(const Prob &p, int precision) {
    if (prec_of(precision) < 0) return false;
    const int up = pick_up(p.U);
    if (up == 0) return false;
    if (pick_maxt(p, up) == 0) return false;
    const size_t lds = up == 16 ? Lds<16>::bytes(kMaxKFused) : Lds<32>::bytes(kMaxKFused);
    if (lds > kLdsMax - 256) return false;
    if (p.arch == kPD) return p.pd_fp64 == 0;
    for (int c = 0; c < p.C; ++c) {
        if (p.fp64[c]) return false;
        if (p.off[c + 1] - p.off[c] < p.U) return false;
    }
    return true;
}

hipError_t fused_run(const Prob &p, int precision, const float2 *H, const float2 *s, float2 *x, float *scale_out,
                     int *status, hipStream_t st) {
    if (!fused_supported(p, precision)) return hipErrorNotSupported;
    if (p.n_sc == 0) return hipSuccess;
    // full path: factors are written by the first slice only (ainv unused)
    return run_mode(p, precision, kFull, p.K, H, s, x, nullptr, scale_out, status, st);
}

hipError_t fused_prepare(const Prob &p, int precision, const float2 *H, float2 *ainv, float *scale_out, int *status,
                         hipStream_t st) {
    if (!fused_supported(p, precision)) return hipErrorNotSupported;
    if (p.n_sc == 0) return hipSuccess;
    return run_mode(p, precision, kPrepare, 0, H, nullptr, nullptr, (cx<float> *)ainv, scale_out, status, st);
}

hipError_t fused_symbols(const Prob &p, int precision, int nk, const float2 *H, const float2 *ainv, const float2 *s,
                         float2 *x, hipStream_t st) {
    if (!fused_supported(p, precision)) return hipErrorNotSupported;
    if (p.n_sc == 0 || nk == 0) return hipSuccess;
    return run_mode(p, precision, kSymbols, nk, H, s, x, (cx<float> *)ainv, nullptr, nullptr, st);
}

}  // namespace pc
