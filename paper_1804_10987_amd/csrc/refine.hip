// refine.hip -- one step of iterative refinement after the fused
// factorization, with the residual in FP64 from the complex64 channel.
//
// A refined call runs the fused kernel's per-frame part (Gram on MFMA at the
// call's precision -- FP32 or split FP16 / BF16 --, inversion, Lemma-1 factor
// and status) into a workspace of factors F = scale A^-1 (scale 1/beta for
// PD, w_c for FD), then this kernel, one wave per local system:
//
//   Gram      G = H^H H accumulated in FP64 over all the system's rows on
//             FP64 MFMA, 32-row tiles loaded coalesced (f64_common.h);
//             complex64 products are exact in FP64, so A = G + kappa I is the
//             exact regularized system the factorization rounded
//   solve     Z = F S per chunk of 16 symbols, in FP64 from the FP32 factor
//   residual  r = S - A Z / scale in FP64: with y = Z / scale the solution of
//             A y = S as solved, r = s - (kappa y + H^H (H y)) up to FP64
//             rounding (A is exactly Hermitian in FP64, so lane (r, c) forms
//             (A Z)[c] from its column of A)
//   update    Z += F r (one refinement step of the FP32 solve)
//   precode   X_c = H_c Z on FP32 MFMA from the rows loaded again, tile by tile
//
// Beta (PD) and the weights (FD) come from the factorization and are not
// refined.  An instance the prepare pass moved to the FP64 route (status
// PRECODE_ST_FP64) is solved on that route here (retry_f64.h).
#include "f64_common.h"

namespace pc {
namespace {

// Waves per workgroup and LDS per wave: the rows area (the symbol chunk
// [KC][UP] and the complex64 Z chunk [UP][KC]) and two FP64 chunks [KC][UP]
// (Z, then the residual); at 32 users the Gram passes through the first
// 16 KiB first.
template <int UP>
struct RefL {
    static constexpr int waves = UP == 16 ? 4 : 2;
    static constexpr size_t per_wave = F64L<UP>::rows_bytes + 2 * F64L<UP>::z64_bytes;
    static_assert(per_wave >= f64r::lds_bytes(UP), "FP64 retry area");
    static_assert(per_wave >= F64L<UP>::gram_bytes, "Gram area at 32 users");
};

// v = M w over one chunk: lane (r, c) holds M[c][q R + r] (mre / mim, q < NS);
// w is read as [k][upos(i)] complex FP64 (or complex64 when W32); the sum for
// row c of symbol k ends in every lane of column c.  conj_m: use conj(M[i][c])
// held as column c instead (M Hermitian).
template <int UP, bool W32>
__device__ __forceinline__ void apply_rows(const double (&mre)[F64L<UP>::NS], const double (&mim)[F64L<UP>::NS],
                                           const void *w, int k, double &vr, double &vi) {
    constexpr int NS = F64L<UP>::NS;
    const int r = lane_id() / UP;
    vr = 0.0;
    vi = 0.0;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double wr, wi;
        if constexpr (W32) {
            const cx<float> v = ((const cx<float> *)w)[k * UP + r * NS + q];
            wr = v.re;
            wi = v.im;
        } else {
            const cx<double> v = ((const cx<double> *)w)[k * UP + r * NS + q];
            wr = v.re;
            wi = v.im;
        }
        vr = fma(mre[q], wr, fma(-mim[q], wi, vr));
        vi = fma(mre[q], wi, fma(mim[q], wr, vi));
    }
    vr = group_sum_d<UP>(vr);
    vi = group_sum_d<UP>(vi);
}

// apply_rows for all 16 symbols of a chunk at 16 users, on FP64 MFMA:
// V^T = W^T M^T, K step q over indices 4 q .. 4 q + 3; lane (r, c) feeds
// W[4 q + r][c] (index 4 q + r, symbol c) as A[c][r] and its slot q,
// M[c][4 q + r], as B[r][c]; V[c][k] lands in lane (k % 4, c), register
// k / 4 (vr[t], vi[t] for symbol 4 t + r).
template <bool W32>
__device__ __forceinline__ void apply_mfma16(const double (&mre)[4], const double (&mim)[4], const void *w,
                                             double (&vr)[4], double (&vi)[4]) {
    const int lane = lane_id();
    const int r = lane >> 4, c = lane & 15;
    f64x4 dre = {0.0, 0.0, 0.0, 0.0}, dim = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double wr, wi;
        const int e = c * 16 + upos<16>(4 * q + r);
        if constexpr (W32) {
            const cx<float> v = ((const cx<float> *)w)[e];
            wr = v.re;
            wi = v.im;
        } else {
            const cx<double> v = ((const cx<double> *)w)[e];
            wr = v.re;
            wi = v.im;
        }
        dre = __builtin_amdgcn_mfma_f64_16x16x4f64(wr, mre[q], dre, 0, 0, 0);
        dre = __builtin_amdgcn_mfma_f64_16x16x4f64(-wi, mim[q], dre, 0, 0, 0);
        dim = __builtin_amdgcn_mfma_f64_16x16x4f64(wi, mre[q], dim, 0, 0, 0);
        dim = __builtin_amdgcn_mfma_f64_16x16x4f64(wr, mim[q], dim, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        vr[t] = dre[t];
        vi[t] = dim[t];
    }
}

// A = G + kappa I in the column layout with its imaginary part negated
// ((A Z)[c] = sum_i conj(A[i][c]) Z[i]), and F = scale A^-1 of system sys in
// the row layout (lane (r, c) holds F[c][q R + r]).
template <int UP>
__device__ __forceinline__ void ref_setup(double (&are)[F64L<UP>::NS], double (&aim)[F64L<UP>::NS],
                                          double (&fre)[F64L<UP>::NS], double (&fim)[F64L<UP>::NS], double kap,
                                          int U, int sys, const cx<float> *__restrict__ fac) {
    constexpr int R = F64L<UP>::R, NS = F64L<UP>::NS;
    const int lane = lane_id();
    const int r = lane / UP, c = lane % UP;
#pragma unroll
    for (int q = 0; q < NS; ++q)
        if (q * R + r == c) are[q] += kap;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int i = q * R + r;
        const bool in = c < U && i < U;
        const cx<float> v = fac[(size_t)sys * U * U + (in ? c * U + i : 0)];
        fre[q] = in ? v.re : 0.0;
        fim[q] = in ? v.im : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) aim[q] = -aim[q];
}

// One chunk of kc symbols from k0: Z = F S, r = S - A Z / scale, Z += F r
// (FP64), the refined Z rounded to complex64 into zb32 ([UP][KC]).  Ends
// with zb32 complete in this wave.
template <int UP>
__device__ __forceinline__ void ref_products(const double (&are)[F64L<UP>::NS], const double (&aim)[F64L<UP>::NS],
                                             const double (&fre)[F64L<UP>::NS], const double (&fim)[F64L<UP>::NS],
                                             bool ok, double inv_scale, const float2 *__restrict__ s, int k0,
                                             int kc, int n, int n_sc, int U, cx<float> *sb, cx<double> *zb,
                                             cx<double> *rb, cx<float> *zb32) {
    const int lane = lane_id();
    const int r = lane / UP, c = lane % UP;
    float2 sym[F64L<UP>::SPL];
    load_syms<UP>(s, k0, kc, n, n_sc, U, sym);
    stage_syms<UP>(sym, kc, U, sb);
    wave_sync();
    if constexpr (UP == 16) {
        // the three products on FP64 MFMA, every lane writing its 4 symbols
        double vr[4], vi[4];
        // Z = F S
        apply_mfma16<true>(fre, fim, sb, vr, vi);
#pragma unroll
        for (int t = 0; t < 4; ++t) zb[(4 * t + r) * UP + upos<UP>(c)] = {vr[t], vi[t]};
        wave_sync();
        // r = S - A Z / scale
        apply_mfma16<false>(are, aim, zb, vr, vi);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * t + r;
            const cx<float> sk = sb[k * UP + upos<UP>(c)];
            const bool live = ok && c < U && k < kc;
            rb[k * UP + upos<UP>(c)] = {live ? (double)sk.re - vr[t] * inv_scale : 0.0,
                                        live ? (double)sk.im - vi[t] * inv_scale : 0.0};
        }
        wave_sync();
        // Z += F r, rounded to complex64 for the precode
        apply_mfma16<false>(fre, fim, rb, vr, vi);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * t + r;
            const cx<double> z = zb[k * UP + upos<UP>(c)];
            const bool live = ok && c < U && k < kc;
            zb32[c * KC + k] = {live ? (float)(z.re + vr[t]) : 0.f, live ? (float)(z.im + vi[t]) : 0.f};
        }
        wave_sync();
    } else {
        // Z = F S
        for (int k = 0; k < KC; ++k) {
            double vr, vi;
            apply_rows<UP, true>(fre, fim, sb, k, vr, vi);
            if (r == 0) zb[k * UP + upos<UP>(c)] = {vr, vi};
        }
        wave_sync();
        // r = S - A Z / scale
        for (int k = 0; k < KC; ++k) {
            double vr, vi;
            apply_rows<UP, false>(are, aim, zb, k, vr, vi);
            if (r == 0) {
                const cx<float> sk = sb[k * UP + upos<UP>(c)];
                const bool live = ok && c < U && k < kc;
                rb[k * UP + upos<UP>(c)] = {live ? (double)sk.re - vr * inv_scale : 0.0,
                                            live ? (double)sk.im - vi * inv_scale : 0.0};
            }
        }
        wave_sync();
        // Z += F r, rounded to complex64 for the precode
        for (int k = 0; k < KC; ++k) {
            double vr, vi;
            apply_rows<UP, false>(fre, fim, rb, k, vr, vi);
            if (r == 0) {
                const cx<double> z = zb[k * UP + upos<UP>(c)];
                const bool live = ok && c < U && k < kc;
                zb32[c * KC + k] = {live ? (float)(z.re + vr) : 0.f, live ? (float)(z.im + vi) : 0.f};
            }
        }
        wave_sync();
    }
}

// X = H Z for the row tiles t0, t0 + dt, ... of a system on FP32 MFMA from
// the refined Z chunk zb32, the tiles loaded again.
template <int UP>
__device__ __forceinline__ void ref_precode(const float2 *__restrict__ Hn, int U, int r0, int nrows, int t0, int dt,
                                            const cx<float> *zb32, int k0, int kc, int n, int n_sc, int B,
                                            float2 *__restrict__ x) {
    const int ntile = (nrows + 31) >> 5;
    ZOp<UP, kF32> z;
    make_zop<UP, kF32>(zb32, KC, 1, kc, z);
    for (int t = t0; t < ntile; t += dt) {
        Tile<UP, kF32> tq;
        const int nt = min(32, nrows - 32 * t);
        load_tile<UP, kF32, false>(Hn, U, r0 + 32 * t, nt, tq);
        store_x(mfma_apply_packed<UP, kF32>(tq, z), r0 + 32 * t, nt, k0, kc, n, n_sc, B, x);
    }
}

template <int UP>
__device__ __forceinline__ void refine_system(const Prob &p, const Prob *__restrict__ pk, int sys, int K,
                                              const float2 *__restrict__ H, const float2 *__restrict__ s,
                                              float2 *__restrict__ x, const cx<float> *__restrict__ fac,
                                              const float *__restrict__ scale_in, const int *__restrict__ status,
                                              char *wb) {
    constexpr int NS = F64L<UP>::NS;
    const bool pd = p.arch == kPD;
    const int B = p.B, U = p.U, C = p.C, n_sc = p.n_sc;
    const int n = pd ? sys : sys / C;
    const int cl = pd ? 0 : sys - n * C;
    const int r0 = pd ? 0 : pk->off[cl], r1 = pd ? B : pk->off[cl + 1];
    const int nrows = r1 - r0, ntile = (nrows + 31) >> 5;
    if (on_f64_route(status, sys)) {
        f64r::instance(f64r::shape_of(p), pk, sys, K, false, H, s, x, nullptr, nullptr, wb);
        return;
    }
    const float2 *Hn = H + (size_t)n * B * U;
    cx<float> *sb = (cx<float> *)wb;                                          // [KC][UP] symbols (upos order)
    cx<float> *zb32 = (cx<float> *)(wb + F64L<UP>::s_bytes);                  // [UP][KC] refined Z (complex64)
    cx<double> *zb = (cx<double> *)(wb + F64L<UP>::rows_bytes);               // [KC][UP] Z (upos order)
    cx<double> *rb = (cx<double> *)(wb + F64L<UP>::rows_bytes + F64L<UP>::z64_bytes);  // [KC][UP] residual
    const double kap = pd ? (double)pd_kappa(p) : (double)fd_kappa_c(pk, cl);
    const float sv = scale_in[sys];
    // F = scale A^-1: scale = 1 / beta (PD) or w_c (FD); 0 for a failed instance
    const double scale = pd ? (sv > 0.f ? 1.0 / (double)sv : 0.0) : (double)sv;

    // A = G + kappa I in FP64 (column layout)
    double are[NS], aim[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) are[q] = aim[q] = 0.0;
    if constexpr (UP == 16) {
        for (int t = 0; t < ntile; ++t)
            gram_mfma16<1>(Hn, U, r0 + 32 * t, min(32, nrows - 32 * t), are, aim);  // FP64 MFMA
    } else {
        // FP64 MFMA blocks per tile, then through LDS into the column layout
        f64x4 acc[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) acc[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
        for (int t = 0; t < ntile; ++t) gram_mfma32_tile(Hn, U, r0 + 32 * t, min(32, nrows - 32 * t), acc);
        gram32_to_regs(acc, (cx<double> *)wb, are, aim);
    }
    double fre[NS], fim[NS];
    ref_setup<UP>(are, aim, fre, fim, kap, U, sys, fac);
    const bool ok = scale > 0.0;
    const double inv_scale = ok ? 1.0 / scale : 0.0;
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kc = min(KC, K - k0);
        ref_products<UP>(are, aim, fre, fim, ok, inv_scale, s, k0, kc, n, n_sc, U, sb, zb, rb, zb32);
        ref_precode<UP>(Hn, U, r0, nrows, 0, 1, zb32, k0, kc, n, n_sc, B, x);
        wave_sync();  // the chunks are rewritten by the next one
    }
}

// One PD subcarrier per workgroup of kSplitW waves: wave w forms the FP64
// partial Gram of the row tiles w, w + kSplitW, ... (the partials are added in
// LDS in fixed wave order), the master (wave 0) runs the three products of
// each symbol chunk, and every wave precodes its own tiles from the master's
// refined Z.  An instance on the FP64 route is solved there by the master.
constexpr int kSplitW = 4;

template <int UP>
struct SplitL {
    // per wave: its partial Gram (UP = 16: NS = 4 real and 4 imaginary parts
    // per lane; 32: the six 16 x 16 MFMA accumulators, 24 doubles per lane)
    static constexpr size_t part = (size_t)64 * (UP == 16 ? 8 : 24) * 8;
    static constexpr size_t bytes = RefL<UP>::per_wave + kSplitW * part;
};

template <int UP>
__global__ void __launch_bounds__(64 * kSplitW, 1)
    refine_split_k(Prob p, int K, const float2 *__restrict__ H, const float2 *__restrict__ s, float2 *__restrict__ x,
                   const cx<float> *__restrict__ fac, const float *__restrict__ scale_in,
                   const int *__restrict__ status) {
    extern __shared__ float4 smem_split[];
    constexpr int NS = F64L<UP>::NS;
    const Prob *pk = (const Prob *)__builtin_amdgcn_kernarg_segment_ptr();  // p: the first argument
    char *wb = (char *)smem_split;                                           // the master's buffers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    const int n = blockIdx.x, B = p.B, U = p.U, n_sc = p.n_sc;
    const int ntile = (B + 31) >> 5;
    if (on_f64_route(status, n)) {
        if (wave == 0) f64r::instance(f64r::shape_of(p), pk, n, K, false, H, s, x, nullptr, nullptr, wb);
        return;
    }
    const float2 *Hn = H + (size_t)n * B * U;
    double *part = (double *)(wb + RefL<UP>::per_wave);
    double are[NS], aim[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) are[q] = aim[q] = 0.0;
    if constexpr (UP == 16) {
        for (int t = wave; t < ntile; t += kSplitW)
            gram_mfma16<1>(Hn, U, 32 * t, min(32, B - 32 * t), are, aim);
        double *pw = part + (size_t)wave * 64 * 8;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pw[(2 * q) * 64 + lane] = are[q];
            pw[(2 * q + 1) * 64 + lane] = aim[q];
        }
        __syncthreads();
        if (wave == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double a = 0.0, b = 0.0;
#pragma unroll
                for (int w = 0; w < kSplitW; ++w) {
                    a += part[(size_t)w * 64 * 8 + (2 * q) * 64 + lane];
                    b += part[(size_t)w * 64 * 8 + (2 * q + 1) * 64 + lane];
                }
                are[q] = a;
                aim[q] = b;
            }
    } else {
        f64x4 acc[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) acc[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
        for (int t = wave; t < ntile; t += kSplitW) gram_mfma32_tile(Hn, U, 32 * t, min(32, B - 32 * t), acc);
        double *pw = part + (size_t)wave * 64 * 24;
#pragma unroll
        for (int t = 0; t < 6; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) pw[(4 * t + i) * 64 + lane] = acc[t][i];
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int t = 0; t < 6; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    double a = 0.0;
#pragma unroll
                    for (int w = 0; w < kSplitW; ++w) a += part[(size_t)w * 64 * 24 + (4 * t + i) * 64 + lane];
                    acc[t][i] = a;
                }
            gram32_to_regs(acc, (cx<double> *)wb, are, aim);
        }
    }
    cx<float> *sb = (cx<float> *)wb;
    cx<float> *zb32 = (cx<float> *)(wb + F64L<UP>::s_bytes);
    cx<double> *zb = (cx<double> *)(wb + F64L<UP>::rows_bytes);
    cx<double> *rb = (cx<double> *)(wb + F64L<UP>::rows_bytes + F64L<UP>::z64_bytes);
    double fre[NS], fim[NS];
    bool ok = false;
    double inv_scale = 0.0;
    if (wave == 0) {
        const float sv = scale_in[n];
        const double scale = sv > 0.f ? 1.0 / (double)sv : 0.0;
        ref_setup<UP>(are, aim, fre, fim, (double)pd_kappa(p), U, n, fac);
        ok = scale > 0.0;
        inv_scale = ok ? 1.0 / scale : 0.0;
    }
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kc = min(KC, K - k0);
        if (wave == 0) ref_products<UP>(are, aim, fre, fim, ok, inv_scale, s, k0, kc, n, n_sc, U, sb, zb, rb, zb32);
        __syncthreads();  // the refined Z chunk is complete
        ref_precode<UP>(Hn, U, 0, B, wave, kSplitW, zb32, k0, kc, n, n_sc, B, x);
        __syncthreads();  // the chunk buffers are rewritten by the next one
    }
}

template <int UP>
__global__ void __launch_bounds__(64 * RefL<UP>::waves, 2)
    refine_k(Prob p, int K, const float2 *__restrict__ H, const float2 *__restrict__ s, float2 *__restrict__ x,
             const cx<float> *__restrict__ fac, const float *__restrict__ scale_in, const int *__restrict__ status) {
    extern __shared__ float4 smem_ref[];
    const Prob *pk = (const Prob *)__builtin_amdgcn_kernarg_segment_ptr();  // p: the first argument
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sys = blockIdx.x * RefL<UP>::waves + wave;
    if (sys >= n_inst(p)) return;
    refine_system<UP>(p, pk, sys, K, H, s, x, fac, scale_in, status,
                      (char *)smem_ref + (size_t)wave * RefL<UP>::per_wave);
}

template <int UP>
hipError_t launch_refine(const Prob &p, const float2 *H, const float2 *s, float2 *x, const void *fac,
                         const float *scale_in, const int *status, hipStream_t st) {
    if (p.arch == kPD && p.B >= 32 * kSplitW) {
        // PD over at least kSplitW row tiles: the subcarrier split over a workgroup
        const size_t lds = SplitL<UP>::bytes;
        if (lds > 64 * 1024) {
            const hipError_t e = hipFuncSetAttribute((const void *)refine_split_k<UP>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((refine_split_k<UP>), dim3((unsigned)p.n_sc), dim3(64 * kSplitW), lds, st, p, p.K, H, s,
                           x, (const cx<float> *)fac, scale_in, status);
        return hipGetLastError();
    }
    constexpr int W = RefL<UP>::waves;
    const unsigned blocks = (unsigned)((n_inst(p) + W - 1) / W);
    const size_t lds = RefL<UP>::per_wave * W;
    hipLaunchKernelGGL((refine_k<UP>), dim3(blocks), dim3(64 * W), lds, st, p, p.K, H, s, x,
                       (const cx<float> *)fac, scale_in, status);
    return hipGetLastError();
}

}  // namespace

size_t fused_refine_ws_bytes(const Prob &p) {
    const size_t ni = (size_t)n_inst(p);
    return ((ni * p.U * p.U * sizeof(float2) + 255) & ~(size_t)255) + ((ni * sizeof(float) + 255) & ~(size_t)255) +
           ni * sizeof(int);
}

hipError_t fused_refine_run(const Prob &p, int precision, const float2 *H, const float2 *s, float2 *x,
                            float *scale_out, int *status, void *ws, hipStream_t st) {
    if (!fused_supported(p, precision)) return hipErrorNotSupported;
    const size_t ni = (size_t)n_inst(p);
    if (ni == 0) return hipSuccess;
    char *w = (char *)ws;
    float2 *fac = (float2 *)w;
    float *sc = (float *)(w + ((ni * p.U * p.U * sizeof(float2) + 255) & ~(size_t)255));
    int *stt = (int *)((char *)sc + ((ni * sizeof(float) + 255) & ~(size_t)255));
    hipError_t e = fused_prepare(p, precision, H, fac, sc, stt, st);
    if (e == hipSuccess && p.K > 0)
        e = p.U <= 16 ? launch_refine<16>(p, H, s, x, fac, sc, stt, st) : launch_refine<32>(p, H, s, x, fac, sc, stt, st);
    if (e == hipSuccess && scale_out) e = hipMemcpyAsync(scale_out, sc, ni * sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && status) e = hipMemcpyAsync(status, stt, ni * sizeof(int), hipMemcpyDeviceToDevice, st);
    return e;
}

}  // namespace pc
