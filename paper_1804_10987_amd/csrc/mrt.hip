// mrt.hip -- maximum ratio transmission, the matched-filter comparison precoder
// of the paper's evaluation (Sec. III-D), with the per-cluster power
// normalization of Sec. III-C (C = 1: centralized MRT):
//
//   x_c = w_c H_c s,   w_c = sqrt(rho_c^2 / (||H_c||_F^2 Es)),
//
// rho_c^2 = rho^2 / C or the call's per-cluster budgets.  A cluster whose
// ||H_c||_F^2 is zero or not finite gets w_c = 0 (x_c = 0) and status FAIL.
//
// Two kernels, one workgroup per subcarrier:
// - mrt_mfma_k (U = 16 or 32, a 16-byte aligned channel, B <= 512): each
//   wave loads its 32-row channel tiles in whole cache lines into registers
//   and moves them into the matrix-core operand layout through a per-wave LDS
//   scratch.  The tiles stay in registers: the row norms come from them, and
//   after one barrier for the cluster weights X^T = S^T H^T runs on FP32
//   matrix cores, 16 symbols per product, each output scaled by its row's
//   cluster weight and stored non-temporally.  HBM sees the channel once and
//   x once, and the workgroups are small enough that a frame's subcarriers
//   are resident together.
// - mrt_k (any shape): rows staged in LDS in chunks, one output per thread.
#include <stdint.h>

#include "fused_kernel.h"

namespace pc {
namespace {

// acc + a b
__device__ __forceinline__ float2 mac(float2 acc, float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}

// row norms [B]; cluster weights [C]
__host__ __device__ inline size_t mrt_mfma_head(int B, int C) {
    return ((size_t)(B + C) * sizeof(float) + 15) & ~(size_t)15;
}
template <int UP>
inline size_t mrt_mfma_lds(int B, int C, int NW) {
    return mrt_mfma_head(B, C) + (size_t)NW * 32 * Shape<UP>::RS * sizeof(float);
}

// Waves per SIMD the register budget must allow (what each shape needs
// without spilling).
constexpr int mrt_min_waves(int UP, int MAXT) { return UP == 16 ? (MAXT == 1 ? 8 : 4) : (MAXT == 1 ? 4 : 2); }

// Wave w of NW holds tiles w, w + NW, .. (MAXT at most) of the subcarrier's
// 32-row tiles; lane (j, g) = (lane % 32, lane / 32) holds row j of a tile,
// real columns g UP .. g UP + UP - 1 (users g UP / 2 ..).

template <int UP, int NW, int MAXT>
__global__ void __launch_bounds__(64 * NW, mrt_min_waves(UP, MAXT)) mrt_mfma_k(Prob p, const float2 *__restrict__ H,
                                                         const float2 *__restrict__ s, float2 *__restrict__ x,
                                                         float *__restrict__ wgt, int *__restrict__ status) {
    extern __shared__ float4 smem_mm[];
    const Prob *pk = (const Prob *)__builtin_amdgcn_kernarg_segment_ptr();  // p: the first argument
    const int n = blockIdx.x, wave = threadIdx.x >> 6, lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    const int B = p.B, C = p.C, K = p.K, n_sc = p.n_sc;
    const int ntile = (B + 31) >> 5;
    float *rn = (float *)smem_mm;  // [B] row norms
    float *cw = rn + B;            // [C] cluster weights
    float *scr = (float *)((char *)smem_mm + mrt_mfma_head(B, C)) + wave * 32 * Shape<UP>::RS;
    const float2 *Hn = H + (size_t)n * B * UP;
    Tile<UP, kF32> tl[MAXT];
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const int tt = wave + NW * q;
        load_tile_raw<UP, kF32>(Hn, tt < ntile ? 32 * tt : 0, tt < ntile ? min(32, B - 32 * tt) : 0, tl[q]);
    }
    SymRaw<UP> sym;
    if (K > 0) load_sym<UP>(s + (size_t)n * UP, (size_t)n_sc * UP, UP, min(K, KC), sym);
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const int tt = wave + NW * q;
        if (tt < ntile) {
            const int nr = min(32, B - 32 * tt);
            tile_to_precode<UP, kF32>(tl[q], nr, scr);  // rows >= nr read as zero
            float f = 0.f;
#pragma unroll
            for (int m = 0; m < UP; ++m) f = fmaf(tl[q].f[m], tl[q].f[m], f);
            f += __shfl_xor(f, 32);
            if (g == 0 && j < nr) rn[32 * tt + j] = f;
        }
    }
    __syncthreads();
    for (int cl = threadIdx.x; cl < C; cl += 64 * NW) {
        float f = 0.f;
        for (int b = pk->off[cl]; b < pk->off[cl + 1]; ++b) f += rn[b];
        const bool bad = !(f > 0.f) || !(f - f == 0.f);
        const float w = bad ? 0.f : sqrtf(fd_power_c(pk, cl) / (f * p.Es));
        cw[cl] = w;
        if (wgt) wgt[(size_t)n * C + cl] = w;
        if (status) status[(size_t)n * C + cl] = bad ? PRECODE_ST_FAIL : PRECODE_ST_OK;
    }
    __syncthreads();
    float wr[MAXT];  // the weight of the row this lane stores, per tile
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const int row = 32 * (wave + NW * q) + j;
        int lo = 0, hi = C - 1;  // cluster of the row: off[lo] <= row < off[lo + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pk->off[mid] <= row) lo = mid; else hi = mid - 1;
        }
        wr[q] = row < B ? cw[lo] : 0.f;
    }
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kc = min(KC, K - k0);
        if (k0 > 0) load_sym<UP>(s + ((size_t)k0 * n_sc + n) * UP, (size_t)n_sc * UP, UP, kc, sym);
        ZOp<UP, kF32> z;
        sym_to_zop<UP, kF32>(sym, UP, kc, z);
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int tt = wave + NW * q;
            if (tt < ntile) {
                floatx16 a = mfma_apply_tile<UP, kF32>(tl[q], z);
                a *= wr[q];
                store_x(a, 32 * tt, min(32, B - 32 * tt), k0, kc, n, n_sc, B, x);
            }
            __builtin_amdgcn_sched_barrier(0);  // one tile's product and stores at a time
        }
    }
}

// MRT, one workgroup per subcarrier, in two passes over chunks of antenna
// rows staged in LDS with coalesced loads (rows padded to U + 1 entries
// against bank conflicts): row norms, then per-cluster weights (and each
// row's weight), then the outputs x_k[b] = w_c sum_u H[b][u] s_k[u] with
// consecutive threads on consecutive rows of one symbol (coalesced stores),
// the symbols staged in LDS kMrtSyms at a time.  ONE: the subcarrier's
// channel fits one chunk, staged once for both passes (HBM sees it once);
// otherwise each chunk is staged again for the second pass.
constexpr size_t kMrtChunkLds = 48 * 1024;
constexpr int kMrtSyms = 16;

__host__ __device__ inline int mrt_chunk_rows(int B, int U) {
    const int r = (int)(kMrtChunkLds / ((size_t)(U + 1) * sizeof(float2)));
    return r < B ? r : B;
}
// row norms, then row weights [B]; cluster weights [C]; symbols [kMrtSyms][U]
__host__ __device__ inline size_t mrt_head(int B, int C, int U) {
    return (((size_t)(B + C) * sizeof(float) + 15) & ~(size_t)15) + (size_t)kMrtSyms * U * sizeof(float2);
}

template <bool ONE>
__global__ void __launch_bounds__(256) mrt_k(Prob p, const float2 *__restrict__ H, const float2 *__restrict__ s,
                                            float2 *__restrict__ x, float *__restrict__ wgt,
                                            int *__restrict__ status) {
    extern __shared__ float4 smem_mrt[];
    const Prob *pk = (const Prob *)__builtin_amdgcn_kernarg_segment_ptr();  // p: the first argument
    const int n = blockIdx.x, tid = threadIdx.x;
    const int B = p.B, U = p.U, C = p.C, K = p.K, ru = U + 1;
    const int R = mrt_chunk_rows(B, U);
    float *rn = (float *)smem_mrt;  // [B] row norms, then row weights
    float *cw = rn + B;             // [C] cluster weights
    float2 *sl = (float2 *)((char *)smem_mrt + (((size_t)(B + C) * sizeof(float) + 15) & ~(size_t)15));  // [kMrtSyms][U]
    float2 *Hl = (float2 *)((char *)smem_mrt + mrt_head(B, C, U));  // [R][U + 1]
    const float2 *Hn = H + (size_t)n * B * U;
    auto stage = [&](int b0, int nb) {
        __syncthreads();  // the previous chunk is consumed
        for (int e = tid; e < nb * U; e += 256) {
            const int b = e / U;
            Hl[b * ru + (e - b * U)] = Hn[(size_t)b0 * U + e];
        }
        __syncthreads();
    };
    for (int b0 = 0; b0 < B; b0 += R) {
        const int nb = min(R, B - b0);
        if (!ONE || b0 == 0) stage(b0, nb);
        for (int b = tid; b < nb; b += 256) {
            float f = 0.f;
            for (int u = 0; u < U; ++u) {
                const float2 h = Hl[b * ru + u];
                f = fmaf(h.x, h.x, fmaf(h.y, h.y, f));
            }
            rn[b0 + b] = f;
        }
    }
    __syncthreads();
    for (int cl = tid; cl < C; cl += 256) {
        float f = 0.f;
        for (int b = pk->off[cl]; b < pk->off[cl + 1]; ++b) f += rn[b];
        const bool bad = !(f > 0.f) || !(f - f == 0.f);
        const float w = bad ? 0.f : sqrtf(fd_power_c(pk, cl) / (f * p.Es));
        cw[cl] = w;
        if (wgt) wgt[(size_t)n * C + cl] = w;
        if (status) status[(size_t)n * C + cl] = bad ? PRECODE_ST_FAIL : PRECODE_ST_OK;
    }
    __syncthreads();
    // each row's weight, over the row norms (no longer needed)
    for (int b = tid; b < B; b += 256) {
        int lo = 0, hi = C - 1;  // cluster of row b: off[lo] <= b < off[lo + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pk->off[mid] <= b) lo = mid; else hi = mid - 1;
        }
        rn[b] = cw[lo];
    }
    for (int b0 = 0; b0 < B; b0 += R) {
        const int nb = min(R, B - b0);
        if (!ONE) stage(b0, nb);
        for (int k0 = 0; k0 < K; k0 += kMrtSyms) {
            const int ks = min(kMrtSyms, K - k0);
            __syncthreads();  // the previous symbols are consumed (and the row weights written)
            for (int e = tid; e < ks * U; e += 256) {
                const int kk = e / U;
                sl[e] = s[((size_t)(k0 + kk) * p.n_sc + n) * U + (e - kk * U)];
            }
            __syncthreads();
            for (int o = tid; o < nb * ks; o += 256) {
                const int kk = o / nb, b = o - kk * nb;
                const float2 *sk = sl + kk * U;
                const float2 *hb = Hl + b * ru;
                float2 acc = make_float2(0.f, 0.f);
                for (int u = 0; u < U; ++u) acc = mac(acc, hb[u], sk[u]);
                const float w = rn[b0 + b];
                __builtin_nontemporal_store((floatx2){acc.x * w, acc.y * w},
                                            (floatx2 *)(x + ((size_t)(k0 + kk) * p.n_sc + n) * B + b0 + b));
            }
        }
    }
}

}  // namespace

template <int UP, int NW, int MAXT>
static hipError_t mrt_mfma_launch(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *wgt,
                                  int *status, hipStream_t st) {
    hipLaunchKernelGGL((mrt_mfma_k<UP, NW, MAXT>), dim3(p.n_sc), dim3(64 * NW), mrt_mfma_lds<UP>(p.B, p.C, NW), st, p,
                       H, s, x, wgt, status);
    return hipGetLastError();
}

hipError_t mrt_run(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *wgt, int *status,
                   hipStream_t st) {
    if (p.n_sc == 0) return hipSuccess;
    const int ntile = (p.B + 31) / 32;
    // 8 waves of one tile each took 21 us per frame at 256 antennas / 16 users
    // (4 waves of two tiles: 23 us); 8 waves of two tiles 181 us at 512 / 32
    // (4 of four: 189 us).
    if ((p.U == 16 || p.U == 32) && ((uintptr_t)H & 15) == 0 && ntile <= 16) {
        if (p.U == 16) {
            if (ntile <= 4) return mrt_mfma_launch<16, 4, 1>(p, H, s, x, wgt, status, st);
            if (ntile <= 8) return mrt_mfma_launch<16, 8, 1>(p, H, s, x, wgt, status, st);
            return mrt_mfma_launch<16, 8, 2>(p, H, s, x, wgt, status, st);
        }
        if (ntile <= 4) return mrt_mfma_launch<32, 4, 1>(p, H, s, x, wgt, status, st);
        if (ntile <= 8) return mrt_mfma_launch<32, 8, 1>(p, H, s, x, wgt, status, st);
        return mrt_mfma_launch<32, 8, 2>(p, H, s, x, wgt, status, st);
    }
    const int R = mrt_chunk_rows(p.B, p.U);
    const size_t lds = mrt_head(p.B, p.C, p.U) + (size_t)R * (p.U + 1) * sizeof(float2);
    if (lds > 64 * 1024) {
        const void *fn = R == p.B ? (const void *)mrt_k<true> : (const void *)mrt_k<false>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (R == p.B)
        hipLaunchKernelGGL(mrt_k<true>, dim3(p.n_sc), dim3(256), lds, st, p, H, s, x, wgt, status);
    else
        hipLaunchKernelGGL(mrt_k<false>, dim3(p.n_sc), dim3(256), lds, st, p, H, s, x, wgt, status);
    return hipGetLastError();
}

}  // namespace pc
