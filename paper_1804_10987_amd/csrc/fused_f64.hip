// fused_f64.hip -- the FP64 route in one fused launch: local systems whose
// conditioning calls for FP64 (U / B_eff >= fp64_ratio, or precision FP64 not
// requested: see fused_f64_supported) with U <= 16 and U <= B_eff <= 32 rows.
//
// One wave per local system (FD cluster c of subcarrier n, or a PD subcarrier
// of at most 32 antennas), four systems per workgroup, no workgroup barrier:
//
//   load      the system's rows (one 32-row tile) into registers, in the
//             precode's operand layout (as the FP32 kernel)
//   Gram      G_c = H_c^H H_c in FP64 on the VALU: the rows go to LDS as
//             complex64; lane (r, c) accumulates G[4s + r][c], s = 0..3, over
//             the rows (complex64 products are exact in FP64)
//   invert    A_c = G_c + kappa_c I inverted in FP64 by Gauss-Jordan without
//             pivoting (Hermitian positive definite), in the register layout
//             of the FP32 inversion
//   factor    t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1) in FP64; PD beta,
//             FD w_c = sqrt(rho_c^2 / (t Es)) (Sec. III-C)
//   solve     Z = scale A^-1 S in FP64 per chunk of 16 symbols, rounded to
//             complex64
//   precode   X_c = H_c Z on FP32 MFMA from the register tile (Sec. III-B/C)
//
// Status of every instance: PRECODE_ST_FP64, plus PRECODE_ST_FAIL when a
// pivot is not above kRelPivot64 times its original diagonal entry or t is
// not positive (then x = 0 and the scale output is 0).
#include "fused_kernel.h"

namespace pc {
namespace {

constexpr int kF64Waves = 4;
constexpr int kF64Up = 16;
// LDS per wave: the rows (32 x 16 complex64) then A^-1 (16 x 16 complex
// FP64) in the same area, and the symbol chunk / Z chunk (16 x 16 complex64).
constexpr size_t kF64RowsBytes = 32 * kF64Up * 8;
constexpr size_t kF64ZBytes = kF64Up * KC * 8;
constexpr size_t kF64PerWave = kF64RowsBytes + kF64ZBytes;
static_assert(kF64Up * kF64Up * 16 <= kF64RowsBytes, "A^-1 overlays the rows");

__device__ __forceinline__ double dpp_bcast16_d(double v, int k) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const float lo = dpp_bcast16_dyn(ffrom((unsigned)b), k);
    const float hi = dpp_bcast16_dyn(ffrom((unsigned)(b >> 32)), k);
    return __builtin_bit_cast(double, (unsigned long long)fbits(lo) | ((unsigned long long)fbits(hi) << 32));
}

// lane (r, c) receives v of lane (rk, c) (row groups of 16 lanes)
__device__ __forceinline__ double bperm_group_d(double v, int c4, int rk) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int addr = rk * 16 * 4 + c4;
    const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

// Gauss-Jordan inversion of the m x m Hermitian positive-definite system in
// registers (lane (r, c) holds column c of rows 4s + r, s = 0..3; rows and
// columns >= m are the identity), in FP64: step k divides row k by the pivot
// and eliminates column k from every other row.  Returns whether every pivot
// is finite and above kRelPivot64 times its original diagonal entry d0.
__device__ bool wave_inverse_f64(double (&re)[4], double (&im)[4], int m, double d0) {
    const int lane = lane_id();
    const int r = lane >> 4, c = lane & 15, c4 = 4 * c;
    double pv = 1.0;
    double akc_re = bperm_group_d(re[0], c4, 0);
    double akc_im = bperm_group_d(im[0], c4, 0);
#pragma unroll
    for (int k = 0; k < kF64Up; ++k) {
        const int sk = k >> 2, rk = k & 3;
        const double piv = dpp_bcast16_d(akc_re, k);
        const bool iscol = c == k;
        pv = iscol ? piv : pv;
        // 1 / piv: hardware reciprocal and two Newton steps (the error
        // squares per step: below an ulp of FP64); a zero or non-finite
        // pivot fails the pivot test anyway
        double inv = __builtin_amdgcn_rcp(piv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        const double mre = iscol ? 1.0 + inv : akc_re * inv;
        const double mim = iscol ? 0.0 : akc_im * inv;
        const double rowre = iscol ? inv : mre, rowim = mim;
        const int k1 = k + 1, s1 = k1 >> 2;
        auto update = [&](int s) {
            const double aik_re = dpp_bcast16_d(re[s], k), aik_im = dpp_bcast16_d(im[s], k);
            double x = re[s] - (aik_re * mre - aik_im * mim);
            double y = im[s] - (aik_re * mim + aik_im * mre);
            if (s == sk) {
                const bool isrow = r == rk;
                x = isrow ? rowre : x;
                y = isrow ? rowim : y;
            }
            re[s] = x;
            im[s] = y;
        };
        if (k1 < kF64Up) {
            update(s1);
            akc_re = bperm_group_d(re[s1], c4, k1 & 3);
            akc_im = bperm_group_d(im[s1], c4, k1 & 3);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (k1 >= kF64Up || s != s1) update(s);
    }
    (void)m;
    return __all((pv > kRelPivot64 * d0) && (pv < (double)INFINITY));
}

template <bool VEC>
__device__ __forceinline__ void f64_system(const Prob &p, const int *__restrict__ off, int sys, int K,
                                           const float2 *__restrict__ H, const float2 *__restrict__ s,
                                           float2 *__restrict__ x, float *__restrict__ scale_out,
                                           int *__restrict__ status, char *wb) {
    const int lane = lane_id();
    const int r = lane >> 4, c = lane & 15;
    const bool pd = p.arch == kPD;
    const int B = p.B, U = p.U, C = p.C, n_sc = p.n_sc;
    const int n = pd ? sys : sys / C;
    const int cl = pd ? 0 : sys - n * C;
    const int r0 = pd ? 0 : off[cl], r1 = pd ? B : off[cl + 1];
    const int nrows = r1 - r0;
    const float2 *Hn = H + (size_t)n * B * U;
    float2 *rows = (float2 *)wb;                 // [32][16] complex64, then A^-1
    cx<double> *ainv = (cx<double> *)wb;          // [16][16] complex FP64
    cx<float> *zb = (cx<float> *)(wb + kF64RowsBytes);  // [16][KC] complex64
    const double kap = pd ? (double)pd_kappa(p) : (double)fd_kappa(p);

    Tile<kF64Up, kF32> tl;
    load_tile<kF64Up, kF32, VEC>(Hn, U, r0, nrows, tl);

    // rows to LDS as [row][user] complex64, rows >= nrows and users >= U zero
    {
        const int j = lane & 31, g = lane >> 5;
        const bool live = j < nrows;
#pragma unroll
        for (int m2 = 0; m2 < 8; m2 += 2) {
            const int u = g * 8 + m2;
            float4 v;
            v.x = (live && u < U) ? tl.f[2 * m2] : 0.f;
            v.y = (live && u < U) ? tl.f[2 * m2 + 1] : 0.f;
            v.z = (live && u + 1 < U) ? tl.f[2 * m2 + 2] : 0.f;
            v.w = (live && u + 1 < U) ? tl.f[2 * m2 + 3] : 0.f;
            *(float4 *)(rows + j * kF64Up + u) = v;
        }
    }
    wave_sync();
    // Gram in FP64: lane (r, c) forms G[4s + r][c] = sum_j conj(h_j,4s+r) h_jc
    double gre[4] = {0.0, 0.0, 0.0, 0.0}, gim[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int j = 0; j < 32; ++j) {
        const float2 hc = rows[j * kF64Up + c];
        const double xr = hc.x, xi = hc.y;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float2 hu = rows[j * kF64Up + 4 * q + r];
            const double ar = hu.x, ai = hu.y;
            gre[q] = fma(ar, xr, fma(ai, xi, gre[q]));
            gim[q] = fma(ar, xi, fma(-ai, xr, gim[q]));
        }
    }
    wave_sync();  // the rows area becomes A^-1
    // A = G + kappa I, identity past U
    double d0 = 1.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = 4 * q + r;
        const bool in = i < U && c < U;
        if (i == c) {
            gre[q] = in ? gre[q] + kap : 1.0;
            d0 = gre[q];
        } else if (!in) {
            gre[q] = 0.0;
        }
        gim[q] = in && i != c ? gim[q] : 0.0;
    }
    // d0 of column c lives in lane (c & 3, c) slot c >> 2; broadcast it down the column
    d0 = bperm_group_d(d0, 4 * c, c & 3);
    // invert 2^-e A with its largest diagonal entry in [0.5, 1), so that no
    // pivot exceeds 1 and 1 + 1/pivot in the update keeps 1/pivot exact to an
    // ulp; A^-1 = 2^-e (2^-e A)^-1
    const double dmax = wave_max_d(c < U ? d0 : 0.0);
    int e = 0;
    if (dmax > 0.0 && dmax < (double)INFINITY) e = ilogb(dmax) + 1;
    const double sc = ldexp(1.0, -e);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool in = 4 * q + r < U && c < U;
        gre[q] = in ? gre[q] * sc : gre[q];
        gim[q] = in ? gim[q] * sc : gim[q];
    }
    d0 = c < U ? d0 * sc : d0;
    bool ok = wave_inverse_f64(gre, gim, U, d0);
    double tr = 0.0, fro = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = 4 * q + r;
        const double vr = gre[q] * sc, vi = gim[q] * sc;
        if (i < U && c < U) {
            fro += vr * vr + vi * vi;
            if (i == c) tr += vr;
        }
        ainv[i * kF64Up + c] = {vr, vi};
    }
    tr = wave_sum_d(tr);
    fro = wave_sum_d(fro);
    const double t = tr - kap * fro;
    ok = ok && t > 0.0 && t < (double)INFINITY;
    double out = 0.0, scale = 0.0;
    if (ok) {
        if (pd) {
            out = sqrt((double)p.Es / (double)p.power * t);  // beta
            scale = 1.0 / out;
        } else {
            out = sqrt((double)p.power / (double)C / (t * (double)p.Es));  // w_c
            scale = out;
        }
    }
    if (lane == 0) {
        if (scale_out) scale_out[sys] = (float)out;
        if (status) status[sys] = (ok ? PRECODE_ST_OK : PRECODE_ST_FAIL) | PRECODE_ST_FP64;
    }
    wave_sync();
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kc = min(KC, K - k0);
        // symbol chunk to LDS as [user][k] complex64 (zero past U / kc)
#pragma unroll
        for (int e = lane; e < kF64Up * KC; e += 64) {
            const int u = e / KC, k = e % KC;
            float2 v = make_float2(0.f, 0.f);
            if (u < U && k < kc) v = s[((size_t)(k0 + k) * n_sc + n) * U + u];
            zb[e] = {v.x, v.y};
        }
        wave_sync();
        // Z(u, k) = scale (A^-1 S)(u, k) in FP64: lane -> u = lane & 15, k = (lane >> 4) + 4 q
        cx<double> zacc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) zacc[q] = {0.0, 0.0};
        const int u = lane & 15;
#pragma unroll 4
        for (int v = 0; v < kF64Up; ++v) {
            const cx<double> a = ainv[u * kF64Up + v];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const cx<float> sv = zb[v * KC + (lane >> 4) + 4 * q];
                const double sr = sv.re, si = sv.im;
                zacc[q].re = fma(a.re, sr, fma(-a.im, si, zacc[q].re));
                zacc[q].im = fma(a.re, si, fma(a.im, sr, zacc[q].im));
            }
        }
        wave_sync();  // every read of the symbol chunk is done
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = (lane >> 4) + 4 * q;
            const bool live = ok && u < U && k < kc;
            zb[u * KC + k] = {live ? (float)(scale * zacc[q].re) : 0.f, live ? (float)(scale * zacc[q].im) : 0.f};
        }
        wave_sync();
        ZOp<kF64Up, kF32> z;
        make_zop<kF64Up, kF32>(zb, KC, 1, kc, z);
        store_x(mfma_apply_packed<kF64Up, kF32>(tl, z), r0, nrows, k0, kc, n, n_sc, B, x);
        wave_sync();  // zb is rewritten by the next chunk
    }
}

template <bool VEC>
__global__ void __launch_bounds__(64 * kF64Waves, 2)
    fused_f64_k(Prob p, int K, const float2 *__restrict__ H, const float2 *__restrict__ s, float2 *__restrict__ x,
                float *__restrict__ scale_out, int *__restrict__ status) {
    extern __shared__ float4 smem_f64[];
    const int *off = (const int *)((const char *)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(Prob, off));
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sys = blockIdx.x * kF64Waves + wave;
    if (sys >= n_inst(p)) return;
    f64_system<VEC>(p, off, sys, K, H, s, x, scale_out, status, (char *)smem_f64 + (size_t)wave * kF64PerWave);
}

}  // namespace

bool fused_f64_supported(const Prob &p, int precision, int K) {
    if (K < 1 || p.U > kF64Up || precision == PRECODE_PREC_FP64) return false;
    if (p.arch == kPD) return p.pd_fp64 && p.B >= p.U && p.B <= 32;
    for (int c = 0; c < p.C; ++c) {
        const int bc = p.off[c + 1] - p.off[c];
        if (!p.fp64[c] || bc < p.U || bc > 32) return false;
    }
    return true;
}

hipError_t fused_f64_run(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *scale_out, int *status,
                         hipStream_t st) {
    const int ni = n_inst(p);
    if (ni == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((ni + kF64Waves - 1) / kF64Waves);
    const size_t lds = kF64PerWave * kF64Waves;
    const bool vec = pick_vec(p, H);
    if (vec)
        hipLaunchKernelGGL((fused_f64_k<true>), dim3(blocks), dim3(64 * kF64Waves), lds, st, p, p.K, H, s, x,
                           scale_out, status);
    else
        hipLaunchKernelGGL((fused_f64_k<false>), dim3(blocks), dim3(64 * kF64Waves), lds, st, p, p.K, H, s, x,
                           scale_out, status);
    return hipGetLastError();
}

}  // namespace pc
