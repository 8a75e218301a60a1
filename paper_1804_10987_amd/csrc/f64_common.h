// f64_common.h -- FP64 building blocks of one wave per local system shared
// by the fused FP64 route (fused_f64.hip) and the refinement kernel
// (refine.hip).  Register layout of an UP x UP system (UP = 16 or 32): lane
// (r, c) = (lane / UP, lane % UP) holds column c of rows s R + r, s < NS
// (R = 64 / UP row groups, NS = UP / R slots), in FP64.  Internal.
#pragma once

#include "fused_kernel.h"

namespace pc {
namespace {

template <int UP>
struct F64L {
    static constexpr int R = 64 / UP;   // row groups
    static constexpr int NS = UP / R;   // slots per lane
    // LDS per wave: one staged row tile (32 x UP complex64), whose area then
    // holds the symbol chunk [KC][UP] and the FP32 Z chunk [UP][KC]
    // (complex64); the FP64 Z chunk [KC][UP] (complex FP64, precode in
    // FP64 only); a row buffer of UP complex FP64 for the inversion
    static constexpr size_t rows_bytes = (size_t)32 * UP * 8;
    static constexpr size_t s_bytes = (size_t)KC * UP * 8;
    static constexpr size_t z64_bytes = (size_t)KC * UP * 16;
    static constexpr size_t rowbuf_bytes = (size_t)UP * 16;
    // at 32 users the Gram passes through LDS as a full 32 x 32 complex FP64
    // matrix (gram32_to_regs), overlaying the rows and the FP64 Z chunk
    static constexpr size_t gram_bytes = UP == 32 ? (size_t)UP * UP * 16 : 0;
    static constexpr size_t base_bytes(bool p64) {
        return rows_bytes + (p64 ? z64_bytes : 0) > gram_bytes ? rows_bytes + (p64 ? z64_bytes : 0) : gram_bytes;
    }
    // the inversion's row buffer follows
    static constexpr size_t per_wave(bool p64) { return base_bytes(p64) + rowbuf_bytes; }
    static_assert(2 * s_bytes <= rows_bytes, "symbol and FP32 Z chunks overlay the rows");
    // symbols a lane loads per chunk
    static constexpr int SPL = UP * KC / 64;
};

// Position of user u in a staged row (and in a staged FP64 row of the
// inversion): users s R + r, s < NS, are contiguous for row group r.
template <int UP>
__device__ __forceinline__ int upos(int u) {
    return (u % F64L<UP>::R) * F64L<UP>::NS + u / F64L<UP>::R;
}

__device__ __forceinline__ double swap16_d(double v, bool odd) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    float a0, a1, b0, b1;
    swap16(ffrom((unsigned)b), a0, a1);
    swap16(ffrom((unsigned)(b >> 32)), b0, b1);
    const unsigned lo = fbits(odd ? a1 : a0), hi = fbits(odd ? b1 : b0);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}
__device__ __forceinline__ double swap32_d(double v, bool hi_half) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    float a0, a1, b0, b1;
    swap32(ffrom((unsigned)b), a0, a1);
    swap32(ffrom((unsigned)(b >> 32)), b0, b1);
    const unsigned lo = fbits(hi_half ? a1 : a0), hi = fbits(hi_half ? b1 : b0);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// Sum of v over the R row groups (lanes c, c + UP, ...): every lane of a
// column ends with the same sum.
template <int UP>
__device__ __forceinline__ double group_sum_d(double v) {
    const int lane = lane_id();
    if constexpr (UP == 16) {
        // rows of 16 lanes: pair 0+1, 2+3 (permlane16 swap), then halves
        v = v + swap16_d(v, (lane & 16) == 0);
    }
    return v + swap32_d(v, lane < 32);
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

__device__ __forceinline__ double readlane_d(double v, int l) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}

// Stages rows [row0, row0 + nr) of a local system (U users; its rows are one
// contiguous block of complex64 in HBM) in LDS as [row][upos(user)], rows
// >= nr and users >= U zero: entry e = lane + 64 i of the 32 x UP tile is
// loaded by lane e % 64, so each load instruction reads consecutive
// addresses; every load is issued (from a clamped in-range address) before
// the first LDS write.
template <int UP>
__device__ __forceinline__ void stage_rows_direct(const float2 *__restrict__ Hn, int U, int row0, int nr,
                                                  float2 *rowsL) {
    constexpr int PER = 32 * UP / 64;
    const int lane = lane_id();
    const float2 *src = Hn + (size_t)row0 * U;
    const int last = nr * U - 1;
    float2 v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = lane + 64 * i, row = e / UP, u = e % UP;
        const int g = row * U + u;
        v[i] = src[g < last ? g : last];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = lane + 64 * i, row = e / UP, u = e % UP;
        const bool in = row < nr && u < U;
        rowsL[row * UP + upos<UP>(u)] = in ? v[i] : make_float2(0.f, 0.f);
    }
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// G += H^H H over rows [row0, row0 + nrows) (nrows <= 32 NT) of a system
// with at most 16 users, on FP64 MFMA (v_mfma_f64_16x16x4f64, four rows per
// step).  A[i][k] and B[k][j] both
// come from lane j + 16 k (i, j: users; k: row), so every lane feeds its own
// entry h = H[row0 + 4 s + lane / 16][lane % 16] to both operands:
//   Re G += Re h^T Re h + Im h^T Im h,   Im G += Re h^T Im h - Im h^T Re h
// (conj(h_i) h_j).  D[i][j] lands in lane (i % 4, j), register i / 4: the
// inversion's register layout (slot q = i / 4 of row group r = i % 4).  Each
// lane converts two floats per four rows; the loads (consecutive addresses
// for U = 16) are all issued first, from clamped in-range addresses.
template <int NT>
__device__ __forceinline__ void gram_mfma16(const float2 *__restrict__ Hn, int U, int row0, int nrows,
                                            double (&gre)[4], double (&gim)[4]) {
    constexpr int STEPS = 8 * NT;
    const int lane = lane_id();
    const int kr = lane >> 4, u = lane & 15;
    const float2 *src = Hn + (size_t)row0 * U;
    float2 h[STEPS];
#pragma unroll
    for (int st = 0; st < STEPS; ++st) {
        const int row = 4 * st + kr;
        h[st] = src[row < nrows && u < U ? row * U + u : 0];
    }
    f64x4 are = {gre[0], gre[1], gre[2], gre[3]}, aim = {gim[0], gim[1], gim[2], gim[3]};
#pragma unroll
    for (int st = 0; st < STEPS; ++st) {
        // masked at the use, so that no select waits on a load in flight
        const bool in = 4 * st + kr < nrows && u < U;
        const double hr = in ? h[st].x : 0.0, hi = in ? h[st].y : 0.0;
        are = __builtin_amdgcn_mfma_f64_16x16x4f64(hr, hr, are, 0, 0, 0);
        are = __builtin_amdgcn_mfma_f64_16x16x4f64(hi, hi, are, 0, 0, 0);
        aim = __builtin_amdgcn_mfma_f64_16x16x4f64(hr, hi, aim, 0, 0, 0);
        aim = __builtin_amdgcn_mfma_f64_16x16x4f64(-hi, hr, aim, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        gre[q] = are[q];
        gim[q] = aim[q];
    }
}

// G += H^H H over the 32-row tile at row0 (rows past nrows zero) of a system
// with 17..32 users, on FP64 MFMA: the blocks (0,0), (0,1), (1,1) of users
// 0..15 / 16..31, with the operand layout of gram_mfma16 (lane l feeds
// row row0 + 4 s + l / 16, user l % 16 of its block), into acc[2 t] (real
// part) and acc[2 t + 1] (imaginary part) of block t.  The tile's loads are
// all issued first, from clamped in-range addresses.
__device__ __forceinline__ void gram_mfma32_tile(const float2 *__restrict__ Hn, int U, int row0, int nrows,
                                                 f64x4 (&acc)[6]) {
    const int lane = lane_id();
    const int kr = lane >> 4, u = lane & 15;
    const float2 *src = Hn + (size_t)row0 * U;
    float2 h0[8], h1[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) {
        const int row = 4 * st + kr;
        h0[st] = src[row < nrows && u < U ? row * U + u : 0];
        h1[st] = src[row < nrows && 16 + u < U ? row * U + 16 + u : 0];
    }
#pragma unroll
    for (int st = 0; st < 8; ++st) {
        // masked at the use, so that no select waits on a load in flight
        const bool rin = 4 * st + kr < nrows;
        const bool in0 = rin && u < U, in1 = rin && 16 + u < U;
        const double a = in0 ? h0[st].x : 0.0, b = in0 ? h0[st].y : 0.0;
        const double c = in1 ? h1[st].x : 0.0, d = in1 ? h1[st].y : 0.0;
        // conj(h_i) h_j: Re = a_i a'_j + b_i b'_j, Im = a_i b'_j - b_i a'_j
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, acc[0], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[1], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-b, a, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, c, acc[2], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(b, d, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, d, acc[3], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(-b, c, acc[3], 0, 0, 0);
        acc[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, c, acc[4], 0, 0, 0);
        acc[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(d, d, acc[4], 0, 0, 0);
        acc[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, d, acc[5], 0, 0, 0);
        acc[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(-d, c, acc[5], 0, 0, 0);
    }
}

// The 32 x 32 Hermitian Gram of gram_mfma32_tile's blocks in the register
// layout of UP = 32 (lane (r, c) holds G[2 s + r][c], s < 16), through this
// wave's LDS (gbuf: 32 x 32 complex FP64; block D[i][j] sits in lane
// (i % 4) 16 + j, register i / 4; block (1,0) is block (0,1) conjugated and
// transposed).
__device__ __forceinline__ void gram32_to_regs(const f64x4 (&acc)[6], cx<double> *gbuf, double (&gre)[16],
                                               double (&gim)[16]) {
    const int lane = lane_id();
    const int kr = lane >> 4, u = lane & 15;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = 4 * q + kr;
        gbuf[i * 32 + u] = {acc[0][q], acc[1][q]};
        gbuf[i * 32 + 16 + u] = {acc[2][q], acc[3][q]};
        gbuf[(16 + u) * 32 + i] = {acc[2][q], -acc[3][q]};
        gbuf[(16 + i) * 32 + 16 + u] = {acc[4][q], acc[5][q]};
    }
    wave_sync();
    const int r = lane >> 5, c = lane & 31;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const cx<double> g = gbuf[(2 * s + r) * 32 + c];
        gre[s] = g.re;
        gim[s] = g.im;
    }
    wave_sync();  // the area is rewritten by the staged symbols and rows
}

// G[s R + r][c] += sum over the staged tile's 32 rows of conj(h_{s R + r}) h_c.
template <int UP>
__device__ __forceinline__ void gram_rows(const float2 *rowsL, double (&gre)[F64L<UP>::NS],
                                          double (&gim)[F64L<UP>::NS]) {
    constexpr int R = F64L<UP>::R, NS = F64L<UP>::NS;
    const int lane = lane_id();
    const int r = lane / UP, c = lane % UP;
    const int pc = upos<UP>(c);
#pragma unroll 2
    for (int b = 0; b < 32; ++b) {
        const float2 hc = rowsL[b * UP + pc];
        const double xr = hc.x, xi = hc.y;
        const float4 *hu = (const float4 *)(rowsL + b * UP + r * NS);
#pragma unroll
        for (int s2 = 0; s2 < NS / 2; ++s2) {
            const float4 v = hu[s2];
            const double a0 = v.x, b0 = v.y, a1 = v.z, b1 = v.w;
            gre[2 * s2] = fma(a0, xr, fma(b0, xi, gre[2 * s2]));
            gim[2 * s2] = fma(a0, xi, fma(-b0, xr, gim[2 * s2]));
            gre[2 * s2 + 1] = fma(a1, xr, fma(b1, xi, gre[2 * s2 + 1]));
            gim[2 * s2 + 1] = fma(a1, xi, fma(-b1, xr, gim[2 * s2 + 1]));
        }
    }
    (void)R;
}

// The symbols of chunk k0 a lane stages: entry e = lane + 64 i of the
// [KC][UP] chunk (symbol e / UP, user e % UP), loaded from clamped in-range
// addresses (masked when staged).
template <int UP>
__device__ __forceinline__ void load_syms(const float2 *__restrict__ s, int k0, int kc, int n, int n_sc, int U,
                                          float2 (&v)[F64L<UP>::SPL]) {
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < F64L<UP>::SPL; ++i) {
        const int e = lane + 64 * i, k = e / UP, u = e % UP;
        const int kk = k < kc ? k : kc - 1, uu = u < U ? u : U - 1;
        v[i] = s[((size_t)(k0 + kk) * n_sc + n) * U + uu];
    }
}

template <int UP>
__device__ __forceinline__ void stage_syms(const float2 (&v)[F64L<UP>::SPL], int kc, int U, cx<float> *sb) {
    const int lane = lane_id();
#pragma unroll
    for (int i = 0; i < F64L<UP>::SPL; ++i) {
        const int e = lane + 64 * i, k = e / UP, u = e % UP;
        const bool in = k < kc && u < U;
        sb[k * UP + upos<UP>(u)] = {in ? v[i].x : 0.f, in ? v[i].y : 0.f};
    }
}

}  // namespace
}  // namespace pc
