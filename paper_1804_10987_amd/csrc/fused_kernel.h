// fused_kernel.h -- device code of the fused PD / FD kernel (one problem per
// workgroup set), shared by the single-problem launches (fused.hip) and the
// heterogeneous batch launches (batch.hip).  Internal to the library.
#pragma once
#include <stddef.h>

#include "common.h"
#include "retry_f64.h"

namespace pc {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int KC = 16;  // symbols per MFMA chunk: 2*KC = 32 rows of X^T

enum Prec { kF32 = 0, kF16 = 1, kBF16 = 2 };

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Orders LDS accesses of one wave (a wave's LDS operations execute in order;
// this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ unsigned fbits(float v) { return __builtin_bit_cast(unsigned, v); }
__device__ __forceinline__ float ffrom(unsigned v) { return __builtin_bit_cast(float, v); }

// The two results of a gfx950 permlane swap of v with itself, as floats:
// permlane16_swap gives [r0, r0, r2, r2] and [r1, r1, r3, r3] over the four
// DPP rows r0..r3 of v; permlane32_swap gives [lo, lo] and [hi, hi] over the
// two half-waves.  (The elements are copied out by value: a bit cast applied
// directly to an element of the returned vector reads element 0.)
__device__ __forceinline__ void swap16(float v, float &a, float &b) {
    const auto p = __builtin_amdgcn_permlane16_swap(fbits(v), fbits(v), false, false);
    const unsigned p0 = p[0], p1 = p[1];
    a = ffrom(p0);
    b = ffrom(p1);
}
__device__ __forceinline__ void swap32(float v, float &a, float &b) {
    const auto q = __builtin_amdgcn_permlane32_swap(fbits(v), fbits(v), false, false);
    const unsigned q0 = q[0], q1 = q[1];
    a = ffrom(q0);
    b = ffrom(q1);
}

// Wave-wide sum and max from DPP (within rows of 16 lanes) and the permlane
// swaps (across rows), no LDS.  Every lane ends with the same bits: each step
// adds a lane's value to its partner's, and both partners form the same
// (commutative) sum.
template <int CTRL>
__device__ __forceinline__ float dpp_c(float v) {
    return ffrom(__builtin_amdgcn_mov_dpp((int)fbits(v), CTRL, 0xf, 0xf, true));
}
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_c<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_c<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_c<0x141>(v);  // row_half_mirror
    v += dpp_c<0x140>(v);  // row_mirror
    float a, b;
    swap16(v, a, b);
    swap32(a + b, a, b);
    return a + b;
}

__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_c<0xB1>(v));
    v = fmaxf(v, dpp_c<0x4E>(v));
    v = fmaxf(v, dpp_c<0x141>(v));
    v = fmaxf(v, dpp_c<0x140>(v));
    float a, b;
    swap16(v, a, b);
    swap32(fmaxf(a, b), a, b);
    return fmaxf(a, b);
}

// Power-of-two exponent e with m * 2^e in [2^13, 2^14) (0 for m = 0): the
// scale that brings operands of magnitude <= m into the FP16 range while
// keeping their low parts away from subnormals.
__device__ __forceinline__ int fp16_exp(float m) { return m > 0.f ? 13 - ilogbf(m) : 0; }

template <int UP>
struct Shape {
    static constexpr int NT = (2 * UP) / 32;       // 32-wide real column tiles
    static constexpr int NTT = NT * (NT + 1) / 2;  // tiles with ti <= tj
    static constexpr int LDc = UP + 2;             // slot leading dim (complex), rows 16B aligned
    static constexpr int RS = 2 * UP + 4;          // transpose scratch row stride (floats)
    static constexpr int SLOT = UP * LDc;          // complex elements per slot
};

// ---- 16-bit split operands -------------------------------------------------
template <int PREC>
struct Split;

template <>
struct Split<kF16> {
    typedef half8 V;
    static __device__ __forceinline__ void split(const float *x, V &hi, V &lo) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const _Float16 h = (_Float16)x[e];
            hi[e] = h;
            lo[e] = (_Float16)(x[e] - (float)h);
        }
    }
    // hi = f16(x sc), lo = f16(x sc - hi), each one fused multiply-add with
    // a single rounding to FP16 (x sc - hi is exact)
    static __device__ __forceinline__ void split_scaled(const float *x, float sc, V &hi, V &lo) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const _Float16 h = (_Float16)fmaf(x[e], sc, 0.f);
            hi[e] = h;
            lo[e] = (_Float16)fmaf(x[e], sc, -(float)h);
        }
    }
    static __device__ __forceinline__ floatx16 mfma(V a, V b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Split<kBF16> {
    typedef bf16x8 V;
    static __device__ __forceinline__ void split(const float *x, V &hi, V &lo) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const __bf16 h = (__bf16)x[e];
            hi[e] = h;
            lo[e] = (__bf16)(x[e] - (float)h);
        }
    }
    // BF16 has the FP32 exponent range: no scale is needed (sc = 1)
    static __device__ __forceinline__ void split_scaled(const float *x, float, V &hi, V &lo) { split(x, hi, lo); }
    static __device__ __forceinline__ floatx16 mfma(V a, V b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// a b ~= ah bh + ah bl + al bh
template <int PREC>
__device__ __forceinline__ floatx16 mfma3(typename Split<PREC>::V ah, typename Split<PREC>::V al,
                                          typename Split<PREC>::V bh, typename Split<PREC>::V bl, floatx16 c) {
    c = Split<PREC>::mfma(ah, bh, c);
    c = Split<PREC>::mfma(ah, bl, c);
    return Split<PREC>::mfma(al, bh, c);
}

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// ---- Gram ----------------------------------------------------------------------
// Channel rows in the Gram operand layout: the A and B operands of an MFMA
// step are the same register, lane (j, g) holding real column 32 ti + j of
//   FP32 (32x32x2, one step per row pair):  v[ti][s] = row 2 s + g;
//   16-bit (32x32x16, one step per 16 rows): v[ti][8 b + e] = row 16 b + 8 g + e.
template <int UP>
struct GramBuf {
    float v[Shape<UP>::NT][16];
};

// Loads rows [row0, row0 + nrows) (nrows <= 32) of one subcarrier's channel
// Hf (real row stride u2 = 2U) from global memory; columns >= u2 and rows
// >= nrows read as 0.  Lanes of one load instruction read two whole rows.
template <int UP, int PREC>
__device__ __forceinline__ void gram_load(const float *__restrict__ Hf, int u2, int row0, int nrows,
                                          GramBuf<UP> &b) {
    constexpr int NT = Shape<UP>::NT;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    const int rg = PREC == kF32 ? g : 8 * g;
    // loads only (see load_tile): rows past the tile read its last row,
    // columns past 2U read column 0; gram_mask zeroes both before use
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int rq = PREC == kF32 ? 2 * q : 16 * (q / 8) + (q % 8);
        const int rsel = rq + rg < nrows ? rq + rg : nrows - 1;
        const float *rowp = Hf + (size_t)(row0 + rsel) * u2;
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
            const int col = 32 * ti + j;
            b.v[ti][q] = rowp[col < u2 ? col : 0];
        }
    }
}

// Zeroes the rows >= nrows and columns >= u2 of a loaded Gram buffer.
template <int UP, int PREC>
__device__ __forceinline__ void gram_mask(GramBuf<UP> &b, int u2, int nrows) {
    constexpr int NT = Shape<UP>::NT;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    const int rg = PREC == kF32 ? g : 8 * g;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int rq = PREC == kF32 ? 2 * q : 16 * (q / 8) + (q % 8);
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
            b.v[ti][q] = (rq + rg < nrows && 32 * ti + j < u2) ? b.v[ti][q] : 0.f;
    }
}

// acc[t] += real Gram of the buffered rows, t over the tile pairs ti <= tj.
// 16-bit: the rows are scaled by a power of two 2^e into the FP16 range
// (BF16: e = 0), split hi + lo, and the tile's product is unscaled exactly
// into acc.  Returns e (0 for FP32), which also suits the same rows in the
// precode layout (their magnitudes are the same).
template <int UP, int PREC>
__device__ __forceinline__ int gram_mma(const GramBuf<UP> &b, floatx16 (&acc)[Shape<UP>::NTT]) {
    constexpr int NT = Shape<UP>::NT;
    constexpr int NTT = Shape<UP>::NTT;
    if constexpr (PREC == kF32) {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            int t = 0;
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = ti; tj < NT; ++tj) {
                    acc[t] = mfma32(b.v[ti][s], b.v[tj][s], acc[t]);
                    ++t;
                }
        }
        return 0;
    } else {
        typedef typename Split<PREC>::V V;
        int e2 = 0;
        if constexpr (PREC == kF16) {
            float m = 0.f;
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int q = 0; q < 16; ++q) m = fmaxf(m, fabsf(b.v[ti][q]));
            e2 = fp16_exp(wave_max(m));
        }
        const float sc = ldexpf(1.f, e2);
        floatx16 part[NTT];
#pragma unroll
        for (int t = 0; t < NTT; ++t) part[t] = floatx16{0};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            V hi[NT], lo[NT];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti) Split<PREC>::split_scaled(&b.v[ti][8 * s], sc, hi[ti], lo[ti]);
            int t = 0;
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = ti; tj < NT; ++tj) {
                    part[t] = mfma3<PREC>(hi[ti], lo[ti], hi[tj], lo[tj], part[t]);
                    ++t;
                }
        }
        const float un = ldexpf(1.f, -2 * e2);
#pragma unroll
        for (int t = 0; t < NTT; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[t][r] = fmaf(part[t][r], un, acc[t][r]);
        return e2;
    }
}

// 16-bit Gram of the buffered rows with a given exponent e: the products of
// the rows scaled by 2^e accumulate in acc directly (acc holds 2^(2e) times
// the Gram; the caller unscales once).  FP32: plain gram_mma.
template <int UP, int PREC>
__device__ __forceinline__ void gram_mma_scaled(const GramBuf<UP> &b, floatx16 (&acc)[Shape<UP>::NTT], int e) {
    if constexpr (PREC == kF32) {
        (void)gram_mma<UP, PREC>(b, acc);
    } else {
        constexpr int NT = Shape<UP>::NT;
        typedef typename Split<PREC>::V V;
        const float sc = ldexpf(1.f, e);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            V hi[NT], lo[NT];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti) Split<PREC>::split_scaled(&b.v[ti][8 * s], sc, hi[ti], lo[ti]);
            int t = 0;
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = ti; tj < NT; ++tj) {
                    acc[t] = mfma3<PREC>(hi[ti], lo[ti], hi[tj], lo[tj], acc[t]);
                    ++t;
                }
        }
    }
}

// Turns the real Gram tiles into the complex U x U matrix in an LDS slot:
// G[u][v] = post * ((M[2u][2v] + M[2u+1][2v+1]) + i (M[2u][2v+1] - M[2u+1][2v])),
// plus diag_add on the diagonal for u < m.  Output layout of the 32x32 MFMA:
// lane l, register r holds row 8(r/4) + 4(l/32) + r%4, column l%32.  The
// even-column lane of each pair combines its values with its partner's.
template <int UP>
__device__ __forceinline__ void gram_store(const floatx16 (&acc)[Shape<UP>::NTT], cx<float> *dst, float post,
                                           float diag_add, int m) {
    constexpr int NT = Shape<UP>::NT;
    constexpr int LDc = Shape<UP>::LDc;
    const int lane = lane_id();
    const int jj = lane & 31, g = lane >> 5;
    const bool even = (jj & 1) == 0;
    int t = 0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj) {
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
                const float own0 = acc[t][r], own1 = acc[t][r + 1];
                // partner lane l ^ 1 (DPP quad_perm [1,0,3,2])
                const float par0 = dpp_c<0xB1>(own0), par1 = dpp_c<0xB1>(own1);
                if (even) {
                    const int i = 8 * (r / 4) + 4 * g + (r % 4);
                    const int u = (32 * ti + i) >> 1, v = (32 * tj + jj) >> 1;
                    float gre = (own0 + par1) * post;
                    const float gim = (par0 - own1) * post;
                    if (u == v && u < m) gre += diag_add;
                    dst[u * LDc + v] = {gre, gim};
                    if (ti != tj) dst[v * LDc + u] = {gre, -gim};
                }
            }
            ++t;
        }
}

// ---- products X^T = Zbar^T Rows^T -----------------------------------------------
// Per-lane A operands for X^T = Zbar^T Rows^T, X^T rows i = 2k + q (symbol k,
// q = re/im), contraction kk = 2u + p over the real columns of Rows.  The
// contraction is permuted so that lane half g covers kk = g*UP .. g*UP+UP-1
// (contiguous columns of a row).  Zbar[2u+p][2k+q] is
// (p,q)=(0,0): Re z, (1,0): -Im z, (0,1): Im z, (1,1): Re z.
// Z(u, k) is read at Z[u*su + k*sk]; symbols k >= kvalid read as 0.
template <int UP>
__device__ __forceinline__ void load_zop(const cx<float> *Z, int su, int sk, int kvalid, float (&zop)[UP]) {
    const int lane = lane_id();
    const int i = lane & 31, g = lane >> 5;
    const int k = i >> 1, q = i & 1;
#pragma unroll
    for (int mm = 0; mm < UP; mm += 2) {
        const int u = (g * UP + mm) >> 1;
        cx<float> z = {0.f, 0.f};
        if (k < kvalid) z = Z[u * su + k * sk];
        zop[mm] = q ? z.im : z.re;
        zop[mm + 1] = q ? z.re : -z.im;
    }
}

// Z operand ready for the MFMA of precision PREC (scaled by 2^ez for 16-bit).
template <int UP, int PREC>
struct ZOp {
    float f[UP];
    typename Split<PREC == kF32 ? kF16 : PREC>::V hi[UP / 8], lo[UP / 8];
    float unscale;  // 2^-ez
};

// For 16-bit MFMA: scales the loaded operand by a power of two into the FP16
// range and splits it hi + lo (z.unscale undoes the scale).
template <int UP, int PREC>
__device__ __forceinline__ void zop_finish(ZOp<UP, PREC> &z) {
    z.unscale = 1.f;
    if constexpr (PREC != kF32) {
        float m = 0.f;
#pragma unroll
        for (int e = 0; e < UP; ++e) m = fmaxf(m, fabsf(z.f[e]));
        const int ez = fp16_exp(wave_max(m));
        const float sc = ldexpf(1.f, ez);
        z.unscale = ldexpf(1.f, -ez);
#pragma unroll
        for (int q = 0; q < UP / 8; ++q) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = z.f[8 * q + e] * sc;
            Split<PREC>::split(v, z.hi[q], z.lo[q]);
        }
    }
}

template <int UP, int PREC>
__device__ __forceinline__ void make_zop(const cx<float> *Z, int su, int sk, int kvalid, ZOp<UP, PREC> &z) {
    load_zop<UP>(Z, su, sk, kvalid, z.f);
    zop_finish<UP, PREC>(z);
}

// Symbols s(u, k) at sk0[k * kstride + u] as loaded for the symbol operand:
// lane (i, g) holds symbol k = i / 2, users (g UP + mm) / 2, mm even.  Loads
// only, from clamped in-range addresses (see load_tile); sym_to_zop masks.
template <int UP>
struct SymRaw {
    float2 v[UP / 2];
};

template <int UP>
__device__ __forceinline__ void load_sym(const float2 *__restrict__ sk0, size_t kstride, int U, int kvalid,
                                         SymRaw<UP> &r) {
    const int lane = lane_id();
    const int i = lane & 31, g = lane >> 5;
    const int k = i >> 1;
    const int kk = k < kvalid ? k : (kvalid > 0 ? kvalid - 1 : 0);
#pragma unroll
    for (int m = 0; m < UP / 2; ++m) {
        const int u = g * (UP / 2) + m;
        r.v[m] = sk0[(size_t)kk * kstride + (u < U ? u : U - 1)];
    }
}

// The symbol operand (zero for u >= U, k >= kvalid), split for 16-bit MFMA.
template <int UP, int PREC>
__device__ __forceinline__ void sym_to_zop(const SymRaw<UP> &r, int U, int kvalid, ZOp<UP, PREC> &z) {
    const int lane = lane_id();
    const int i = lane & 31, g = lane >> 5;
    const int k = i >> 1, q = i & 1;
#pragma unroll
    for (int m = 0; m < UP / 2; ++m) {
        const int u = g * (UP / 2) + m;
        const float2 v = (k < kvalid && u < U) ? r.v[m] : make_float2(0.f, 0.f);
        z.f[2 * m] = q ? v.y : v.x;
        z.f[2 * m + 1] = q ? v.x : -v.y;
    }
    zop_finish<UP, PREC>(z);
}

// X^T tile (32 x 32): rows (k, re/im) for a 16-symbol chunk, columns = rows
// 0..31 of `rows` (row-major floats, stride rs; rows >= nvalid read as 0),
// multiplied by `post`.  Lane l supplies B = Rows[l%32][g*UP + m].  For 16-bit
// operands the rows are scaled by sc before splitting and the result is also
// multiplied by the Z unscale.
template <int UP, int PREC>
__device__ __forceinline__ floatx16 mfma_apply(const float *rows, int rs, int nvalid, float sc, float post,
                                               const ZOp<UP, PREC> &z) {
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    float h[UP];
    const float *rp = rows + j * rs + g * UP;
    if (j < nvalid) {
#pragma unroll
        for (int m4 = 0; m4 < UP; m4 += 4) {
            const float4 v = *(const float4 *)(rp + m4);
            h[m4] = v.x;
            h[m4 + 1] = v.y;
            h[m4 + 2] = v.z;
            h[m4 + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int m = 0; m < UP; ++m) h[m] = 0.f;
    }
    floatx16 acc = {0};
    if constexpr (PREC == kF32) {
#pragma unroll
        for (int m = 0; m < UP; ++m) acc = mfma32(z.f[m], h[m], acc);
        acc *= post;
    } else {
#pragma unroll
        for (int q = 0; q < UP / 8; ++q) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = h[8 * q + e] * sc;
            typename Split<PREC>::V hh, hl;
            Split<PREC>::split(v, hh, hl);
            acc = mfma3<PREC>(z.hi[q], z.lo[q], hh, hl, acc);
        }
        acc *= post * z.unscale;
    }
    return acc;
}

// Symbol index held by register pair (r, r+1) of an X^T tile.
__device__ __forceinline__ int tile_k(int r, int g) { return 4 * (r / 4) + 2 * g + ((r % 4) >> 1); }

// ---- inversion ----------------------------------------------------------------
// Register layout of an UP x UP system: lane (r, c) = (lane / UP, lane % UP)
// holds column c of rows i = s*R + r (R = 64 / UP row groups, NS = UP / R
// slots).  For UP = 16 a row group is one DPP row of 16 lanes; for UP = 32 it
// is a half-wave (two DPP rows).  The broadcasts below move register data
// only (DPP and the gfx950 permlane swaps): no LDS round trip.

// Lane l receives v of lane 16 (l / 16) + k (DPP row_newbcast).
template <int k>
__device__ __forceinline__ float dpp_bcast16(float v) {
    return ffrom(__builtin_amdgcn_mov_dpp((int)fbits(v), 0x150 + k, 0xf, 0xf, true));
}

__device__ __forceinline__ float dpp_bcast16_dyn(float v, int k) {
    switch (k) {
        case 0: return dpp_bcast16<0>(v);
        case 1: return dpp_bcast16<1>(v);
        case 2: return dpp_bcast16<2>(v);
        case 3: return dpp_bcast16<3>(v);
        case 4: return dpp_bcast16<4>(v);
        case 5: return dpp_bcast16<5>(v);
        case 6: return dpp_bcast16<6>(v);
        case 7: return dpp_bcast16<7>(v);
        case 8: return dpp_bcast16<8>(v);
        case 9: return dpp_bcast16<9>(v);
        case 10: return dpp_bcast16<10>(v);
        case 11: return dpp_bcast16<11>(v);
        case 12: return dpp_bcast16<12>(v);
        case 13: return dpp_bcast16<13>(v);
        case 14: return dpp_bcast16<14>(v);
        default: return dpp_bcast16<15>(v);
    }
}

// Row r0 or r1 of each half-wave (swap16), or one half-wave (swap32), to all
// the lanes of its half-wave or of the wave.
__device__ __forceinline__ float even_rows16(float v, bool odd) {
    float a, b;
    swap16(v, a, b);
    return odd ? b : a;
}
__device__ __forceinline__ float half32(float v, bool hi) {
    float a, b;
    swap32(v, a, b);
    return hi ? b : a;
}

// Within each row group: lane (r, c) receives the value of lane (r, k).
// k is a constant after unrolling.
template <int UP>
__device__ __forceinline__ float bcast_col(float v, int k) {
    if constexpr (UP == 16) {
        return dpp_bcast16_dyn(v, k);
    } else {
        return even_rows16(dpp_bcast16_dyn(v, k & 15), k >= 16);
    }
}

// Across row groups: lane (r, c) receives the value of lane (rk, c).
template <int UP>
__device__ __forceinline__ float bcast_group(float v, int rk) {
    if constexpr (UP == 16) {
        return half32(even_rows16(v, rk & 1), rk >= 2);
    } else {
        return half32(v, rk != 0);
    }
}

// Across row groups through the LDS crossbar (ds_bpermute, no memory
// access): lane (r, c) receives the value of lane (rk, c).  Fewer VALU slots
// than bcast_group; its latency is hidden when issued ahead of use.
template <int UP>
__device__ __forceinline__ float bperm_group(float v, int c4, int rk) {
    return ffrom(__builtin_amdgcn_ds_bpermute(rk * UP * 4 + c4, (int)fbits(v)));
}

// The update of step k of the UP = 16 inversion for slots of the register
// layout, as v_fmac_f32_dpp with column k broadcast in the DPP operand
// (row_newbcast:k):  y += a_k(x) (-mim);  x += a_k(y) mim;  y += a_k(y) (-mre);
// x += a_k(x) (-mre), where a_k(v) is v's column-k value.  Each one reads
// column k before this step changes it (mult_k is real: the first two leave
// column k as it was).  The DPP read-after-VALU-write distances (2 wait
// states) are explicit: an s_nop opens each block, and the one-slot block
// spaces its dependent pairs with s_nop; the three-slot block interleaves the
// slots term by term so that each read is 2 or more instructions after its
// write.
#define GJ_FMAC(d, s, m) "v_fmac_f32_dpp " d ", " s ", " m " row_newbcast:%[k] row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
template <int K>
__device__ __forceinline__ void gj_upd1(float &x, float &y, float mim, float nmim, float nmre) {
    asm("s_nop 1\n\t" GJ_FMAC("%[y]", "%[x]", "%[nmim]") "s_nop 1\n\t" GJ_FMAC("%[x]", "%[y]", "%[mim]")
            GJ_FMAC("%[y]", "%[y]", "%[nmre]") "s_nop 0\n\t" GJ_FMAC("%[x]", "%[x]", "%[nmre]")
        : [x] "+v"(x), [y] "+v"(y)
        : [mim] "v"(mim), [nmim] "v"(nmim), [nmre] "v"(nmre), [k] "i"(K));
}
template <int K>
__device__ __forceinline__ void gj_upd3(float &x0, float &y0, float &x1, float &y1, float &x2, float &y2, float mim,
                                        float nmim, float nmre) {
    asm("s_nop 1\n\t" GJ_FMAC("%[y0]", "%[x0]", "%[nmim]") GJ_FMAC("%[y1]", "%[x1]", "%[nmim]")
            GJ_FMAC("%[y2]", "%[x2]", "%[nmim]") GJ_FMAC("%[x0]", "%[y0]", "%[mim]")
                GJ_FMAC("%[x1]", "%[y1]", "%[mim]") GJ_FMAC("%[x2]", "%[y2]", "%[mim]")
                    GJ_FMAC("%[y0]", "%[y0]", "%[nmre]") GJ_FMAC("%[y1]", "%[y1]", "%[nmre]")
                        GJ_FMAC("%[y2]", "%[y2]", "%[nmre]") GJ_FMAC("%[x0]", "%[x0]", "%[nmre]")
                            GJ_FMAC("%[x1]", "%[x1]", "%[nmre]") GJ_FMAC("%[x2]", "%[x2]", "%[nmre]")
        : [x0] "+v"(x0), [y0] "+v"(y0), [x1] "+v"(x1), [y1] "+v"(y1), [x2] "+v"(x2), [y2] "+v"(y2)
        : [mim] "v"(mim), [nmim] "v"(nmim), [nmre] "v"(nmre), [k] "i"(K));
}
#undef GJ_FMAC

#define GJ_DISPATCH(F, k, ...)                 \
    switch (k) {                               \
        case 0: F<0>(__VA_ARGS__); break;      \
        case 1: F<1>(__VA_ARGS__); break;      \
        case 2: F<2>(__VA_ARGS__); break;      \
        case 3: F<3>(__VA_ARGS__); break;      \
        case 4: F<4>(__VA_ARGS__); break;      \
        case 5: F<5>(__VA_ARGS__); break;      \
        case 6: F<6>(__VA_ARGS__); break;      \
        case 7: F<7>(__VA_ARGS__); break;      \
        case 8: F<8>(__VA_ARGS__); break;      \
        case 9: F<9>(__VA_ARGS__); break;      \
        case 10: F<10>(__VA_ARGS__); break;    \
        case 11: F<11>(__VA_ARGS__); break;    \
        case 12: F<12>(__VA_ARGS__); break;    \
        case 13: F<13>(__VA_ARGS__); break;    \
        case 14: F<14>(__VA_ARGS__); break;    \
        default: F<15>(__VA_ARGS__); break;    \
    }

// Power-of-two exponent e that brings the largest diagonal entry dmax of a
// Hermitian positive-definite A into [0.5, 1) (0 when dmax is not a positive
// finite number).  The inversions below run on 2^-e A: every pivot (a Schur
// complement, at most its diagonal entry) is then at most 1, so the update
// term 1 + 1/pivot keeps 1/pivot to full precision whatever the channel's
// scale (with a pivot of 3e6, 1 + 1/pivot in FP32 keeps only a third of
// 1/pivot's bits), and A^-1 = 2^-e (2^-e A)^-1 exactly.
__device__ __forceinline__ int diag_exp(float dmax) {
    if (!(dmax > 0.f) || !(dmax < INFINITY)) return 0;
    const int e = ilogbf(dmax) + 1;
    return e < -100 ? -100 : (e > 100 ? 100 : e);
}

// In-register inversion of the m x m Hermitian positive-definite system held
// in an LDS slot (full matrix), one wave, by Gauss-Jordan elimination without
// pivoting: step k divides row k by the pivot and eliminates column k from
// every other row, so that after m steps the slot holds A^-1.  For a Hermitian
// positive-definite A the pivots are the squared diagonal of its Cholesky
// factor and need no row exchanges.
// Per step and slot the update a_ic -= a_ik * mult_c is four fused
// multiply-adds with a DPP operand (gj_upd1 / gj_upd3).  Row k + 1 is fetched
// (bperm_group) as soon as its slot is updated, ahead of the other slots.
// Returns false when a pivot is not finite or not above kRelPivot32 times its
// original diagonal entry (numerically singular; a NaN pivot fails the test
// too).  On success writes A^-1 back to the slot and returns tr A^-1, ||A^-1||_F^2 and max |A^-1_ij|.
template <int UP>
__device__ bool wave_inverse(cx<float> *S, int m, float *tr_out, float *fro_out, float *max_out) {
    static_assert(UP == 16, "straight-line inversion: UP = 16 only");
    constexpr int R = 64 / UP;
    constexpr int NS = UP / R;
    constexpr int LDc = Shape<UP>::LDc;
    const int lane = lane_id();
    const int r = lane / UP, c = lane % UP, c4 = 4 * c;
    float re[NS], im[NS];
    // 2^-e A (diag_exp): lane c's diagonal entry, maximum over the columns
    const float dc = c < m ? S[c * LDc + c].re : 0.f;
    const int e = diag_exp(wave_max(dc));
    const float sc = ldexpf(1.f, -e);
    // rows and columns >= m are replaced by the identity, so that all UP
    // steps run unconditionally (straight-line code the scheduler can overlap
    // across steps) and leave the leading m x m block exactly as m steps would
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = s * R + r;
        const cx<float> v = S[i * LDc + c];
        const bool in = i < m && c < m;
        re[s] = in ? v.re * sc : (i == c ? 1.f : 0.f);
        im[s] = in ? v.im * sc : 0.f;
    }
    const float d0 = c < m ? dc * sc : 1.f;  // original (scaled) diagonal entry of column c
    float pv = 1.f;  // lane (r, c) keeps pivot c, checked against d0 after the last step
    // row 0, column c
    float akc_re = bperm_group<UP>(re[0], c4, 0);
    float akc_im = bperm_group<UP>(im[0], c4, 0);
#pragma unroll
    for (int k = 0; k < UP; ++k) {
        const int sk = k / R;  // slot of row k
        const int rk = k % R;  // row group of row k
        const float piv = bcast_col<UP>(akc_re, k);
        const bool iscol = c == k;
        pv = iscol ? piv : pv;
        const float inv = __builtin_amdgcn_rcpf(piv);
        // multiplier row: a_kc / a_kk for c != k and 1 + 1/a_kk for c = k,
        // so that one update a_ic - a_ik * mult_c also turns column k into
        // -a_ik / a_kk; row k itself becomes a_kc / a_kk (pivot 1/a_kk)
        const float mre = iscol ? 1.f + inv : akc_re * inv;
        const float mim = iscol ? 0.f : akc_im * inv;
        const float rowre = iscol ? inv : mre, rowim = mim;
        const float nmre = -mre, nmim = -mim;
        const int k1 = k + 1, s1 = k1 / R;
        auto row_select = [&](int s) {
            if (s == sk) {
                const bool isrow = r == rk;
                re[s] = isrow ? rowre : re[s];
                im[s] = isrow ? rowim : im[s];
            }
        };
        // slot a first (the one holding row k + 1, fetched right after it is
        // final), then the other three
        const int a = k1 < UP ? s1 : 0, b0 = a == 0 ? 1 : 0, b1 = a <= 1 ? 2 : 1, b2 = a <= 2 ? 3 : 2;
        GJ_DISPATCH(gj_upd1, k, re[a], im[a], mim, nmim, nmre);
        row_select(a);
        if (k1 < UP) {
            akc_re = bperm_group<UP>(re[a], c4, k1 % R);
            akc_im = bperm_group<UP>(im[a], c4, k1 % R);
        }
        GJ_DISPATCH(gj_upd3, k, re[b0], im[b0], re[b1], im[b1], re[b2], im[b2], mim, nmim, nmre);
        row_select(b0);
        row_select(b1);
        row_select(b2);
    }
    // every pivot finite and above kRelPivot32 times its original diagonal entry
    const bool ok = __all((pv > kRelPivot32 * d0) && (pv < INFINITY));
    float tr = 0.f, fro = 0.f, mx = 0.f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = s * R + r;
        const float vr = re[s] * sc, vi = im[s] * sc;  // A^-1 = 2^-e (2^-e A)^-1
        if (i < m && c < m) {
            fro += vr * vr + vi * vi;
            mx = fmaxf(mx, fmaxf(fabsf(vr), fabsf(vi)));
            if (i == c) tr += vr;
        }
        S[i * LDc + c] = {vr, vi};
    }
    *tr_out = wave_sum(tr);
    *fro_out = wave_sum(fro);
    *max_out = wave_max(mx);
    return ok;
}

// The same inversion for UP = 32 with one branch per step (a straight-line
// body of 32 steps over 16 slots takes the compiler far too long inside the
// larger kernels): row k reaches every lane through a bpermute, column k
// through bcast_col, the pivot through readlane.  Returns false when a pivot is not finite or not above kRelPivot32
// times the original diagonal entry (numerically singular).  On success writes
// A^-1 back to the slot and returns tr A^-1, ||A^-1||_F^2 and max |A^-1_ij|.
template <int UP>
__device__ bool wave_inverse_steps(cx<float> *S, int m, float *tr_out, float *fro_out, float *max_out) {
    constexpr int R = 64 / UP;
    constexpr int NS = UP / R;
    constexpr int LDc = Shape<UP>::LDc;
    const int lane = lane_id();
    const int r = lane / UP, c = lane % UP;
    float re[NS], im[NS];
    // 2^-e A (diag_exp)
    const float dc = S[c * LDc + c].re;
    const int e = diag_exp(wave_max(c < m ? dc : 0.f));
    const float sc = ldexpf(1.f, -e);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const cx<float> v = S[(s * R + r) * LDc + c];
        re[s] = v.re * sc;
        im[s] = v.im * sc;
    }
    const float d0 = dc * sc;  // original (scaled) diagonal entry of column c
    bool ok = true;
#pragma unroll
    for (int k = 0; k < UP; ++k) {
        if (k < m) {
            const int sk = k / R;  // slot of row k
            const int rk = k % R;  // row group of row k
            const float piv = readlane_f(re[sk], rk * UP + k);
            const float a0 = readlane_f(d0, k);
            ok = ok && (piv > kRelPivot32 * a0) && (piv < INFINITY);
            const float inv = __builtin_amdgcn_rcpf(piv);
            // row k, column c, before this step's update
            const float akc_re = __shfl(re[sk], rk * UP + c);
            const float akc_im = __shfl(im[sk], rk * UP + c);
            // multiplier row: a_kc / a_kk for c != k and 1 + 1/a_kk for c = k,
            // so that one update a_ic - a_ik * mult_c also turns column k into
            // -a_ik / a_kk; row k itself becomes a_kc / a_kk (pivot 1/a_kk)
            const bool iscol = c == k;
            const float mre = iscol ? 1.f + inv : akc_re * inv;
            const float mim = iscol ? 0.f : akc_im * inv;
            const float rowre = iscol ? inv : mre, rowim = mim;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const float aik_re = bcast_col<UP>(re[s], k);
                const float aik_im = bcast_col<UP>(im[s], k);
                const float nre = re[s] - (aik_re * mre - aik_im * mim);
                const float nim = im[s] - (aik_re * mim + aik_im * mre);
                if (s == sk) {
                    const bool isrow = r == rk;
                    re[s] = isrow ? rowre : nre;
                    im[s] = isrow ? rowim : nim;
                } else {
                    re[s] = nre;
                    im[s] = nim;
                }
            }
        }
    }
    float tr = 0.f, fro = 0.f, mx = 0.f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = s * R + r;
        const float vr = re[s] * sc, vi = im[s] * sc;  // A^-1 = 2^-e (2^-e A)^-1
        if (i < m && c < m) {
            fro += vr * vr + vi * vi;
            mx = fmaxf(mx, fmaxf(fabsf(vr), fabsf(vi)));
            if (i == c) tr += vr;
        }
        S[i * LDc + c] = {vr, vi};
    }
    *tr_out = wave_sum(tr);
    *fro_out = wave_sum(fro);
    *max_out = wave_max(mx);
    return ok;
}

// Factor one system held in slot A (A = G + kappa I, full Hermitian matrix):
// on success slot A holds A^-1, *t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1)
// and *amax = max |A^-1_ij|.
template <int UP>
__device__ bool wave_factor(cx<float> *sA, int m, float kap, float *t_out, float *amax) {
    float tr = 0.f, fro = 0.f;
    bool ok;
    if constexpr (UP == 16)
        ok = wave_inverse<UP>(sA, m, &tr, &fro, amax);
    else
        ok = wave_inverse_steps<UP>(sA, m, &tr, &fro, amax);
    const float t = tr - kap * fro;
    ok = ok && (t > 0.f) && (t < INFINITY);
    wave_sync();
    *t_out = t;
    return ok;
}

// Z(u, k) = scale * (A^-1 S)(u, k) for one chunk of symbols (operand zs)
// into slot B as [UP][KC]; a failed system (ok false) gets Z = 0.
template <int UP, int PREC>
__device__ void wave_solve_chunk(const cx<float> *sA, cx<float> *sB, const ZOp<UP, PREC> &zs, int kc, int m,
                                 float scale, float amax, bool ok) {
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    const int ea = PREC == kF32 ? 0 : fp16_exp(amax);
    const floatx16 a = mfma_apply<UP, PREC>((const float *)sA, 2 * Shape<UP>::LDc, m, ldexpf(1.f, ea),
                                            ldexpf(scale, -ea), zs);
    if (j < UP) {
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
            const int k = tile_k(r, g);
            if (k < KC) {
                cx<float> zz = {0.f, 0.f};
                if (ok && k < kc) zz = {a[r], a[r + 1]};
                sB[j * KC + k] = zz;
            }
        }
    }
}

// ---- channel tiles for the precode -------------------------------------------
// 32 channel rows in the B-operand layout of the precode MFMA: lane (j, g)
// holds row row0 + j, real columns g*UP .. g*UP + UP - 1 (users g*UP/2 ..
// g*UP/2 + UP/2 - 1).  For 16-bit MFMA the tile is split (hi + lo of the
// values scaled by a power of two into the FP16 range).
template <int UP, int PREC>
struct Tile {
    float f[UP];
    typename Split<PREC == kF32 ? kF16 : PREC>::V hi[UP / 8], lo[UP / 8];
    int e;  // packed tiles: hi + lo = f * 2^e
};

// 16-bit register tiles are split once, right after their Gram (with the
// exponent the Gram chose), and kept packed until the precode: the FP32
// values are dead from then on.
template <int UP, int PREC>
__device__ __forceinline__ void tile_pack(Tile<UP, PREC> &tl, int e) {
    if constexpr (PREC != kF32) {
        const float sc = ldexpf(1.f, e);
#pragma unroll
        for (int q = 0; q < UP / 8; ++q) Split<PREC>::split_scaled(&tl.f[8 * q], sc, tl.hi[q], tl.lo[q]);
        tl.e = e;
    }
}

// Loads rows [row0, row0 + nrows) (0 <= nrows <= 32; row0 a valid row) of a
// subcarrier's channel Hn (B x U) into a tile.  The loads go straight into
// the tile registers with nothing consuming them, so the loads of all of a
// wave's tiles stay in flight together (any instruction using a loaded value,
// or a branch around a load, makes the compiler wait for it there).  Lanes
// past nrows read the last row and users past U read user U - 1: the tile
// holds finite copies of real entries there, which the Gram masks out
// (tile_to_gram), the precode never stores, and the zero-padded symbol
// operand multiplies by zero.
// VEC (U == UP, 16-byte aligned channel): 16-byte loads at immediate offsets
// from one row address per tile; otherwise one 8-byte load per user.
template <int UP, int PREC, bool VEC>
__device__ __forceinline__ void load_tile(const float2 *__restrict__ Hn, int U, int row0, int nrows,
                                          Tile<UP, PREC> &tl) {
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    const int jr = j < nrows ? j : (nrows > 0 ? nrows - 1 : 0);
    if constexpr (VEC) {
        const float4 *rp = (const float4 *)(Hn + (size_t)(row0 + jr) * UP + g * (UP / 2));
#pragma unroll
        for (int m4 = 0; m4 < UP / 4; ++m4) {
            const float4 v = rp[m4];
            tl.f[4 * m4] = v.x;
            tl.f[4 * m4 + 1] = v.y;
            tl.f[4 * m4 + 2] = v.z;
            tl.f[4 * m4 + 3] = v.w;
        }
    } else {
        const float2 *rp = Hn + (size_t)(row0 + jr) * U;
#pragma unroll
        for (int m2 = 0; m2 < UP / 2; ++m2) {
            const int u = g * (UP / 2) + m2;
            const float2 v = rp[u < U ? u : U - 1];
            tl.f[2 * m2] = v.x;
            tl.f[2 * m2 + 1] = v.y;
        }
    }
}

// Register tiles with U == UP (VEC) load their rows in whole cache lines:
// instruction m, lane l reads the 16 bytes at m * 1 KiB + 16 l of the tile
// (rows m * RPI + l / LPR, float4 l % LPR of the row; LPR = UP / 2 lanes
// per row, RPI = 128 / UP rows per instruction), non-temporally (a register
// tile is a row's only read in a launch).  tile_to_gram stages this "raw"
// layout in LDS and reads back both the Gram operands and the precode
// layout; a row-per-lane load would touch 32 lines per instruction and
// fetch each line four times through the cache.
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int UP, int PREC>
__device__ __forceinline__ void load_tile_raw(const float2 *__restrict__ Hn, int row0, int nrows,
                                              Tile<UP, PREC> &tl) {
    constexpr int LPR = UP / 2, RPI = 128 / UP;
    const int lane = lane_id();
    const int lr = lane / LPR, c4 = lane % LPR;
#pragma unroll
    for (int m = 0; m < UP / 4; ++m) {
        const int row = m * RPI + lr;
        const int rr = row < nrows ? row : (nrows > 0 ? nrows - 1 : 0);
        const floatx4 v = __builtin_nontemporal_load((const floatx4 *)(Hn + (size_t)(row0 + rr) * UP) + c4);
        tl.f[4 * m] = v.x;
        tl.f[4 * m + 1] = v.y;
        tl.f[4 * m + 2] = v.z;
        tl.f[4 * m + 3] = v.w;
    }
}

// Exponent for packing a tile whose Gram is not formed (per-symbol mode):
// from the tile's own values (its copies of valid entries included).
template <int UP, int PREC>
__device__ __forceinline__ int tile_exp(const Tile<UP, PREC> &tl) {
    if constexpr (PREC == kF16) {
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < UP; ++q) m = fmaxf(m, fabsf(tl.f[q]));
        return fp16_exp(wave_max(m));
    } else {
        return 0;
    }
}

// X^T tile: rows (k, re/im) of a 16-symbol chunk, columns = the tile's 32
// rows.  16-bit: the tile is scaled into the FP16 range and split here and the
// product unscaled (with the Z unscale).
template <int UP, int PREC>
__device__ __forceinline__ floatx16 mfma_apply_tile(Tile<UP, PREC> &tl, const ZOp<UP, PREC> &z) {
    floatx16 acc = {0};
    if constexpr (PREC == kF32) {
#pragma unroll
        for (int m = 0; m < UP; ++m) acc = mfma32(z.f[m], tl.f[m], acc);
    } else {
        tile_pack<UP, PREC>(tl, tile_exp<UP, PREC>(tl));
#pragma unroll
        for (int q = 0; q < UP / 8; ++q) acc = mfma3<PREC>(z.hi[q], z.lo[q], tl.hi[q], tl.lo[q], acc);
        acc *= ldexpf(z.unscale, -tl.e);
    }
    return acc;
}

// The Gram of register tile tl (16-bit): FP16 scales each tile by the
// running exponent ea, the smallest per-tile exponent so far (the largest
// values so far), so that a tile's products start as soon as that tile has
// arrived; when a tile lowers ea, the products accumulated so far are
// rescaled exactly first (acc holds 2^(2 ea) times the Gram).  The tile keeps
// its own exponent (tl.e) for its precode split.  BF16 and FP32: no scale.
template <int UP, int PREC>
__device__ __forceinline__ void gram_tile(const GramBuf<UP> &b, Tile<UP, PREC> &tl,
                                          floatx16 (&acc)[Shape<UP>::NTT], int &ea, bool &have) {
    if constexpr (PREC == kF16) {
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < UP; ++q) m = fmaxf(m, fabsf(tl.f[q]));
        m = wave_max(m);
        const int eq = __builtin_amdgcn_readfirstlane(fp16_exp(m));
        tl.e = eq;
        // an all-zero tile (a silent cluster) sets no exponent: its products
        // are zero at any scale, and the next tiles keep their own range
        if (m > 0.f && (!have || eq < ea)) {
            if (have) {
                const float f = ldexpf(1.f, 2 * (eq - ea));
#pragma unroll
                for (int t2 = 0; t2 < Shape<UP>::NTT; ++t2) acc[t2] *= f;
            }
            ea = eq;
            have = true;
        }
    }
    gram_mma_scaled<UP, PREC>(b, acc, ea);
}

// X^T tile from a packed register tile (16-bit) or the FP32 tile.
template <int UP, int PREC>
__device__ __forceinline__ floatx16 mfma_apply_packed(const Tile<UP, PREC> &tl, const ZOp<UP, PREC> &z) {
    floatx16 acc = {0};
    if constexpr (PREC == kF32) {
#pragma unroll
        for (int m = 0; m < UP; ++m) acc = mfma32(z.f[m], tl.f[m], acc);
    } else {
#pragma unroll
        for (int q = 0; q < UP / 8; ++q) acc = mfma3<PREC>(z.hi[q], z.lo[q], tl.hi[q], tl.lo[q], acc);
        acc *= ldexpf(z.unscale, -tl.e);
    }
    return acc;
}

// The Gram operand buffer of a register tile, transposed through the wave's
// LDS scratch (rows stored row-major with stride RS, read back by column).
// Rows >= nrows and users >= U are zeroed here (the tile holds copies there).
template <int UP, int PREC, bool RAW = false>
__device__ __forceinline__ void tile_to_gram(Tile<UP, PREC> &tl, int nrows, int U, float *scr, GramBuf<UP> &b) {
    constexpr int NT = Shape<UP>::NT;
    constexpr int RS = Shape<UP>::RS;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    if constexpr (RAW) {
        // load_tile_raw's layout (U == UP); rows >= nrows are zeroed
        constexpr int LPR = UP / 2, RPI = 128 / UP;
        const int lr = lane / LPR, c4 = lane % LPR;
#pragma unroll
        for (int m = 0; m < UP / 4; ++m) {
            const int row = m * RPI + lr;
            const bool live = row < nrows;
            *(float4 *)(scr + row * RS + 4 * c4) =
                live ? make_float4(tl.f[4 * m], tl.f[4 * m + 1], tl.f[4 * m + 2], tl.f[4 * m + 3])
                     : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    } else {
        const bool live = j < nrows;
        float *rp = scr + j * RS + g * UP;
#pragma unroll
        for (int m4 = 0; m4 < UP; m4 += 4) {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (live && g * (UP / 2) + (m4 + e) / 2 < U) ? tl.f[m4 + e] : 0.f;
            *(float4 *)(rp + m4) = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int row = PREC == kF32 ? 2 * q + g : 16 * (q / 8) + 8 * g + (q % 8);
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) b.v[ti][q] = scr[row * RS + 32 * ti + j];
    }
    if constexpr (RAW) {
        // the precode layout: lane (j, g) holds row j, real columns g UP ..
        const float *rp = scr + j * RS + g * UP;
#pragma unroll
        for (int m4 = 0; m4 < UP; m4 += 4) {
            const float4 v = *(const float4 *)(rp + m4);
            tl.f[m4] = v.x;
            tl.f[m4 + 1] = v.y;
            tl.f[m4 + 2] = v.z;
            tl.f[m4 + 3] = v.w;
        }
    }
    wave_sync();  // the scratch is rewritten by the next tile
}

// A raw register tile (load_tile_raw) in the precode layout through the
// wave's LDS scratch, without a Gram (per-symbol mode); rows >= nrows zero.
template <int UP, int PREC>
__device__ __forceinline__ void tile_to_precode(Tile<UP, PREC> &tl, int nrows, float *scr) {
    constexpr int RS = Shape<UP>::RS;
    constexpr int LPR = UP / 2, RPI = 128 / UP;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    const int lr = lane / LPR, c4 = lane % LPR;
#pragma unroll
    for (int m = 0; m < UP / 4; ++m) {
        const int row = m * RPI + lr;
        *(float4 *)(scr + row * RS + 4 * c4) = row < nrows
                                                   ? make_float4(tl.f[4 * m], tl.f[4 * m + 1], tl.f[4 * m + 2], tl.f[4 * m + 3])
                                                   : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    wave_sync();
    const float *rp = scr + j * RS + g * UP;
#pragma unroll
    for (int m4 = 0; m4 < UP; m4 += 4) {
        const float4 v = *(const float4 *)(rp + m4);
        tl.f[m4] = v.x;
        tl.f[m4 + 1] = v.y;
        tl.f[m4 + 2] = v.z;
        tl.f[m4 + 3] = v.w;
    }
    wave_sync();
}

// Stores the X^T tile of rows [row0, row0 + nrows), symbols k0 .. k0 + kc - 1.
// Symbol k = tile_k(r, g) = kr + 2 g: a uniform symbol pointer per register
// pair and one lane offset.  The stores are non-temporal: nothing in the
// launch reads x back, and keeping it out of the caches leaves them to the
// channel and symbol reads (about 8% per frame at 256 antennas).
typedef float floatx2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void store_x(const floatx16 &a, int row0, int nrows, int k0, int kc, int n, int n_sc,
                                        int B, float2 *__restrict__ x) {
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    const size_t kstride = (size_t)n_sc * B;
    const size_t loff = 2 * g * kstride + j;
    if (j < nrows) {
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
            const int kr = tile_k(r, 0);
            float2 *xp = x + (size_t)(k0 + kr) * kstride + (size_t)n * B + row0;
            if (kr + 2 * g < kc) __builtin_nontemporal_store((floatx2){a[r], a[r + 1]}, (floatx2 *)(xp + loff));
        }
    }
}

// LDS per wave: the Z chunk (UP x KC complex) and one system slot (SLOT complex).
template <int UP>
struct Lds {
    static constexpr size_t zbytes = (size_t)UP * KC * 8;
    static constexpr size_t sbytes = (size_t)Shape<UP>::SLOT * 8;
    static constexpr size_t tbytes = (size_t)32 * Shape<UP>::RS * 4;
    // per wave: the Z chunk and the system slot, which the Gram's tile
    // transpose scratch overlays before either is written
    static constexpr size_t per_wave = zbytes + sbytes > tbytes ? zbytes + sbytes : tbytes;
    static __host__ __device__ constexpr size_t bytes(int nw) { return nw * per_wave; }
    // the split kernel's raw partial Gram accumulators also fit per wave
    static_assert(per_wave >= (size_t)Shape<UP>::NTT * 64 * 16 * 4, "raw Gram area");
    // and the FP64 retry of a failed system (f64r::instance, order U <= UP)
    static_assert(per_wave >= f64r::lds_bytes(UP), "FP64 retry area");
};

// Kernel modes: the whole frame, the per-frame part only (factors to
// global memory), or the per-symbol part from stored factors.
enum Mode { kFull = 0, kPrepare = 1, kSymbols = 2 };

// scale * A^-1 (m x m, from an LDS slot) to global memory, row-major m x m;
// scale = 0 (a failed instance) stores zeros.
template <int UP>
__device__ __forceinline__ void store_factor(const cx<float> *S, int m, float scale, cx<float> *__restrict__ g) {
    constexpr int LDc = Shape<UP>::LDc;
    for (int e = lane_id(); e < m * m; e += 64) {
        const int i = e / m, j = e - i * m;
        const cx<float> v = S[i * LDc + j];
        g[e] = scale != 0.f ? cx<float>{v.re * scale, v.im * scale} : cx<float>{0.f, 0.f};
    }
}

// A zero factor (an instance the FP64 route re-solves at every symbol pass).
__device__ __forceinline__ void zero_factor(int m, cx<float> *__restrict__ g) {
    for (int e = lane_id(); e < m * m; e += 64) g[e] = {0.f, 0.f};
}

// Whether the stored factors of instance sys were replaced by the FP64 route
// (prepare found the FP32 factorization failing and the FP64 one succeeding):
// the symbol pass then solves it in FP64 again.
__device__ __forceinline__ bool on_f64_route(const int *__restrict__ status, int sys) {
    return status && status[sys] == PRECODE_ST_FP64;
}

// Loads a stored factor into a zeroed-then-filled LDS slot; returns max |entry|.
template <int UP>
__device__ __forceinline__ float load_factor(const cx<float> *__restrict__ g, int m, cx<float> *S) {
    constexpr int LDc = Shape<UP>::LDc;
    constexpr int SLOT = Shape<UP>::SLOT;
    for (int e = lane_id(); e < SLOT; e += 64) S[e] = {0.f, 0.f};
    wave_sync();
    float mx = 0.f;
    for (int e = lane_id(); e < m * m; e += 64) {
        const int i = e / m, j = e - i * m;
        const cx<float> v = g[e];
        S[i * LDc + j] = v;
        mx = fmaxf(mx, fmaxf(fabsf(v.re), fabsf(v.im)));
    }
    wave_sync();
    return wave_max(mx);
}

// Tiles in flight when a wave streams its rows (MAXT = 0).
constexpr int kDepth = 4;

// Channel tiles a wave may keep in registers (MAXT; 0 streams the rows twice).
// (More than 4 tiles of 16 users would spill at the occupancy the launch
// needs; such systems stream.)
constexpr int max_tiles(int up) { return 4; }

// Minimum waves per SIMD the register allocation targets: more tiles held
// in registers need more registers per wave.  The split PD kernel with 4
// tiles per wave fits 3 (so that 2-wave workgroups of a 1200-subcarrier
// frame are all resident at once); the one-system-per-wave kernel with 4
// tiles needs the room of 2.
template <int UP, int MAXT, int PREC, bool SPLIT = false>
constexpr int min_waves() {
    if (UP == 16)
        return MAXT == 0 ? 2 : MAXT == 1 ? (PREC == kF32 ? 4 : 3) : MAXT == 2 ? 3 : (SPLIT ? 3 : 2);
    return MAXT == 1 ? 2 : 1;
}

// ---- one system per wave --------------------------------------------------------
// The whole chain of one local system, run by one wave with no workgroup
// barrier: PD system n = subcarrier n over all B rows; FD system n * C + c =
// cluster c of subcarrier n over its rows [o_c, o_{c+1}) (B_c >= U).
//   Gram      streams the rows in 32-row tiles (next tile's loads issued
//             before the current tile's MFMAs), A = G + kappa I into the slot
//   factor    A^-1 in registers (Gauss-Jordan), Lemma-1 t, scale
//             PD 1 / beta, beta = sqrt(Es / rho^2 t); FD w_c = sqrt(rho_c^2 / (t Es))
//   symbols   per chunk of 16: Z = scale A^-1 S (MFMA, S read from global
//             memory), then the rows are streamed again (from cache) for
//             X_c = H_c Z and stored
// Modes kPrepare / kSymbols store / load scale * A^-1 per system instead.
template <int UP, int PREC, int MAXT, bool VEC>
__device__ __forceinline__ void wave_system(const Prob &p, const Prob *__restrict__ pk, int sys, int K, int mode,
                                            const float2 *__restrict__ H, const float2 *__restrict__ s,
                                            float2 *__restrict__ x, cx<float> *__restrict__ ainv_g,
                                            float *__restrict__ scale_out, int *__restrict__ status, cx<float> *Zw,
                                            cx<float> *sA) {
    constexpr int SLOT = Shape<UP>::SLOT;
    constexpr int NTT = Shape<UP>::NTT;
    const int lane = lane_id();
    const bool pd = p.arch == kPD;
    const int B = p.B, U = p.U, C = p.C, n_sc = p.n_sc;
    const int n = pd ? sys : sys / C;
    const int c = pd ? 0 : sys - n * C;
    const int r0 = pd ? 0 : pk->off[c], r1 = pd ? B : pk->off[c + 1];
    const int ntile = (r1 - r0 + 31) >> 5;
    const float2 *Hn = H + (size_t)n * B * U;
    const float *Hf = (const float *)Hn;
    const float kap = pd ? pd_kappa(p) : fd_kappa_c(pk, c);
    cx<float> *fac = ainv_g ? ainv_g + (size_t)sys * U * U : nullptr;
    float scale = 1.f, amax = 0.f;
    bool ok = true;
    // MAXT > 0: the rows stay in registers from the first load to the
    // precode (loads of every tile issued up front; the Gram's column-layout
    // loads of the same lines are then served by the cache)
    Tile<UP, PREC> tiles[MAXT > 0 ? MAXT : 1];
    if constexpr (MAXT > 0) {
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int rq = r0 + 32 * q;
            // tiles past the system load (and zero) its first rows: no branch
            if constexpr (VEC)
                load_tile_raw<UP, PREC>(Hn, q < ntile ? rq : r0, q < ntile ? min(32, r1 - rq) : 0, tiles[q]);
            else
                load_tile<UP, PREC, VEC>(Hn, U, q < ntile ? rq : r0, q < ntile ? min(32, r1 - rq) : 0, tiles[q]);
        }
    }
    // the first chunk's symbols: loaded after the Gram, in flight during the
    // factorization (kept out of the Gram's register budget)
    SymRaw<UP> sym0;
    const bool pre_sym = mode != kPrepare && K > 0;
    // 16-bit register tiles: the Gram runs on a running exponent (gram_tile),
    // and the tiles are packed, each with its own exponent, at a single point
    // for every mode (packing in two branches keeps both forms of the tiles
    // live across the join)
    int ew = 0;
    bool have_e = false;
#pragma unroll
    for (int q = 0; q < (MAXT > 0 ? MAXT : 1); ++q) tiles[q].e = 0;
    floatx16 acc[NTT];
#pragma unroll
    for (int q = 0; q < NTT; ++q) acc[q] = floatx16{0};
    if (mode != kSymbols) {
        if constexpr (MAXT > 0) {
            // from the register tiles, transposed through LDS (the scratch
            // overlays Z and the slot, both unused until the Gram is done)
            float *scr = (float *)Zw;
#pragma unroll
            for (int q = 0; q < MAXT; ++q) {
                if (q < ntile) {
                    GramBuf<UP> b;
                    tile_to_gram<UP, PREC, VEC>(tiles[q], min(32, r1 - (r0 + 32 * q)), U, scr, b);
                    gram_tile<UP, PREC>(b, tiles[q], acc, ew, have_e);
                }
                // one tile at a time: keeps the scheduler from overlapping
                // several tiles' buffers on top of the resident tiles
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            // ring of kDepth tile buffers: the loads of the next kDepth - 1
            // tiles are in flight while a tile's MFMAs run (tile indices
            // past the end reload the last tile: no branch around a load)
            GramBuf<UP> ring[kDepth];
#pragma unroll
            for (int i = 0; i < kDepth - 1; ++i) {
                const int ti = min(i, ntile - 1), r = r0 + 32 * ti;
                gram_load<UP, PREC>(Hf, 2 * U, r, min(32, r1 - r), ring[i]);
            }
            // the loop body is one basic block (tiles past the end are
            // masked to zero, not skipped): the compiler then waits for each
            // tile's loads only, not for every load at the loop head
            for (int t = 0; t < ntile; t += kDepth) {
#pragma unroll
                for (int i = 0; i < kDepth; ++i) {
                    const int tl = min(t + i + kDepth - 1, ntile - 1), rl = r0 + 32 * tl;
                    gram_load<UP, PREC>(Hf, 2 * U, rl, min(32, r1 - rl), ring[(i + kDepth - 1) % kDepth]);
                    const int r = r0 + 32 * (t + i);
                    gram_mask<UP, PREC>(ring[i], 2 * U, t + i < ntile ? min(32, r1 - r) : 0);
                    gram_mma<UP, PREC>(ring[i], acc);
                }
            }
        }
    }
    if constexpr (MAXT > 0) {
        if (mode == kSymbols) {
#pragma unroll
            for (int q = 0; q < MAXT; ++q) {
                if constexpr (VEC) tile_to_precode<UP, PREC>(tiles[q], q < ntile ? min(32, r1 - (r0 + 32 * q)) : 0,
                                                             (float *)Zw);
                tiles[q].e = tile_exp<UP, PREC>(tiles[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < MAXT; ++q) tile_pack<UP, PREC>(tiles[q], tiles[q].e);
    }
    if (mode == kSymbols) {
        if (on_f64_route(status, sys)) {
            f64r::instance(f64r::shape_of(p), pk, sys, K, false, H, s, x, nullptr, nullptr, (char *)Zw);
            return;
        }
        if (pre_sym) load_sym<UP>(s + (size_t)n * U, (size_t)n_sc * U, U, min(KC, K), sym0);
        amax = load_factor<UP>(fac, U, sA);
    } else {
        if constexpr (MAXT > 0 && PREC != kF32) {
            const float un = ldexpf(1.f, -2 * ew);
#pragma unroll
            for (int t2 = 0; t2 < NTT; ++t2) acc[t2] *= un;
        }
        if (pre_sym) load_sym<UP>(s + (size_t)n * U, (size_t)n_sc * U, U, min(KC, K), sym0);
        for (int e = lane; e < SLOT; e += 64) sA[e] = {0.f, 0.f};
        wave_sync();
        gram_store<UP>(acc, sA, 1.f, kap, U);
        wave_sync();
        float tr = 0.f;
        ok = wave_factor<UP>(sA, U, kap, &tr, &amax);
        if (!ok) {
            // the FP32 factorization failed: the FP64 route solves the
            // instance (factors, status and every symbol) in this wave
            f64r::instance(f64r::shape_of(p), pk, sys, mode == kPrepare ? 0 : K, true, H, s, x, scale_out, status, (char *)Zw);
            if (mode == kPrepare) zero_factor(U, fac);
            return;
        }
        float out;
        if (pd) {
            out = sqrtf(p.Es / p.power * tr);  // beta
            scale = 1.f / out;
        } else {
            out = sqrtf(fd_power_c(pk, c) / (tr * p.Es));  // w_c
            scale = out;
        }
        if (lane == 0) {
            if (scale_out) scale_out[sys] = out;
            if (status) status[sys] = PRECODE_ST_OK;
        }
        if (mode == kPrepare) {
            store_factor<UP>(sA, U, scale, fac);
            return;
        }
    }
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kc = min(KC, K - k0);
        {
            SymRaw<UP> sym;
            if (k0 == 0) sym = sym0;
            else load_sym<UP>(s + ((size_t)k0 * n_sc + n) * U, (size_t)n_sc * U, U, kc, sym);
            // the solve is small: FP32 MFMA at every precision (exact
            // products, and no split operands next to the resident tiles)
            ZOp<UP, kF32> zs;
            sym_to_zop<UP, kF32>(sym, U, kc, zs);
            wave_solve_chunk<UP, kF32>(sA, Zw, zs, kc, U, scale, amax, ok);
        }
        wave_sync();
        ZOp<UP, PREC> z;
        make_zop<UP, PREC>(Zw, KC, 1, kc, z);
        if constexpr (MAXT > 0) {
#pragma unroll
            for (int q = 0; q < MAXT; ++q) {
                const int rq = r0 + 32 * q;
                if (q < ntile)
                    store_x(mfma_apply_packed<UP, PREC>(tiles[q], z), rq, min(32, r1 - rq), k0, kc, n, n_sc, B, x);
                __builtin_amdgcn_sched_barrier(0);
            }
            wave_sync();
            continue;
        }
        // the rows streamed again through a ring of kDepth tiles
        Tile<UP, PREC> ring[kDepth];
#pragma unroll
        for (int i = 0; i < kDepth - 1; ++i) {
            const int ti = min(i, ntile - 1), r = r0 + 32 * ti;
            load_tile<UP, PREC, VEC>(Hn, U, r, min(32, r1 - r), ring[i]);
        }
        for (int t = 0; t < ntile; t += kDepth) {
#pragma unroll
            for (int i = 0; i < kDepth; ++i) {
                const int tl = min(t + i + kDepth - 1, ntile - 1), rl = r0 + 32 * tl;
                load_tile<UP, PREC, VEC>(Hn, U, rl, min(32, r1 - rl), ring[(i + kDepth - 1) % kDepth]);
                // no branch around the product (see the Gram ring); a tile
                // past the end stores no rows
                const int r = r0 + 32 * (t + i);
                store_x(mfma_apply_tile<UP, PREC>(ring[i], z), r, t + i < ntile ? min(32, r1 - r) : 0, k0, kc, n,
                        n_sc, B, x);
            }
        }
        wave_sync();  // Zw is rewritten by the next chunk
    }
}

// ---- one PD subcarrier per workgroup (split over the rows) ----------------------
// For PD systems too large for one wave's registers: the NW waves of a
// workgroup share subcarrier blk.  Wave w keeps the channel tiles t = w,
// w + NW, ... (MAXT of them) in registers from the first load to the
// precode (all loads issued up front), forms their partial Gram (the split
// rows are the cluster sum of the adder tree in another order), and all
// partials are summed in LDS in fixed wave order.  One master wave, rotating
// with the block index so co-resident workgroups use different SIMDs,
// factors and solves; every wave then precodes its own rows.
template <int UP, int PREC, int NW, int MAXT, bool VEC>
__device__ __forceinline__ void wg_pd_split(const Prob &p, int blk, int K, int mode, const float2 *__restrict__ H,
                                            const float2 *__restrict__ s, float2 *__restrict__ x,
                                            cx<float> *__restrict__ ainv_g, float *__restrict__ scale_out,
                                            int *__restrict__ status, char *lds) {
    constexpr int NTT = Shape<UP>::NTT;
    __shared__ float sh_scale, sh_amax;
    __shared__ int sh_ok;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int mw = blk % NW;
    const int B = p.B, U = p.U, n_sc = p.n_sc, n = blk;
    const int ntile = (B + 31) >> 5;
    const float2 *Hn = H + (size_t)n * B * U;
    auto zw_of = [&](int w) { return (cx<float> *)(lds + (size_t)w * Lds<UP>::per_wave); };
    auto slot_of = [&](int w) { return (cx<float> *)(lds + (size_t)w * Lds<UP>::per_wave + Lds<UP>::zbytes); };
    auto raw_of = [&](int w) { return (float *)(lds + (size_t)w * Lds<UP>::per_wave); };
    cx<float> *Zm = zw_of(mw), *Am = slot_of(mw);
    cx<float> *fac = ainv_g ? ainv_g + (size_t)n * U * U : nullptr;

    Tile<UP, PREC> tiles[MAXT];
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const int tt = wave + NW * q;
        const bool v = tt < ntile;
        if constexpr (VEC)
            load_tile_raw<UP, PREC>(Hn, v ? 32 * tt : 0, v ? min(32, B - 32 * tt) : 0, tiles[q]);
        else
            load_tile<UP, PREC, VEC>(Hn, U, v ? 32 * tt : 0, v ? min(32, B - 32 * tt) : 0, tiles[q]);
    }
    const float kap = pd_kappa(p);
    // the first chunk's symbols, loaded by the master while it factors
    SymRaw<UP> sym0;
    const bool pre_sym = mode != kPrepare && K > 0;
    const float2 *s0 = s + (size_t)n * U;
    // the master's subcarrier goes to the FP64 route (the FP32
    // factorization failed, or prepare found it so)
    bool retry = false;
    // 16-bit: the Gram runs on a running exponent (gram_tile); the tiles are
    // packed, each with its own exponent, at a single point for every mode
    // (packing in two branches keeps both forms of the tiles live across the
    // join)
    int ew = 0;
    bool have_e = false;
#pragma unroll
    for (int q = 0; q < MAXT; ++q) tiles[q].e = 0;
    floatx16 acc[NTT];
#pragma unroll
    for (int q = 0; q < NTT; ++q) acc[q] = floatx16{0};
    if (mode != kSymbols) {
        float *scr = (float *)zw_of(wave);
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int tt = wave + NW * q;
            if (tt < ntile) {
                GramBuf<UP> b;
                tile_to_gram<UP, PREC, VEC>(tiles[q], min(32, B - 32 * tt), U, scr, b);
                gram_tile<UP, PREC>(b, tiles[q], acc, ew, have_e);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        float *scr = (float *)zw_of(wave);
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int tt = wave + NW * q;
            if constexpr (VEC) tile_to_precode<UP, PREC>(tiles[q], tt < ntile ? min(32, B - 32 * tt) : 0, scr);
            tiles[q].e = tile_exp<UP, PREC>(tiles[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < MAXT; ++q) tile_pack<UP, PREC>(tiles[q], tiles[q].e);
    if (mode == kSymbols) {
        if (wave == mw) {
            // an instance prepare moved to the FP64 route (its stored factor
            // is zero) is solved again on that route at the end; the factor
            // is loaded after the tiles' transposes, which overlay the slot
            retry = on_f64_route(status, n);
            if (pre_sym) load_sym<UP>(s0, (size_t)n_sc * U, U, min(KC, K), sym0);
            const float amax = load_factor<UP>(fac, U, Am);
            if (lane == 0) {
                sh_scale = 1.f;
                sh_amax = amax;
                sh_ok = !retry;
            }
        }
    }
    if (mode != kSymbols) {
        if constexpr (PREC != kF32) {
            const float un = ldexpf(1.f, -2 * ew);
#pragma unroll
            for (int t2 = 0; t2 < NTT; ++t2) acc[t2] *= un;
        }
        // every wave's partial accumulators, raw, to its LDS area; the master
        // adds them in fixed wave order and stores G + kappa I into its slot
        wave_sync();
#pragma unroll
        for (int q = 0; q < NTT; ++q)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4)
                *(float4 *)(raw_of(wave) + ((q * 4 + r4) * 64 + lane) * 4) =
                    make_float4(acc[q][4 * r4], acc[q][4 * r4 + 1], acc[q][4 * r4 + 2], acc[q][4 * r4 + 3]);
        __syncthreads();
        if (wave == mw) {
            // the master's partial sums, inversion and solve are the serial
            // chain every wave of the workgroup waits on: it issues ahead of
            // co-resident waves until the first chunk is solved
            __builtin_amdgcn_s_setprio(3);
            if (pre_sym) load_sym<UP>(s0, (size_t)n_sc * U, U, min(KC, K), sym0);
            floatx16 sum[NTT];
#pragma unroll
            for (int w = 0; w < NW; ++w)
#pragma unroll
                for (int q = 0; q < NTT; ++q)
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4) {
                        const float4 v = *(const float4 *)(raw_of(w) + ((q * 4 + r4) * 64 + lane) * 4);
                        if (w == 0) {
                            sum[q][4 * r4] = v.x, sum[q][4 * r4 + 1] = v.y;
                            sum[q][4 * r4 + 2] = v.z, sum[q][4 * r4 + 3] = v.w;
                        } else {
                            sum[q][4 * r4] += v.x, sum[q][4 * r4 + 1] += v.y;
                            sum[q][4 * r4 + 2] += v.z, sum[q][4 * r4 + 3] += v.w;
                        }
                    }
            // the master's slot overlays raw areas: all reads above are done
            wave_sync();
            gram_store<UP>(sum, Am, 1.f, kap, U);
            wave_sync();
            float tr = 0.f, amax = 0.f;
            const bool ok = wave_factor<UP>(Am, U, kap, &tr, &amax);
            if (ok) {
                const float beta = sqrtf(p.Es / p.power * tr);
                if (lane == 0) {
                    sh_scale = 1.f / beta;
                    sh_amax = amax;
                    sh_ok = 1;
                    if (scale_out) scale_out[n] = beta;
                    if (status) status[n] = PRECODE_ST_OK;
                }
                if (mode == kPrepare) store_factor<UP>(Am, U, 1.f / beta, fac);
            } else {
                if (lane == 0) {
                    sh_scale = 0.f;
                    sh_amax = amax;
                    sh_ok = 0;
                }
                retry = true;
                if (mode == kPrepare) {
                    // the FP32 factorization failed: the FP64 route's factors
                    // and status; its symbols are solved at every symbol pass
                    __builtin_amdgcn_s_setprio(0);
                    f64r::instance(f64r::shape_of(p), nullptr, n, 0, true, H, s, x, scale_out, status,
                                   (char *)raw_of(mw));
                    zero_factor(U, fac);
                }
            }
        }
        if (mode == kPrepare) return;
    }
    __syncthreads();
    // a failed subcarrier's chunks are solved to zero (scale 0) and stored;
    // the master then overwrites them from the FP64 route at the end, once no
    // channel tile is live (the last barrier of the loop orders the stores)
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kc = min(KC, K - k0);
        if (wave == mw) {
            ZOp<UP, kF32> zs;  // FP32 solve at every precision (see wave_system)
            if (k0 == 0) {
                sym_to_zop<UP, kF32>(sym0, U, kc, zs);
            } else {
                SymRaw<UP> sym;
                load_sym<UP>(s + ((size_t)k0 * n_sc + n) * U, (size_t)n_sc * U, U, kc, sym);
                sym_to_zop<UP, kF32>(sym, U, kc, zs);
            }
            wave_solve_chunk<UP, kF32>(Am, Zm, zs, kc, U, sh_scale, sh_amax, sh_ok != 0);
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        ZOp<UP, PREC> z;
        make_zop<UP, PREC>(Zm, KC, 1, kc, z);
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int tt = wave + NW * q;
            if (tt < ntile)
                store_x(mfma_apply_packed<UP, PREC>(tiles[q], z), 32 * tt, min(32, B - 32 * tt), k0, kc, n, n_sc, B,
                        x);
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();  // Zm is rewritten by the next chunk
    }
    if (retry) {
        __builtin_amdgcn_s_setprio(0);
        f64r::instance(f64r::shape_of(p), nullptr, n, K, mode != kSymbols, H, s, x, scale_out, status,
                       (char *)raw_of(mw));
    }
}

// ---- the kernel body -----------------------------------------------------------
// Workgroups of NW waves; wave w of block blk runs system blk * NW + w (PD:
// consecutive subcarriers; FD: consecutive clusters of a subcarrier).
// pk: the problem (p) in memory the kernel can index (cluster offsets and
// per-cluster regularizers / budgets).
// MAXT: channel tiles (32 rows) of the largest system that a wave keeps in
// registers (0: the precode streams the rows a second time).  VEC: U == UP
// and a 16-byte aligned channel (wider loads).
// SPLIT (PD only): one subcarrier per workgroup, MAXT tiles per wave
// (wg_pd_split); otherwise one system per wave.
template <int UP, int PREC, int NW, int MAXT, bool VEC, bool SPLIT>
__device__ __forceinline__ void fused_body(const Prob &p, const Prob *__restrict__ pk, int blk, int K, int mode,
                                           const float2 *__restrict__ H,
                                           const float2 *__restrict__ s, float2 *__restrict__ x,
                                           cx<float> *__restrict__ ainv_g, float *__restrict__ scale_out,
                                           int *__restrict__ status) {
    extern __shared__ float4 smem4[];
    if constexpr (SPLIT) {
        wg_pd_split<UP, PREC, NW, MAXT, VEC>(p, blk, K, mode, H, s, x, ainv_g, scale_out, status, (char *)smem4);
        return;
    }
    // the wave index is uniform: keep it (and the system's indices and base
    // addresses) in scalar registers, so that the cluster offsets are scalar
    // loads and no vector load has to be waited for before the channel loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_sys = p.arch == kPD ? p.n_sc : p.n_sc * p.C;
    const int sys = blk * NW + wave;
    if (sys >= n_sys) return;
    char *wb = (char *)smem4 + (size_t)wave * Lds<UP>::per_wave;
    wave_system<UP, PREC, MAXT, VEC>(p, pk, sys, K, mode, H, s, x, ainv_g, scale_out, status, (cx<float> *)wb,
                                (cx<float> *)(wb + Lds<UP>::zbytes));
}

int pick_up(int U) { return U <= 16 ? 16 : (U <= 32 ? 32 : 0); }

int prec_of(int precision) {
    switch (precision) {
        case PRECODE_PREC_FP32: return kF32;
        case PRECODE_PREC_SPLIT_FP16: return kF16;
        case PRECODE_PREC_SPLIT_BF16: return kBF16;
        default: return -1;
    }
}

// Workgroups of nw waves a problem's launch needs (split: one per subcarrier).
int blocks_for(const Prob &p, int nw, bool split = false) {
    if (split) return p.n_sc;
    const long long ns = p.arch == kPD ? (long long)p.n_sc : (long long)p.n_sc * p.C;
    return (int)((ns + nw - 1) / nw);
}

constexpr size_t kLdsMax = 160 * 1024;
constexpr size_t kLdsUsable = kLdsMax - 256;

// Tiles (32 rows) of the largest local system of a problem.
int system_tiles(const Prob &p) {
    int r = p.arch == kPD ? p.B : 0;
    if (p.arch == kFD)
        for (int c = 0; c < p.C; ++c) r = p.off[c + 1] - p.off[c] > r ? p.off[c + 1] - p.off[c] : r;
    return (r + 31) >> 5;
}

// Whether the 16-byte tile loads apply (U == UP, 16-byte aligned channel).
bool pick_vec(const Prob &p, const void *H) { return p.U == pick_up(p.U) && (((uintptr_t)H) & 15) == 0; }

// Split launch for a PD problem whose rows do not fit one wave's registers:
// tiles per wave with nw waves per subcarrier, or 0 if they do not fit either.
int pick_split_maxt(const Prob &p, int nw) {
    if (p.arch != kPD) return 0;
    const int t = (system_tiles(p) + nw - 1) / nw, lim = max_tiles(pick_up(p.U));
    int m = 1;
    while (m < t) m <<= 1;
    return m <= lim ? m : 0;
}

// Register tiles per wave for a problem: the next power of two of its
// largest system's tiles, or 0 (stream) past max_tiles.
int pick_maxt(const Prob &p) {
    const int t = system_tiles(p), lim = max_tiles(pick_up(p.U));
    int m = 1;
    while (m < t) m <<= 1;
    return m <= lim ? m : 0;
}

}  // namespace
}  // namespace pc
