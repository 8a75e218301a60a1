// fused_kernel.h -- device code of the fused PD / FD kernel (one problem per
// workgroup set), shared by the single-problem launches (fused.hip) and the
// heterogeneous batch launches (batch.hip).  Internal to the library.
#pragma once
#include <stddef.h>

#include "common.h"

namespace pc {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int KC = 16;  // symbols per MFMA chunk: 2*KC = 32 rows of X^T
constexpr int kMaxKFused = 64;

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

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Power-of-two exponent e with m * 2^e in [2^13, 2^14) (0 for m = 0): the
// scale that brings operands of magnitude <= m into the FP16 range while
// keeping their low parts away from subnormals.
__device__ __forceinline__ int fp16_exp(float m) { return m > 0.f ? 13 - ilogbf(m) : 0; }

template <int UP>
struct Shape {
    static constexpr int NT = (2 * UP) / 32;       // 32-wide real column tiles
    static constexpr int NTT = NT * (NT + 1) / 2;  // tiles with ti <= tj
    static constexpr int RS = 2 * UP + 4;          // H row stride in LDS (floats)
    static constexpr int LDc = UP + 2;             // slot leading dim (complex), rows 16B aligned
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
// Real Gram of `nrows` rows (row-major floats, stride rs), values scaled by sc:
// acc[t] += M[32ti+i][32tj+j] = sum_r R[r][32ti+i] R[r][32tj+j], ti <= tj.
// 32x32 MFMA operands: lane l supplies A[l%32][k] and B[k][l%32] for its
// contraction slots k; here both are R[row(k)][col], so a lane reads only the
// column l%32 of its rows (two rows per FP32 instruction, 8 per lane half per
// 16-bit instruction).
template <int UP, int PREC>
__device__ __forceinline__ void mfma_gram(const float *rows, int rs, int nrows, float sc,
                                          floatx16 (&acc)[Shape<UP>::NTT]) {
    constexpr int NT = Shape<UP>::NT;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    if constexpr (PREC == kF32) {
        // groups of G instructions (2 rows each); the LDS reads of the next
        // group are issued before the MFMAs of the current one
        constexpr int G = 4;
        float cur[G][NT], nxt[G][NT];
        auto load = [&](float (&v)[G][NT], int r) {
#pragma unroll
            for (int a = 0; a < G; ++a) {
                const int row = r + 2 * a + g;
#pragma unroll
                for (int ti = 0; ti < NT; ++ti) v[a][ti] = row < nrows ? rows[row * rs + 32 * ti + j] : 0.f;
            }
        };
        load(nxt, 0);
#pragma unroll 1
        for (int r = 0; r < nrows; r += 2 * G) {
#pragma unroll
            for (int a = 0; a < G; ++a)
#pragma unroll
                for (int ti = 0; ti < NT; ++ti) cur[a][ti] = nxt[a][ti];
            if (r + 2 * G < nrows) load(nxt, r + 2 * G);
#pragma unroll
            for (int a = 0; a < G; ++a) {
                int t = 0;
#pragma unroll
                for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                    for (int tj = ti; tj < NT; ++tj) {
                        acc[t] = mfma32(cur[a][ti], cur[a][tj], acc[t]);
                        ++t;
                    }
            }
        }
    } else {
        typedef typename Split<PREC>::V V;
        // 16 rows per step; the LDS reads of the next step are issued before
        // the split and MFMAs of the current one
        float cur[NT][8], nxt[NT][8];
        auto load = [&](float (&v)[NT][8], int r) {
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int row = r + 8 * g + e;
                    v[ti][e] = row < nrows ? rows[row * rs + 32 * ti + j] : 0.f;
                }
        };
        load(nxt, 0);
#pragma unroll 1
        for (int r = 0; r < nrows; r += 16) {
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int e = 0; e < 8; ++e) cur[ti][e] = nxt[ti][e] * sc;
            if (r + 16 < nrows) load(nxt, r + 16);
            V hi[NT], lo[NT];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti) Split<PREC>::split(cur[ti], hi[ti], lo[ti]);
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
                const float par0 = __shfl_xor(own0, 1), par1 = __shfl_xor(own1, 1);
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

template <int UP, int PREC>
__device__ __forceinline__ void make_zop(const cx<float> *Z, int su, int sk, int kvalid, ZOp<UP, PREC> &z) {
    load_zop<UP>(Z, su, sk, kvalid, z.f);
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
// Broadcast within the lanes of one matrix row of the register layout below:
// lane (r, c) receives the value of lane (r, k).  For UP = 16 a row is a DPP
// row of 16 lanes (row_newbcast); for UP = 32 it is a half-wave.
template <int UP, int k>
__device__ __forceinline__ float bcast_row(float v) {
    if constexpr (UP == 16) {
        return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + k, 0xf,
                                                                      0xf, false));
    } else {
        return __shfl(v, (lane_id() & ~(UP - 1)) | k);
    }
}

template <int UP>
__device__ __forceinline__ float bcast_row_dyn(float v, int k) {
    if constexpr (UP == 16) {
        switch (k) {
            case 0: return bcast_row<16, 0>(v);
            case 1: return bcast_row<16, 1>(v);
            case 2: return bcast_row<16, 2>(v);
            case 3: return bcast_row<16, 3>(v);
            case 4: return bcast_row<16, 4>(v);
            case 5: return bcast_row<16, 5>(v);
            case 6: return bcast_row<16, 6>(v);
            case 7: return bcast_row<16, 7>(v);
            case 8: return bcast_row<16, 8>(v);
            case 9: return bcast_row<16, 9>(v);
            case 10: return bcast_row<16, 10>(v);
            case 11: return bcast_row<16, 11>(v);
            case 12: return bcast_row<16, 12>(v);
            case 13: return bcast_row<16, 13>(v);
            case 14: return bcast_row<16, 14>(v);
            default: return bcast_row<16, 15>(v);
        }
    } else {
        return __shfl(v, (lane_id() & ~(UP - 1)) | k);
    }
}

// In-register inversion of the m x m Hermitian positive-definite system held
// in an LDS slot (full matrix), one wave, by Gauss-Jordan elimination without
// pivoting: step k divides row k by the pivot and eliminates column k from
// every other row, so that after m steps the slot holds A^-1.  For a Hermitian
// positive-definite A the pivots are the squared diagonal of its Cholesky
// factor and need no row exchanges.
// Layout: lane (r, c) = (lane / UP, lane % UP) holds column c, rows
// i = s*R + r (R = 64 / UP row groups, NS = UP / R slots).  Row k reaches every
// lane through a bpermute, column k through bcast_row, the pivot through
// readlane.  Returns false when a pivot is not finite or not above kRelPivot32
// times the original diagonal entry (numerically singular).  On success writes
// A^-1 back to the slot and returns tr A^-1, ||A^-1||_F^2 and max |A^-1_ij|.
template <int UP>
__device__ bool wave_inverse(cx<float> *S, int m, float *tr_out, float *fro_out, float *max_out) {
    constexpr int R = 64 / UP;
    constexpr int NS = UP / R;
    constexpr int LDc = Shape<UP>::LDc;
    const int lane = lane_id();
    const int r = lane / UP, c = lane % UP;
    float re[NS], im[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const cx<float> v = S[(s * R + r) * LDc + c];
        re[s] = v.re;
        im[s] = v.im;
    }
    const float d0 = S[c * LDc + c].re;  // original diagonal entry of column c
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
                const float aik_re = bcast_row_dyn<UP>(re[s], k);
                const float aik_im = bcast_row_dyn<UP>(im[s], k);
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
        if (i < m && c < m) {
            fro += re[s] * re[s] + im[s] * im[s];
            mx = fmaxf(mx, fmaxf(fabsf(re[s]), fabsf(im[s])));
            if (i == c) tr += re[s];
        }
        S[i * LDc + c] = {re[s], im[s]};
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
    bool ok = wave_inverse<UP>(sA, m, &tr, &fro, amax);
    const float t = tr - kap * fro;
    ok = ok && (t > 0.f) && (t < INFINITY);
    wave_sync();
    *t_out = t;
    return ok;
}

// Z(u, k) = scale * (A^-1 S)(u, k) for one chunk into slot B as [UP][KC].
template <int UP, int PREC>
__device__ void wave_solve_chunk(const cx<float> *sA, cx<float> *sB, const float *Ss, int k0, int kc, int m,
                                 float scale, float amax, bool ok) {
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    ZOp<UP, PREC> z;
    make_zop<UP, PREC>((const cx<float> *)Ss + k0 * UP, 1, UP, kc, z);
    const int ea = PREC == kF32 ? 0 : fp16_exp(amax);
    const floatx16 a = mfma_apply<UP, PREC>((const float *)sA, 2 * Shape<UP>::LDc, m, ldexpf(1.f, ea),
                                            ldexpf(scale, -ea), z);
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

// ---- channel tiles in registers -----------------------------------------------
// A wave keeps the channel rows it precodes in registers, 32 rows per tile, in
// the B-operand layout of the precode MFMA: lane (j, g) holds row row0 + j,
// real columns g*UP .. g*UP + UP - 1 (users g*UP/2 .. g*UP/2 + UP/2 - 1).
// For 16-bit MFMA the tile is kept split (hi + lo of the scaled values).
template <int UP, int PREC>
struct Tile {
    float f[UP];
    typename Split<PREC == kF32 ? kF16 : PREC>::V hi[UP / 8], lo[UP / 8];
};

// Loads rows [row0, row0 + nrows) of a subcarrier's channel Hn (B x U) into a
// tile (rows >= nrows and users >= U read as 0); returns the lane's max |h|.
template <int UP, int PREC>
__device__ __forceinline__ float load_tile(const float2 *__restrict__ Hn, int U, int row0, int nrows, bool vec,
                                           Tile<UP, PREC> &tl) {
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    float mx = 0.f;
    if (j < nrows) {
        const float2 *rp = Hn + (size_t)(row0 + j) * U + g * (UP / 2);
        if (vec) {  // U == UP, 16-byte aligned rows
#pragma unroll
            for (int m4 = 0; m4 < UP; m4 += 4) {
                const float4 v = *(const float4 *)(rp + m4 / 2);
                tl.f[m4] = v.x;
                tl.f[m4 + 1] = v.y;
                tl.f[m4 + 2] = v.z;
                tl.f[m4 + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int m2 = 0; m2 < UP / 2; ++m2) {
                const int u = g * (UP / 2) + m2;
                const float2 v = u < U ? rp[m2] : make_float2(0.f, 0.f);
                tl.f[2 * m2] = v.x;
                tl.f[2 * m2 + 1] = v.y;
            }
        }
#pragma unroll
        for (int m = 0; m < UP; ++m) mx = fmaxf(mx, fabsf(tl.f[m]));
    } else {
#pragma unroll
        for (int m = 0; m < UP; ++m) tl.f[m] = 0.f;
    }
    return mx;
}

// Writes a tile row-major into the wave's LDS scratch (row stride RS floats).
template <int UP, int PREC>
__device__ __forceinline__ void tile_to_lds(const Tile<UP, PREC> &tl, float *scr) {
    constexpr int RS = Shape<UP>::RS;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    float *rp = scr + j * RS + g * UP;
#pragma unroll
    for (int m4 = 0; m4 < UP; m4 += 4)
        *(float4 *)(rp + m4) = make_float4(tl.f[m4], tl.f[m4 + 1], tl.f[m4 + 2], tl.f[m4 + 3]);
}

// For 16-bit MFMA: splits the tile (scaled by sc) into hi + lo once.
template <int UP, int PREC>
__device__ __forceinline__ void tile_split(Tile<UP, PREC> &tl, float sc) {
    if constexpr (PREC != kF32) {
#pragma unroll
        for (int q = 0; q < UP / 8; ++q) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = tl.f[8 * q + e] * sc;
            Split<PREC>::split(v, tl.hi[q], tl.lo[q]);
        }
    }
}

// X^T tile from a register channel tile: rows (k, re/im) of a 16-symbol
// chunk, columns = the tile's 32 rows, times `post` (and the Z unscale).
template <int UP, int PREC>
__device__ __forceinline__ floatx16 mfma_apply_tile(const Tile<UP, PREC> &tl, float post, const ZOp<UP, PREC> &z) {
    floatx16 acc = {0};
    if constexpr (PREC == kF32) {
#pragma unroll
        for (int m = 0; m < UP; ++m) acc = mfma32(z.f[m], tl.f[m], acc);
        acc *= post;
    } else {
#pragma unroll
        for (int q = 0; q < UP / 8; ++q) acc = mfma3<PREC>(z.hi[q], z.lo[q], tl.hi[q], tl.lo[q], acc);
        acc *= post * z.unscale;
    }
    return acc;
}

// Stores the X^T tile of rows [row0, row0 + nrows), symbols k0 .. k0 + kc - 1.
__device__ __forceinline__ void store_x(const floatx16 &a, int row0, int nrows, int k0, int kc, int n, int n_sc,
                                        int B, float2 *__restrict__ x) {
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    if (j < nrows) {
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
            const int k = tile_k(r, g);
            if (k < kc) x[((size_t)(k0 + k) * n_sc + n) * B + row0 + j] = make_float2(a[r], a[r + 1]);
        }
    }
}

template <int UP>
struct Lds {
    static constexpr int SCRF = 32 * Shape<UP>::RS > 2 * Shape<UP>::SLOT ? 32 * Shape<UP>::RS : 2 * Shape<UP>::SLOT;
    // per wave: scratch (SCRF floats; Gram transpose, then partial / Z) and
    // one system slot (SLOT complex)
    static constexpr size_t per_wave = (size_t)SCRF * 4 + (size_t)Shape<UP>::SLOT * 8;
    static __host__ __device__ constexpr size_t bytes(int K, int nw) { return (size_t)K * 2 * UP * 4 + nw * per_wave; }
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

// Minimum waves per SIMD the register allocation targets (more channel tiles
// per wave need more registers).
template <int UP, int MAXT>
constexpr int min_waves() {
    return UP == 16 ? (MAXT <= 2 ? 4 : (MAXT <= 4 ? 2 : 1)) : (MAXT <= 2 ? 2 : 1);
}

// ---- the kernel body -----------------------------------------------------------
// One workgroup of NW waves (block index blk of its problem) per PD
// subcarrier, or per FD (subcarrier, group of NW clusters).  Wave w owns up to
// MAXT channel tiles:
//   PD: tiles t = w, w + NW, ... of 32 rows over the whole array;
//   FD: the tiles (32 rows each) of cluster NW * (group) + w.
// off: the problem's cluster offsets (p.off) in memory the kernel can index.
template <int UP, int ARCH, int PREC, int MAXT, int NW>
__device__ __forceinline__ void fused_body(const Prob &p, const int *__restrict__ off, int blk, int K, int mode,
                                           const float2 *__restrict__ H, const float2 *__restrict__ s,
                                           float2 *__restrict__ x, cx<float> *__restrict__ ainv_g,
                                           float *__restrict__ scale_out, int *__restrict__ status) {
    constexpr int SLOT = Shape<UP>::SLOT;
    constexpr int NTT = Shape<UP>::NTT;
    constexpr int SCRF = Lds<UP>::SCRF;
    constexpr int NT = 64 * NW;
    extern __shared__ float4 smem4[];
    float *Ss = (float *)smem4;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    char *wbase = (char *)(Ss + (size_t)K * 2 * UP);
    float *scr_of[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) scr_of[w] = (float *)(wbase + w * Lds<UP>::per_wave);
    float *scr = scr_of[wave];
    cx<float> *sA = (cx<float> *)(scr + SCRF);
    __shared__ float sh_scale, sh_amax;
    __shared__ int sh_ok;

    // PD: one workgroup per subcarrier; FD: one workgroup per (subcarrier,
    // group of NW clusters), one cluster per wave
    const int CQ = ARCH == kPD ? 1 : (p.C + NW - 1) / NW;
    const int B = p.B, U = p.U, n = blk / CQ, cq = blk % CQ;
    const float2 *Hn = H + (size_t)n * B * U;
    const bool vec = U == UP && (((uintptr_t)H) & 15) == 0;

    // symbols of this subcarrier
    for (int e = tid; e < K * UP; e += NT) {
        const int k = e / UP, u = e % UP;
        const float2 v = (u < U) ? s[((size_t)k * p.n_sc + n) * U + u] : make_float2(0.f, 0.f);
        *(float2 *)(Ss + k * 2 * UP + 2 * u) = v;
    }
    Tile<UP, PREC> tiles[MAXT];
    int t_row0[MAXT], t_rows[MAXT];

    if (ARCH == kPD) {
        const float kap = pd_kappa(p);
        // this wave's tiles: t = wave, wave + 4, ... of 32 rows
        float hmax = 0.f;
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int tt = wave + NW * q;
            t_row0[q] = 32 * tt;
            t_rows[q] = max(0, min(32, B - 32 * tt));
            hmax = fmaxf(hmax, load_tile<UP, PREC>(Hn, U, t_row0[q], t_rows[q], vec, tiles[q]));
        }
        // power-of-two operand scale of this wave's rows (16-bit MFMA)
        const int eh = PREC == kF32 ? 0 : fp16_exp(wave_max(hmax));
        const float hsc = ldexpf(1.f, eh), hunsc = ldexpf(1.f, -eh), gunsc = ldexpf(1.f, -2 * eh);
        // the wave that factors and solves rotates with the block index so that
        // the serial steps of co-resident workgroups land on different SIMDs
        const int mw = blk % NW;
        float *scr_m = (float *)(wbase + mw * Lds<UP>::per_wave);
        cx<float> *A0 = (cx<float> *)(scr_m + SCRF);
        if (mode == kSymbols) {
            // per-frame factors from the prepare pass: scale * A^-1
#pragma unroll
            for (int q = 0; q < MAXT; ++q) tile_split<UP, PREC>(tiles[q], hsc);
            if (wave == mw) {
                const float amax = load_factor<UP>(ainv_g + (size_t)n * U * U, U, A0);
                if (lane == 0) {
                    sh_scale = 1.f;
                    sh_ok = 1;
                    sh_amax = amax;
                }
            }
            __syncthreads();
        } else {
        // split-K Gram over this wave's tiles (transposed through the scratch)
        floatx16 acc[NTT];
#pragma unroll
        for (int q = 0; q < NTT; ++q) acc[q] = floatx16{0};
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            if (t_rows[q] > 0) {
                tile_to_lds<UP, PREC>(tiles[q], scr);
                wave_sync();
                mfma_gram<UP, PREC>(scr, Shape<UP>::RS, t_rows[q], hsc, acc);
                wave_sync();
            }
            tile_split<UP, PREC>(tiles[q], hsc);
        }
        cx<float> *part = (cx<float> *)scr;
        for (int e = lane; e < SLOT; e += 64) part[e] = {0.f, 0.f};
        wave_sync();
        gram_store<UP>(acc, part, gunsc, 0.f, U);
        __syncthreads();
        // partial (cluster) sum in fixed order + kappa I, into the master slot
        for (int e = tid; e < UP * UP; e += NT) {
            const int u = e / UP, v = e % UP;
            const int o = u * Shape<UP>::LDc + v;
            cx<float> sum = ((cx<float> *)scr_of[0])[o];
#pragma unroll
            for (int w = 1; w < NW; ++w) sum = cadd(sum, ((cx<float> *)scr_of[w])[o]);
            if (u == v && u < U) sum.re += kap;
            A0[o] = sum;
        }
        __syncthreads();
        if (wave == mw) {
            float t = 0.f, amax = 0.f;
            const bool ok = wave_factor<UP>(A0, U, kap, &t, &amax);
            const float beta = ok ? sqrtf(p.Es / p.power * t) : 0.f;
            if (lane == 0) {
                sh_scale = ok ? 1.f / beta : 0.f;
                sh_ok = ok;
                sh_amax = amax;
                if (scale_out) scale_out[n] = beta;
                if (status) status[n] = ok ? PRECODE_ST_OK : PRECODE_ST_FAIL;
            }
            if (mode == kPrepare) store_factor<UP>(A0, U, ok ? 1.f / beta : 0.f, ainv_g + (size_t)n * U * U);
        }
        __syncthreads();
        }
        cx<float> *Zw = (cx<float> *)scr_m;  // free after the partial sum
        for (int k0 = 0; mode != kPrepare && k0 < K; k0 += KC) {
            const int kc = min(KC, K - k0);
            if (wave == mw) wave_solve_chunk<UP, PREC>(A0, Zw, Ss, k0, kc, U, sh_scale, sh_amax, sh_ok != 0);
            __syncthreads();
            ZOp<UP, PREC> z;
            make_zop<UP, PREC>(Zw, KC, 1, kc, z);
#pragma unroll
            for (int q = 0; q < MAXT; ++q)
                if (t_rows[q] > 0) {
                    const floatx16 a = mfma_apply_tile<UP, PREC>(tiles[q], hunsc, z);
                    store_x(a, t_row0[q], t_rows[q], k0, kc, n, p.n_sc, B, x);
                }
            __syncthreads();
        }
    } else {
        __syncthreads();  // symbols staged
        const float kap = fd_kappa(p);
        const float rho_c2 = p.power / (float)p.C;
        const int c = NW * cq + wave;
        if (c < p.C) {
            const int o0 = off[c], o1 = off[c + 1];
            // this cluster's rows as tiles of 32
            float hmax = 0.f;
#pragma unroll
            for (int q = 0; q < MAXT; ++q) {
                t_row0[q] = o0 + 32 * q;
                t_rows[q] = max(0, min(32, o1 - t_row0[q]));
                hmax = fmaxf(hmax, load_tile<UP, PREC>(Hn, U, t_row0[q], t_rows[q], vec, tiles[q]));
            }
            const int eh = PREC == kF32 ? 0 : fp16_exp(wave_max(hmax));
            const float hsc = ldexpf(1.f, eh), hunsc = ldexpf(1.f, -eh), gunsc = ldexpf(1.f, -2 * eh);
            cx<float> *fac = ainv_g + ((size_t)n * p.C + c) * U * U;
            float w = 1.f, amax = 0.f;
            bool ok = true;
            if (mode == kSymbols) {
#pragma unroll
                for (int q = 0; q < MAXT; ++q) tile_split<UP, PREC>(tiles[q], hsc);
                amax = load_factor<UP>(fac, U, sA);
            } else {
                for (int e = lane; e < SLOT; e += 64) sA[e] = {0.f, 0.f};
                floatx16 acc[NTT];
#pragma unroll
                for (int q = 0; q < NTT; ++q) acc[q] = floatx16{0};
#pragma unroll
                for (int q = 0; q < MAXT; ++q)
                    if (t_rows[q] > 0) {
                        tile_to_lds<UP, PREC>(tiles[q], scr);
                        wave_sync();
                        mfma_gram<UP, PREC>(scr, Shape<UP>::RS, t_rows[q], hsc, acc);
                        wave_sync();
                        tile_split<UP, PREC>(tiles[q], hsc);
                    }
                gram_store<UP>(acc, sA, gunsc, kap, U);
                wave_sync();
                float t = 0.f;
                ok = wave_factor<UP>(sA, U, kap, &t, &amax);
                w = ok ? sqrtf(rho_c2 / (t * p.Es)) : 0.f;
                if (lane == 0) {
                    if (scale_out) scale_out[(size_t)n * p.C + c] = w;
                    if (status) status[(size_t)n * p.C + c] = ok ? PRECODE_ST_OK : PRECODE_ST_FAIL;
                }
                if (mode == kPrepare) store_factor<UP>(sA, U, w, fac);
            }
            cx<float> *Zw = (cx<float> *)scr;
            for (int k0 = 0; mode != kPrepare && k0 < K; k0 += KC) {
                const int kc = min(KC, K - k0);
                wave_sync();
                wave_solve_chunk<UP, PREC>(sA, Zw, Ss, k0, kc, U, w, amax, ok);
                wave_sync();
                ZOp<UP, PREC> z;
                make_zop<UP, PREC>(Zw, KC, 1, kc, z);
#pragma unroll
                for (int q = 0; q < MAXT; ++q)
                    if (t_rows[q] > 0) {
                        const floatx16 a = mfma_apply_tile<UP, PREC>(tiles[q], hunsc, z);
                        store_x(a, t_row0[q], t_rows[q], k0, kc, n, p.n_sc, B, x);
                    }
            }
        }
    }
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

// Channel tiles (32 rows) a wave holds in registers with nw waves per workgroup.
int tiles_per_wave(const Prob &p, int nw) {
    if (p.arch == kPD) return ((p.B + 31) / 32 + nw - 1) / nw;
    int worst = 0;  // FD: a wave holds one cluster at a time
    for (int c = 0; c < p.C; ++c) {
        const int n = (p.off[c + 1] - p.off[c] + 31) / 32;
        worst = n > worst ? n : worst;
    }
    return worst;
}

// Most channel tiles a wave may hold: register capacity at the occupancy
// min_waves asks for (an 8-wave workgroup already needs two waves per SIMD).
constexpr int max_tiles(int up, int nw) { return up == 16 ? (nw <= 4 ? 8 : 4) : (nw <= 4 ? 4 : 2); }

int pick_maxt(const Prob &p, int up, int nw) {
    const int t = tiles_per_wave(p, nw);
    const int lim = max_tiles(up, nw);
    if (t <= 1) return 1;
    if (t <= 2) return 2;
    if (t <= 4 && lim >= 4) return 4;
    if (t <= 8 && lim >= 8) return 8;
    return 0;
}

constexpr size_t kLdsMax = 160 * 1024;

}  // namespace
}  // namespace pc
