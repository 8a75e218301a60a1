// fused.hip -- single-launch fused PD / FD precoding on gfx950.
//
// Persistent 256-thread workgroups (4 wave64s); a workgroup processes
// subcarriers n = blockIdx.x, blockIdx.x + gridDim.x, ...  The channel of a
// subcarrier (B x U complex64) and its K symbol vectors are staged once in
// LDS (the next subcarrier's channel is prefetched into registers meanwhile);
// every step of the method then runs out of LDS and registers:
//
//   Gram        G_c = H_c^H H_c on MFMA over the real embedding
//               [Re h_u, Im h_u] of the columns: the 2U x 2U real Gram M
//               gives G = (M_rr + M_ii) + i (M_ri - M_ir) (local Gram,
//               Sec. III-B; PD sums the cluster Grams as a split-K reduction,
//               the on-chip form of the adder tree)
//   regularize  A = G + kappa I (PD) / A_c = G_c + kappa_c I (FD,
//               kappa_c = tau_c C kappa, eq. regularization)
//   invert      A^-1 in registers, one wave per system (Gauss-Jordan
//               elimination; for Hermitian positive-definite A its pivots are
//               the squared diagonal of the Cholesky factor)
//   factor      t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1);
//               PD beta = sqrt(Es/rho^2 t); FD w_c = sqrt(rho_c^2/(t Es))
//   solve       Z = scale * A^-1 S for a chunk of 16 symbols, on MFMA
//   precode     X_c = H_c Z on MFMA (the per-cluster product of Sec. III-B;
//               FD x_c = w_c H_c A_c^-1 s, Sec. III-C), stored coalesced.
//
// MFMA precision (template PREC): FP32 (v_mfma_f32_32x32x2f32, exact FP32
// products) or split 16-bit: every operand x is written as hi + lo with
// hi = f16(x), lo = f16(x - hi) (or bf16) and a product a b is accumulated as
// ah bh + ah bl + al bh in FP32 (v_mfma_f32_32x32x16_f16 / _bf16).  Operands
// are scaled by powers of two into the FP16 range first and the FP32 results
// unscaled exactly.
//
// PD: the four waves split the rows for the Gram, wave 0 factors, all four
// waves precode.  FD: each wave owns whole clusters (c = wave, wave+4, ...)
// and runs the full chain for them without workgroup barriers.
#include "common.h"

namespace pc {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
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
        for (int r = 0; r < nrows; r += 2) {
            const int row = r + g;
            float a[NT];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti) a[ti] = row < nrows ? rows[row * rs + 32 * ti + j] : 0.f;
            int t = 0;
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = ti; tj < NT; ++tj) {
                    acc[t] = mfma32(a[ti], a[tj], acc[t]);
                    ++t;
                }
        }
    } else {
        typedef typename Split<PREC>::V V;
        for (int r = 0; r < nrows; r += 16) {
            V hi[NT], lo[NT];
#pragma unroll
            for (int ti = 0; ti < NT; ++ti) {
                float v[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int row = r + 8 * g + e;
                    v[e] = row < nrows ? rows[row * rs + 32 * ti + j] * sc : 0.f;
                }
                Split<PREC>::split(v, hi[ti], lo[ti]);
            }
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
            const bool iscol = c == k;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const bool isrow = (s * R + r) == k;
                const float aik_re = bcast_row_dyn<UP>(re[s], k);
                const float aik_im = bcast_row_dyn<UP>(im[s], k);
                // generic element: a_ic - a_ik a_kc / a_kk
                const float tre = aik_re * akc_re - aik_im * akc_im;
                const float tim = aik_re * akc_im + aik_im * akc_re;
                const float gre = re[s] - tre * inv, gim = im[s] - tim * inv;
                // row k: a_kc / a_kk ; column k: -a_ik / a_kk ; pivot: 1 / a_kk
                const float rre = iscol ? inv : re[s] * inv, rim = iscol ? 0.f : im[s] * inv;
                const float cre = -aik_re * inv, cim = -aik_im * inv;
                re[s] = isrow ? rre : (iscol ? cre : gre);
                im[s] = isrow ? rim : (iscol ? cim : gim);
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

// x rows [r0, r0 + nrows) of subcarrier n for chunk (k0, kc) from Z in slot zs;
// this wave takes the 32-row tiles t = tile0, tile0 + tstep, ...
template <int UP, int PREC>
__device__ void wave_precode_rows(const float *Hs, const cx<float> *zs, int r0, int nrows, int k0, int kc, int n,
                                  int n_sc, int B, float2 *__restrict__ x, int tile0, int tstep, float hsc,
                                  float hunsc) {
    constexpr int RS = Shape<UP>::RS;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    ZOp<UP, PREC> z;
    make_zop<UP, PREC>(zs, KC, 1, kc, z);
    for (int t = tile0; t * 32 < nrows; t += tstep) {
        const int rb = r0 + t * 32;
        const int nv = min(32, nrows - t * 32);
        const floatx16 a = mfma_apply<UP, PREC>(Hs + rb * RS, RS, nv, hsc, hunsc, z);
        if (j < nv) {
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
                const int k = tile_k(r, g);
                if (k < kc) x[((size_t)(k0 + k) * n_sc + n) * B + rb + j] = make_float2(a[r], a[r + 1]);
            }
        }
    }
}

// ---- staging ----------------------------------------------------------------
// Copies the B x U complex64 channel of one subcarrier into LDS rows of stride
// RS floats; returns this thread's max |component| over what it stored.  Each
// thread issues a batch of NB loads before its LDS stores, so a whole batch is
// in flight at once.
template <int UP>
__device__ __forceinline__ float stage_channel(const float2 *__restrict__ Hn, float *Hs, int B, int U) {
    constexpr int RS = Shape<UP>::RS;
    constexpr int NB = 8;
    const int tid = threadIdx.x;
    float mx = 0.f;
    const int nf = B * U;
    for (int base = 0; base < nf; base += kThreads * NB) {
        float2 r[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int f = base + j * kThreads + tid;
            r[j] = f < nf ? Hn[f] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int f = base + j * kThreads + tid;
            if (f < nf) {
                const int b = f / U, u = f - b * U;
                *(float2 *)(Hs + b * RS + 2 * u) = r[j];
                mx = fmaxf(mx, fmaxf(fabsf(r[j].x), fabsf(r[j].y)));
            }
        }
    }
    return mx;
}

// Zeroes the padding users U..UP-1 of every staged row.
template <int UP>
__device__ __forceinline__ void zero_padding(float *Hs, int B, int U) {
    constexpr int RS = Shape<UP>::RS;
    if (U < UP) {
        const int pad = UP - U;
        for (int e = threadIdx.x; e < B * pad; e += kThreads) {
            const int b = e / pad, u = U + (e - b * pad);
            *(float2 *)(Hs + b * RS + 2 * u) = make_float2(0.f, 0.f);
        }
    }
}

// Register prefetch of the next subcarrier's channel: the first kPF float4
// of each thread's share are loaded while the current subcarrier computes and
// written to LDS afterwards (channels with an even user count only).
constexpr int kPF = 8;

__device__ __forceinline__ void prefetch_issue(float4 (&pf)[kPF], const float2 *__restrict__ Hn, int nf) {
    const float4 *src = (const float4 *)Hn;
#pragma unroll
    for (int j = 0; j < kPF; ++j) {
        const int f = j * kThreads + (int)threadIdx.x;
        pf[j] = f < nf ? src[f] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__device__ __forceinline__ float max4(float4 v) {
    return fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w)));
}

template <int UP>
__device__ __forceinline__ float prefetch_commit(const float4 (&pf)[kPF], const float2 *__restrict__ Hn, float *Hs,
                                                 int B, int U) {
    constexpr int RS = Shape<UP>::RS;
    const int hu = U >> 1, nf = B * hu;
    const int tid = threadIdx.x;
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < kPF; ++j) {
        const int f = j * kThreads + tid;
        if (f < nf) {
            const int b = f / hu, c = f - b * hu;
            *(float4 *)(Hs + b * RS + 4 * c) = pf[j];
            mx = fmaxf(mx, max4(pf[j]));
        }
    }
    const float4 *src = (const float4 *)Hn;
    for (int f = kPF * kThreads + tid; f < nf; f += kThreads) {
        const int b = f / hu, c = f - b * hu;
        const float4 v = src[f];
        *(float4 *)(Hs + b * RS + 4 * c) = v;
        mx = fmaxf(mx, max4(v));
    }
    return mx;
}

template <int UP>
__host__ __device__ constexpr size_t lds_bytes(int B, int K) {
    return (size_t)B * Shape<UP>::RS * 4 + (size_t)K * 2 * UP * 4 + (size_t)8 * Shape<UP>::SLOT * 8;
}

// ---- the kernel -----------------------------------------------------------------
template <int UP, int ARCH, int PREC>
__global__ void __launch_bounds__(kThreads, UP == 16 ? 2 : 1) fused_k(Prob p, int K, const float2 *__restrict__ H,
                                                    const float2 *__restrict__ s, float2 *__restrict__ x,
                                                    float *__restrict__ scale_out, int *__restrict__ status) {
    constexpr int RS = Shape<UP>::RS;
    constexpr int SLOT = Shape<UP>::SLOT;
    constexpr int NTT = Shape<UP>::NTT;
    extern __shared__ float4 smem4[];
    float *Hs = (float *)smem4;
    float *Ss = Hs + (size_t)p.B * RS;
    cx<float> *slots = (cx<float> *)(Ss + (size_t)K * 2 * UP);
    __shared__ float sh_scale, sh_amax;
    __shared__ int sh_ok;
    __shared__ float sh_hmax[4];

    const int B = p.B, U = p.U;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    cx<float> *sA = slots + (2 * wave) * SLOT;
    cx<float> *sB = slots + (2 * wave + 1) * SLOT;
    const bool vec = (U & 1) == 0 && (((uintptr_t)H) & 15) == 0;
    const int nf = B * (U >> 1);
    float4 pf[kPF];
    if (vec && (int)blockIdx.x < p.n_sc) prefetch_issue(pf, H + (size_t)blockIdx.x * B * U, nf);

    for (int n = blockIdx.x; n < p.n_sc; n += gridDim.x) {
        // ---- stage H[n] (zero-padded to UP users) and s[:, n] in LDS ------
        float mx = vec ? prefetch_commit<UP>(pf, H + (size_t)n * B * U, Hs, B, U)
                       : stage_channel<UP>(H + (size_t)n * B * U, Hs, B, U);
        zero_padding<UP>(Hs, B, U);
        for (int e = tid; e < K * UP; e += kThreads) {
            const int k = e / UP, u = e % UP;
            const float2 v = (u < U) ? s[((size_t)k * p.n_sc + n) * U + u] : make_float2(0.f, 0.f);
            *(float2 *)(Ss + k * 2 * UP + 2 * u) = v;
        }
        for (int e = tid; e < 8 * SLOT; e += kThreads) slots[e] = {0.f, 0.f};
        if (PREC != kF32) {
            mx = wave_max(mx);
            if (lane == 0) sh_hmax[wave] = mx;
        }
        __syncthreads();
        // the next subcarrier's channel is in flight while this one computes
        if (vec && n + (int)gridDim.x < p.n_sc) prefetch_issue(pf, H + (size_t)(n + gridDim.x) * B * U, nf);
        // power-of-two operand scale of the channel for 16-bit MFMA
        int eh = 0;
        if (PREC != kF32) eh = fp16_exp(fmaxf(fmaxf(sh_hmax[0], sh_hmax[1]), fmaxf(sh_hmax[2], sh_hmax[3])));
        const float hsc = ldexpf(1.f, eh), hunsc = ldexpf(1.f, -eh), gunsc = ldexpf(1.f, -2 * eh);

        if (ARCH == kPD) {
            const float kap = pd_kappa(p);
            // split-K Gram: four contiguous row ranges (multiples of 16 rows)
            const int rows_per = ((B + 63) / 64) * 16;
            const int r0 = min(B, wave * rows_per), r1 = min(B, r0 + rows_per);
            floatx16 acc[NTT];
#pragma unroll
            for (int q = 0; q < NTT; ++q) acc[q] = floatx16{0};
            mfma_gram<UP, PREC>(Hs + r0 * RS, RS, r1 - r0, hsc, acc);
            gram_store<UP>(acc, sA, gunsc, 0.f, U);
            __syncthreads();
            // partial (cluster) sum in fixed order + kappa I, into wave 0's slot A
            for (int e = tid; e < UP * UP; e += kThreads) {
                const int u = e / UP, v = e % UP;
                const int o = u * Shape<UP>::LDc + v;
                cx<float> sum = slots[o];
#pragma unroll
                for (int w = 1; w < 4; ++w) sum = cadd(sum, slots[2 * w * SLOT + o]);
                if (u == v && u < U) sum.re += kap;
                slots[o] = sum;
            }
            __syncthreads();
            if (wave == 0) {
                float t = 0.f, amax = 0.f;
                const bool ok = wave_factor<UP>(sA, U, kap, &t, &amax);
                const float beta = ok ? sqrtf(p.Es / p.power * t) : 0.f;
                if (lane == 0) {
                    sh_scale = ok ? 1.f / beta : 0.f;
                    sh_ok = ok;
                    sh_amax = amax;
                    if (scale_out) scale_out[n] = beta;
                    if (status) status[n] = ok ? PRECODE_ST_OK : PRECODE_ST_FAIL;
                }
            }
            __syncthreads();
            const cx<float> *z0 = slots + SLOT;  // wave 0's slot B
            for (int k0 = 0; k0 < K; k0 += KC) {
                const int kc = min(KC, K - k0);
                if (wave == 0) wave_solve_chunk<UP, PREC>(sA, sB, Ss, k0, kc, U, sh_scale, sh_amax, sh_ok != 0);
                __syncthreads();
                wave_precode_rows<UP, PREC>(Hs, z0, 0, B, k0, kc, n, p.n_sc, B, x, wave, 4, hsc, hunsc);
                __syncthreads();
            }
        } else {
            const float kap = fd_kappa(p);
            const float rho_c2 = p.power / (float)p.C;
            for (int c = wave; c < p.C; c += 4) {
                const int o = p.off[c], Bc = p.off[c + 1] - o;
                for (int e = lane; e < SLOT; e += 64) {
                    sA[e] = {0.f, 0.f};
                    sB[e] = {0.f, 0.f};
                }
                wave_sync();
                floatx16 acc[NTT];
#pragma unroll
                for (int q = 0; q < NTT; ++q) acc[q] = floatx16{0};
                mfma_gram<UP, PREC>(Hs + o * RS, RS, Bc, hsc, acc);
                gram_store<UP>(acc, sA, gunsc, kap, U);
                wave_sync();
                float t = 0.f, amax = 0.f;
                const bool ok = wave_factor<UP>(sA, U, kap, &t, &amax);
                const float w = ok ? sqrtf(rho_c2 / (t * p.Es)) : 0.f;
                if (lane == 0) {
                    if (scale_out) scale_out[(size_t)n * p.C + c] = w;
                    if (status) status[(size_t)n * p.C + c] = ok ? PRECODE_ST_OK : PRECODE_ST_FAIL;
                }
                wave_sync();
                for (int k0 = 0; k0 < K; k0 += KC) {
                    const int kc = min(KC, K - k0);
                    wave_solve_chunk<UP, PREC>(sA, sB, Ss, k0, kc, U, w, amax, ok);
                    wave_sync();
                    wave_precode_rows<UP, PREC>(Hs, sB, o, Bc, k0, kc, n, p.n_sc, B, x, 0, 1, hsc, hunsc);
                    wave_sync();
                }
            }
        }
        __syncthreads();  // every LDS read of this subcarrier precedes the next staging
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

constexpr size_t kLdsMax = 160 * 1024;

template <int UP, int ARCH, int PREC>
hipError_t launch(const Prob &p, int K, const float2 *H, const float2 *s, float2 *x, float *scale_out, int *status,
                  hipStream_t st) {
    const void *fn = (const void *)fused_k<UP, ARCH, PREC>;
    const size_t lds = lds_bytes<UP>(p.B, K);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // persistent grid: as many workgroups as fit on the device at once
    static int cached_lds = -1, cached_grid = 0;
    if (cached_lds != (int)lds) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds);
        if (e != hipSuccess) return e;
        cached_grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
        cached_lds = (int)lds;
    }
    const int grid = p.n_sc < cached_grid ? p.n_sc : cached_grid;
    hipLaunchKernelGGL((fused_k<UP, ARCH, PREC>), dim3(grid), dim3(kThreads), lds, st, p, K, H, s, x, scale_out,
                       status);
    return hipGetLastError();
}

template <int UP, int ARCH>
hipError_t launch_prec(int prec, const Prob &p, int K, const float2 *H, const float2 *s, float2 *x, float *so,
                       int *sto, hipStream_t st) {
    switch (prec) {
        case kF32: return launch<UP, ARCH, kF32>(p, K, H, s, x, so, sto, st);
        case kF16: return launch<UP, ARCH, kF16>(p, K, H, s, x, so, sto, st);
        default: return launch<UP, ARCH, kBF16>(p, K, H, s, x, so, sto, st);
    }
}

}  // namespace

bool fused_supported(const Prob &p, int precision) {
    if (prec_of(precision) < 0) return false;
    const int up = pick_up(p.U);
    if (up == 0) return false;
    const int kmax = p.K < kMaxKFused ? p.K : kMaxKFused;
    const size_t lds = up == 16 ? lds_bytes<16>(p.B, kmax) : lds_bytes<32>(p.B, kmax);
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
    const int up = pick_up(p.U);
    const int prec = prec_of(precision);
    for (int k0 = 0; k0 < p.K; k0 += kMaxKFused) {
        const int kk = p.K - k0 < kMaxKFused ? p.K - k0 : kMaxKFused;
        const float2 *sk = s + (size_t)k0 * p.n_sc * p.U;
        float2 *xk = x + (size_t)k0 * p.n_sc * p.B;
        // factors are identical for every slice; write them once
        float *so = k0 == 0 ? scale_out : nullptr;
        int *sto = k0 == 0 ? status : nullptr;
        hipError_t e;
        if (up == 16)
            e = p.arch == kPD ? launch_prec<16, kPD>(prec, p, kk, H, sk, xk, so, sto, st)
                              : launch_prec<16, kFD>(prec, p, kk, H, sk, xk, so, sto, st);
        else
            e = p.arch == kPD ? launch_prec<32, kPD>(prec, p, kk, H, sk, xk, so, sto, st)
                              : launch_prec<32, kFD>(prec, p, kk, H, sk, xk, so, sto, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pc
