// fused.hip -- single-launch fused PD / FD precoding on gfx950.
//
// One 256-thread workgroup (4 wave64s) per subcarrier.  The channel of the
// subcarrier (B x U complex64) and its K symbol vectors are staged once in
// LDS; every step of the method then runs out of LDS:
//
//   Gram        G_c = H_c^H H_c on MFMA (v_mfma_f32_32x32x2f32) over the
//               real embedding [Re h_u, Im h_u] of the columns: the 2U x 2U
//               real Gram M gives G = (M_rr + M_ii) + i (M_ri - M_ir)
//               (local Gram, Sec. III-B; PD sums the cluster Grams as a
//               split-K reduction, the on-chip form of the adder tree)
//   regularize  A = G + kappa I  (PD)  /  A_c = G_c + kappa_c I  (FD,
//               kappa_c = tau_c C kappa, eq. regularization)
//   Cholesky    A = L L^H, one wave per system, in LDS
//   inverse     W = L^-1 (forward substitution), A^-1 = W^H W on MFMA
//   factor      t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1);
//               PD beta = sqrt(Es/rho^2 t); FD w_c = sqrt(rho_c^2/(t Es))
//   solve       Z = scale * A^-1 S for a chunk of 16 symbols, on MFMA
//   precode     X_c = H_c Z on MFMA (the per-cluster product of Sec. III-B;
//               FD x_c = w_c H_c A_c^-1 s, Sec. III-C), stored coalesced.
//
// PD: the four waves split the rows for the Gram, wave 0 factors, all four
// waves precode.  FD: each wave owns whole clusters (c = wave, wave+4, ...)
// and runs the full chain for them without workgroup barriers.
#include "common.h"

namespace pc {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int KC = 16;        // symbols per MFMA chunk: 2*KC = 32 rows of X^T
constexpr int kMaxKFused = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Orders LDS accesses of one wave (a wave's LDS operations execute in order;
// this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <int UP>
struct Shape {
    static constexpr int NT = (2 * UP) / 32;        // 32-wide real column tiles
    static constexpr int NTT = NT * (NT + 1) / 2;   // tiles with ti <= tj
    static constexpr int RS = 2 * UP + 4;           // H row stride in LDS (floats)
    static constexpr int LDc = UP + 2;              // slot leading dim (complex), rows 16B aligned
    static constexpr int SLOT = UP * LDc;           // complex elements per slot
};

// Real Gram of `nrows` rows (row-major floats, stride rs): accumulates
// M[32ti+i][32tj+j] = sum_r R[r][32ti+i] R[r][32tj+j] for ti <= tj.
// v_mfma_f32_32x32x2f32 operands: lane l supplies A[l%32][l/32] and
// B[l/32][l%32]; here both are R[row][col], so a lane loads one value per
// column tile per two rows.
template <int UP>
__device__ __forceinline__ void mfma_gram(const float *rows, int rs, int nrows,
                                          floatx16 (&acc)[Shape<UP>::NTT]) {
    constexpr int NT = Shape<UP>::NT;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;

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
}

// Turns the real Gram tiles into the complex U x U matrix in an LDS slot:
// G[u][v] = (M[2u][2v] + M[2u+1][2v+1]) + i (M[2u][2v+1] - M[2u+1][2v]),
// plus diag_add on the diagonal for u < m.  Output layout of the 32x32
// MFMA: lane l, register r holds row 8(r/4) + 4(l/32) + r%4, column l%32.
// The even-column lane of each pair combines its values with its partner's.
// With stats, accumulates tr G (u < m) and ||G||_F^2 into *tr, *fro (per lane).
template <int UP>
__device__ __forceinline__ void gram_store(const floatx16 (&acc)[Shape<UP>::NTT], cx<float> *dst,
                                           float diag_add, int m, float *tr, float *fro) {
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
                    float gre = own0 + par1;
                    const float gim = par0 - own1;
                    if (u == v && u < m) gre += diag_add;
                    dst[u * LDc + v] = {gre, gim};
                    if (ti != tj) dst[v * LDc + u] = {gre, -gim};
                    if (tr) {
                        const float w = (ti != tj) ? 2.f : 1.f;
                        *fro += w * (gre * gre + gim * gim);
                        if (u == v) *tr += gre;
                    }
                }
            }
            ++t;
        }
}

// Per-lane A operands for X^T = Zbar^T Rows^T with X^T rows i = 2k + q
// (symbol k, q = re/im) and contraction index kk = 2u + p over the real
// columns of Rows.  The contraction is permuted so that lane half g covers
// kk = g*UP .. g*UP+UP-1 (contiguous columns).  Zbar[2u+p][2k+q] is
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

// X^T tile (32 x 32): rows (k, re/im) for a 16-symbol chunk, columns =
// rows r0 .. r0+31 of `rows` (row-major floats, stride rs; rows >= nvalid
// read as 0).  Lane l supplies B = Rows[l%32][g*UP + m] for instruction m.
template <int UP>
__device__ __forceinline__ floatx16 mfma_apply(const float *rows, int rs, int nvalid, const float (&zop)[UP]) {
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
#pragma unroll
    for (int m = 0; m < UP; ++m) acc = mfma32(zop[m], h[m], acc);
    return acc;
}

// Symbol index held by register pair (r, r+1) of an X^T tile.
__device__ __forceinline__ int tile_k(int r, int g) { return 4 * (r / 4) + 2 * g + ((r % 4) >> 1); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Broadcast within the lanes of one matrix row of the register layout below:
// lane (r, c) receives the value of lane (r, k).  For UP = 16 a row is a DPP
// row of 16 lanes (row_newbcast); for UP = 32 it is a half-wave.
template <int UP, int k>
__device__ __forceinline__ float bcast_row(float v) {
    if constexpr (UP == 16) {
        return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + k,
                                                                      0xf, 0xf, false));
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

__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// In-register inversion of the m x m Hermitian positive-definite system held
// in an LDS slot (full matrix), one wave, by Gauss-Jordan elimination without
// pivoting: step k divides row k by the pivot and eliminates column k from
// every other row, so that after m steps the slot holds A^-1.  For a Hermitian
// positive-definite A the pivots are the squared diagonal of its Cholesky
// factor and need no row exchanges.
// Layout: lane (r, c) = (lane / UP, lane % UP) holds column c, rows
// i = s*R + r (R = 64 / UP row groups, NS = UP / R slots).  Row k of the
// matrix reaches every lane through a bpermute, column k through bcast_row,
// the pivot through readlane.  Returns false when a pivot is not finite or not
// above kRelPivot32 times the original diagonal entry (numerically singular).
// On success writes A^-1 back to the slot and sets tr A^-1, ||A^-1||_F^2.
template <int UP>
__device__ bool wave_inverse(cx<float> *S, int m, float *tr_out, float *fro_out) {
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
            const float inv = 1.f / piv;
            // row k, column c (before this step's update)
            const float akc_re = __shfl(re[sk], rk * UP + c);
            const float akc_im = __shfl(im[sk], rk * UP + c);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int i = s * R + r;
                const float aik_re = bcast_row_dyn<UP>(re[s], k);
                const float aik_im = bcast_row_dyn<UP>(im[s], k);
                float nre, nim;
                if (i == k) {
                    nre = (c == k) ? inv : re[s] * inv;
                    nim = (c == k) ? 0.f : im[s] * inv;
                } else if (c == k) {
                    nre = -aik_re * inv;
                    nim = -aik_im * inv;
                } else {
                    const float tre = aik_re * akc_re - aik_im * akc_im;
                    const float tim = aik_re * akc_im + aik_im * akc_re;
                    nre = re[s] - tre * inv;
                    nim = im[s] - tim * inv;
                }
                re[s] = nre;
                im[s] = nim;
            }
        }
    }
    float tr = 0.f, fro = 0.f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = s * R + r;
        if (i < m && c < m) {
            fro += re[s] * re[s] + im[s] * im[s];
            if (i == c) tr += re[s];
        }
        S[i * LDc + c] = {re[s], im[s]};
    }
    *tr_out = wave_sum(tr);
    *fro_out = wave_sum(fro);
    return ok;
}

// Factor one system held in slot A (A = G + kappa I, full Hermitian matrix):
// on success slot A holds A^-1 and *t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1).
template <int UP>
__device__ bool wave_factor(cx<float> *sA, int m, float kap, float *t_out) {
    float tr = 0.f, fro = 0.f;
    bool ok = wave_inverse<UP>(sA, m, &tr, &fro);
    const float t = tr - kap * fro;
    ok = ok && (t > 0.f) && (t < INFINITY);
    wave_sync();
    *t_out = t;
    return ok;
}

// Z(u, k) = scale * (A^-1 S)(u, k) for one chunk into slot B as [UP][KC].
template <int UP>
__device__ void wave_solve_chunk(const cx<float> *sA, cx<float> *sB, const float *Ss, int k0, int kc, int m,
                                 float scale, bool ok) {
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    float zop[UP];
    load_zop<UP>((const cx<float> *)Ss + k0 * UP, 1, UP, kc, zop);
    const floatx16 a = mfma_apply<UP>((const float *)sA, 2 * Shape<UP>::LDc, m, zop);
    if (j < UP) {
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
            const int k = tile_k(r, g);
            if (k < KC) {
                cx<float> z = {0.f, 0.f};
                if (ok && k < kc) z = {a[r] * scale, a[r + 1] * scale};
                sB[j * KC + k] = z;
            }
        }
    }
}

// x rows [r0, r0 + nrows) of subcarrier n for chunk (k0, kc) from Z in slot zs.
template <int UP>
__device__ void wave_precode_rows(const float *Hs, const cx<float> *zs, int r0, int nrows, int k0, int kc,
                                  int n, int n_sc, int B, float2 *__restrict__ x, int tile0, int tstep) {
    constexpr int RS = Shape<UP>::RS;
    const int lane = lane_id();
    const int j = lane & 31, g = lane >> 5;
    float zop[UP];
    load_zop<UP>(zs, KC, 1, kc, zop);
    for (int t = tile0; t * 32 < nrows; t += tstep) {
        const int rb = r0 + t * 32;
        const int nv = min(32, nrows - t * 32);
        const floatx16 a = mfma_apply<UP>(Hs + rb * RS, RS, nv, zop);
        if (j < nv) {
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
                const int k = tile_k(r, g);
                if (k < kc) x[((size_t)(k0 + k) * n_sc + n) * B + rb + j] = make_float2(a[r], a[r + 1]);
            }
        }
    }
}

// Copies the B x U complex64 channel of one subcarrier into LDS rows of stride
// RS floats and zeroes the padding users U..UP-1.  Each thread issues a batch
// of NB loads before its LDS stores, so a whole batch is in flight at once.
template <int UP>
__device__ __forceinline__ void stage_channel(const float2 *__restrict__ Hn, float *Hs, int B, int U) {
    constexpr int RS = Shape<UP>::RS;
    constexpr int NB = 8;
    const int tid = threadIdx.x;
    if ((U & 1) == 0 && (((uintptr_t)Hn) & 15) == 0) {
        const float4 *src = (const float4 *)Hn;
        const int hu = U >> 1;  // float4 per row
        const int nf = B * hu;
        for (int base = 0; base < nf; base += kThreads * NB) {
            float4 r[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int f = base + j * kThreads + tid;
                r[j] = f < nf ? src[f] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int f = base + j * kThreads + tid;
                if (f < nf) {
                    const int b = f / hu, c = f - b * hu;
                    *(float4 *)(Hs + b * RS + 4 * c) = r[j];
                }
            }
        }
    } else {
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
                }
            }
        }
    }
    if (U < UP) {
        const int pad = UP - U;
        for (int e = tid; e < B * pad; e += kThreads) {
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

template <int UP>
__device__ __forceinline__ void prefetch_commit(const float4 (&pf)[kPF], const float2 *__restrict__ Hn, float *Hs,
                                                int B, int U) {
    constexpr int RS = Shape<UP>::RS;
    const int hu = U >> 1, nf = B * hu;
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kPF; ++j) {
        const int f = j * kThreads + tid;
        if (f < nf) {
            const int b = f / hu, c = f - b * hu;
            *(float4 *)(Hs + b * RS + 4 * c) = pf[j];
        }
    }
    const float4 *src = (const float4 *)Hn;
    for (int f = kPF * kThreads + tid; f < nf; f += kThreads) {
        const int b = f / hu, c = f - b * hu;
        *(float4 *)(Hs + b * RS + 4 * c) = src[f];
    }
    if (U < UP) {
        const int pad = UP - U;
        for (int e = tid; e < B * pad; e += kThreads) {
            const int b = e / pad, u = U + (e - b * pad);
            *(float2 *)(Hs + b * RS + 2 * u) = make_float2(0.f, 0.f);
        }
    }
}

template <int UP>
__host__ __device__ constexpr size_t lds_bytes(int B, int K) {
    return (size_t)B * Shape<UP>::RS * 4 + (size_t)K * 2 * UP * 4 + (size_t)8 * Shape<UP>::SLOT * 8;
}

template <int UP, int ARCH>
__global__ void __launch_bounds__(kThreads) fused_k(Prob p, int K, const float2 *__restrict__ H,
                                                    const float2 *__restrict__ s, float2 *__restrict__ x,
                                                    float *__restrict__ scale_out, int *__restrict__ status) {
    constexpr int RS = Shape<UP>::RS;
    constexpr int SLOT = Shape<UP>::SLOT;
    constexpr int NTT = Shape<UP>::NTT;
    extern __shared__ float4 smem4[];
    float *Hs = (float *)smem4;
    float *Ss = Hs + (size_t)p.B * RS;
    cx<float> *slots = (cx<float> *)(Ss + (size_t)K * 2 * UP);
    __shared__ float sh_scale;
    __shared__ int sh_ok;

    const int B = p.B, U = p.U;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    cx<float> *sA = slots + (2 * wave) * SLOT;
    cx<float> *sB = slots + (2 * wave + 1) * SLOT;
    // persistent blocks: subcarriers n = blockIdx.x, blockIdx.x + gridDim.x, ...
    const bool vec = (U & 1) == 0 && (((uintptr_t)H) & 15) == 0;
    const int nf = B * (U >> 1);
    float4 pf[kPF];
    if (vec && (int)blockIdx.x < p.n_sc) prefetch_issue(pf, H + (size_t)blockIdx.x * B * U, nf);

    for (int n = blockIdx.x; n < p.n_sc; n += gridDim.x) {
    // ---- stage H[n] (zero-padded to UP users) and s[:, n] in LDS ----------
    if (vec)
        prefetch_commit<UP>(pf, H + (size_t)n * B * U, Hs, B, U);
    else
        stage_channel<UP>(H + (size_t)n * B * U, Hs, B, U);
    for (int e = tid; e < K * UP; e += kThreads) {
        const int k = e / UP, u = e % UP;
        const float2 v = (u < U) ? s[((size_t)k * p.n_sc + n) * U + u] : make_float2(0.f, 0.f);
        *(float2 *)(Ss + k * 2 * UP + 2 * u) = v;
    }
    for (int e = tid; e < 8 * SLOT; e += kThreads) slots[e] = {0.f, 0.f};
    __syncthreads();
    // the next subcarrier's channel is in flight while this one computes
    if (vec && n + (int)gridDim.x < p.n_sc) prefetch_issue(pf, H + (size_t)(n + gridDim.x) * B * U, nf);

    if (ARCH == kPD) {
        const float kap = pd_kappa(p);
        // split-K Gram: four contiguous, even-sized row ranges
        const int rows_per = ((B + 7) / 8) * 2;
        const int r0 = min(B, wave * rows_per), r1 = min(B, r0 + rows_per);
        floatx16 acc[NTT];
#pragma unroll
        for (int q = 0; q < NTT; ++q) acc[q] = floatx16{0};
        mfma_gram<UP>(Hs + r0 * RS, RS, r1 - r0, acc);
        gram_store<UP>(acc, sA, 0.f, U, nullptr, nullptr);
        __syncthreads();
        // cluster (partial) sum in fixed order + kappa I, into wave 0's slot A
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
            float t = 0.f;
            const bool ok = wave_factor<UP>(sA, U, kap, &t);
            const float beta = ok ? sqrtf(p.Es / p.power * t) : 0.f;
            if (lane == 0) {
                sh_scale = ok ? 1.f / beta : 0.f;
                sh_ok = ok;
                if (scale_out) scale_out[n] = beta;
                if (status) status[n] = ok ? PRECODE_ST_OK : PRECODE_ST_FAIL;
            }
        }
        __syncthreads();
        const cx<float> *z0 = slots + SLOT;  // wave 0's slot B
        for (int k0 = 0; k0 < K; k0 += KC) {
            const int kc = min(KC, K - k0);
            if (wave == 0) wave_solve_chunk<UP>(sA, sB, Ss, k0, kc, U, sh_scale, sh_ok != 0);
            __syncthreads();
            wave_precode_rows<UP>(Hs, z0, 0, B, k0, kc, n, p.n_sc, B, x, wave, 4);
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
            mfma_gram<UP>(Hs + o * RS, RS, Bc, acc);
            gram_store<UP>(acc, sA, kap, U, nullptr, nullptr);
            wave_sync();
            float t = 0.f;
            const bool ok = wave_factor<UP>(sA, U, kap, &t);
            const float w = ok ? sqrtf(rho_c2 / (t * p.Es)) : 0.f;
            if (lane == 0) {
                if (scale_out) scale_out[(size_t)n * p.C + c] = w;
                if (status) status[(size_t)n * p.C + c] = ok ? PRECODE_ST_OK : PRECODE_ST_FAIL;
            }
            wave_sync();
            for (int k0 = 0; k0 < K; k0 += KC) {
                const int kc = min(KC, K - k0);
                wave_solve_chunk<UP>(sA, sB, Ss, k0, kc, U, w, ok);
                wave_sync();
                wave_precode_rows<UP>(Hs, sB, o, Bc, k0, kc, n, p.n_sc, B, x, 0, 1);
                wave_sync();
            }
        }
    }
    __syncthreads();  // every LDS read of this subcarrier precedes the next staging
    }
}

int pick_up(int U) { return U <= 16 ? 16 : (U <= 32 ? 32 : 0); }

constexpr size_t kLdsMax = 160 * 1024;

template <int UP, int ARCH>
hipError_t launch(const Prob &p, int K, const float2 *H, const float2 *s, float2 *x, float *scale_out,
                  int *status, hipStream_t st) {
    const size_t lds = lds_bytes<UP>(p.B, K);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)fused_k<UP, ARCH>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // persistent grid: as many blocks as fit on the device at once
    static int cached_lds = -1, cached_grid = 0;
    if (cached_lds != (int)lds) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fused_k<UP, ARCH>, kThreads, lds);
        if (e != hipSuccess) return e;
        cached_grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
        cached_lds = (int)lds;
    }
    const int grid = p.n_sc < cached_grid ? p.n_sc : cached_grid;
    hipLaunchKernelGGL((fused_k<UP, ARCH>), dim3(grid), dim3(kThreads), lds, st, p, K, H, s, x, scale_out,
                       status);
    return hipGetLastError();
}

}  // namespace

bool fused_supported(const Prob &p, int precision) {
    if (precision != PRECODE_PREC_FP32) return false;
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

hipError_t fused_run(const Prob &p, int precision, const float2 *H, const float2 *s, float2 *x,
                     float *scale_out, int *status, hipStream_t st) {
    if (!fused_supported(p, precision)) return hipErrorNotSupported;
    if (p.n_sc == 0) return hipSuccess;
    const int up = pick_up(p.U);
    for (int k0 = 0; k0 < p.K; k0 += kMaxKFused) {
        const int kk = p.K - k0 < kMaxKFused ? p.K - k0 : kMaxKFused;
        const float2 *sk = s + (size_t)k0 * p.n_sc * p.U;
        float2 *xk = x + (size_t)k0 * p.n_sc * p.B;
        // factors are identical for every slice; write them once
        float *so = k0 == 0 ? scale_out : nullptr;
        int *sto = k0 == 0 ? status : nullptr;
        hipError_t e;
        if (up == 16)
            e = p.arch == kPD ? launch<16, kPD>(p, kk, H, sk, xk, so, sto, st)
                              : launch<16, kFD>(p, kk, H, sk, xk, so, sto, st);
        else
            e = p.arch == kPD ? launch<32, kPD>(p, kk, H, sk, xk, so, sto, st)
                              : launch<32, kFD>(p, kk, H, sk, xk, so, sto, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pc
