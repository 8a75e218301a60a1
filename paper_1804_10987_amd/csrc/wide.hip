// wide.hip -- local systems of order up to 64 in one fused FP64 launch: the
// systems the register-tile kernels do not take (U in 33..64, FD clusters with
// B_c < U, FP64-route systems past the one-wave FP64 kernel's bounds, calls at
// precision FP64).
//
// One workgroup of 256 threads per local system (a PD subcarrier, or an FD
// (subcarrier, cluster) pair), everything in FP64 (complex64 inputs widened
// exactly).  A system of order N <= NP (NP = 16, 32, 48 or 64) is held as an NP x NP
// matrix that is the identity past N; thread t = 16 bi + bj owns the E x E
// block (E = NP / 16) at rows E bi .. E bi + E - 1, columns E bj .. .
//
//   form      U x U (PD, and FD clusters with B_c >= U):
//               A = sum over the system's rows of h_r^H h_r + kappa I
//             B_c x B_c (FD clusters with B_c < U, Sec. III-C's case split):
//               M_c = H_c H_c^H + kappa_c I, the same sum over the rows of
//               H_c^H, which are staged once (conjugated, transposed)
//   Gram      the contraction rows staged 64 at a time in LDS (coalesced
//             loads of the system's contiguous rows, the next chunk in flight
//             while the current one is multiplied); the 16 x 16 blocks on and
//             above the block diagonal on FP64 MFMA, each wave over a quarter
//             of the rows, the partial sums added in LDS in wave order;
//             complex64 products are exact in FP64
//   invert    Gauss-Jordan without pivoting (Hermitian positive definite) on
//             2^-e A, the largest diagonal entry in [0.5, 1), one barrier per
//             step: the owners of row k write it to LDS.  Before step k the
//             matrix is [[A11^-1, A11^-1 A12], [-A21 A11^-1, S]], so column k
//             is row k conjugated and negated above the diagonal
//   factor    t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1); PD beta =
//             sqrt(Es t / rho^2), FD w_c = sqrt(rho_c^2 / (t Es)) (Sec. III-C)
//   solve     A^-1 to LDS; per chunk of 16 symbols z = scale A^-1 v with
//             v = s (U x U form) or v = H_c s (B_c x B_c form, where
//             x_c = w_c M_c^-1 H_c s is the output)
//   precode   U x U form: x_c = H_c z, rows staged again 64 at a time
//             (transposed), accumulated in FP64
//
// Status of every system: PRECODE_ST_FP64, plus PRECODE_ST_FAIL when a pivot
// is not above kRelPivot64 times its original diagonal entry or t is not
// positive (then x = 0 and the scale output is 0).
//
// Modes: the whole chain in one launch; or a prepare launch that stores
// scale A^-1 (FP64, an NP x NP slot per system) with beta / weights and
// status, and symbol launches that precode released symbols from it (the
// B_c x B_c form stages H_c^H again, the U x U form its rows) -- the frame
// API and serving.
#include "common.h"

#include <algorithm>

namespace pc {
namespace {

constexpr int kWT = 256;  // threads per workgroup
constexpr int kWSR = 64;  // rows staged per chunk
// modes: Gram to precode; Gram to the factors scale A^-1 (FP64, an NP x NP
// slot per system) with beta / weights and status; precode from the factors
enum { kWFull = 0, kWPrep = 1, kWSym = 2 };

template <int NP>
struct WideL {
    // symbols per chunk: 8 at order 48, so that its LDS (72.8 KiB) lets two
    // workgroups share a CU; 16 otherwise
    static constexpr int KC = NP == 48 ? 8 : 16;
    static constexpr int E = NP / 16;   // edge of a thread's block
    static constexpr int G = kWT / NP;  // symbol groups of the solve (threads past G NP idle there)
    static constexpr int PER = kWSR * NP / kWT;  // staged elements per thread
    // staged rows: [64][NP] complex64 (Gram), [NP][65] (transposed precode rows)
    static constexpr size_t stage_b = (size_t)NP * (kWSR + 1) * 8;
    static constexpr size_t ainv_b = (size_t)NP * NP * 16;   // A^-1 [NP][NP] (row buffers while inverting)
    static constexpr size_t vb_b = (size_t)KC * NP * 16;   // right-hand sides [KC][NP]
    // Z chunk [KC][NP] (complex FP64) or symbols [KC][64] (complex64)
    static constexpr size_t zb_b = (size_t)KC * (NP * 16 > 64 * 8 ? NP * 16 : 64 * 8);
    static constexpr size_t o_ainv = stage_b, o_vb = o_ainv + ainv_b, o_zb = o_vb + vb_b, o_dg = o_zb + zb_b;
    static constexpr size_t bytes = o_dg + (size_t)(NP + 8) * 8;  // + diagonal, reduction slots
};

__device__ __forceinline__ double rcp_nr(double v) {
    double inv = __builtin_amdgcn_rcp(v);
    inv = fma(inv, fma(-v, inv, 1.0), inv);
    return fma(inv, fma(-v, inv, 1.0), inv);
}

typedef double wf64x4 __attribute__((ext_vector_type(4)));
// x is written once and never read back by the launch: non-temporal stores.
typedef float wfloat2 __attribute__((ext_vector_type(2)));

template <int NP>
__device__ __forceinline__ void wide_system(const Prob *__restrict__ pk, int sys, int K, int mode,
                                            const float2 *__restrict__ H, const float2 *__restrict__ s,
                                            float2 *__restrict__ x, float *__restrict__ scale_out,
                                            int *__restrict__ status, cx<double> *__restrict__ fac, char *lds) {
    constexpr int E = WideL<NP>::E, G = WideL<NP>::G, PER = WideL<NP>::PER, KC = WideL<NP>::KC, SR = kWSR;
    constexpr int MS = (KC + G - 1) / G;  // symbols per thread in the solve: sg + G m < KC
    const int tid = threadIdx.x, bi = tid >> 4, bj = tid & 15;
    const bool pd = pk->arch == kPD;
    const int B = pk->B, U = pk->U, C = pk->C, n_sc = pk->n_sc;
    const int n = pd ? sys : sys / C, cl = pd ? 0 : sys - n * C;
    const int r0 = pd ? 0 : pk->off[cl];
    const int nrows = (pd ? B : pk->off[cl + 1]) - r0;
    const bool bform = !pd && nrows < U;
    const int N = bform ? nrows : U;
    const double kap = pd ? (double)pd_kappa(*pk) : (double)fd_kappa_c(pk, cl);
    const float2 *Hs = H + ((size_t)n * B + r0) * U;  // the system's rows, contiguous
    float2 *st = (float2 *)lds;
    cx<double> *ainv = (cx<double> *)(lds + WideL<NP>::o_ainv);
    cx<double> *vb = (cx<double> *)(lds + WideL<NP>::o_vb);
    cx<double> *zb = (cx<double> *)(lds + WideL<NP>::o_zb);
    float2 *sy = (float2 *)(lds + WideL<NP>::o_zb);
    double *dg = (double *)(lds + WideL<NP>::o_dg);
    double *red = dg + NP;

    // ---- Gram: G[i][j] = sum_r conj(X[r][i]) X[r][j] over the staged rows X,
    // its 16 x 16 blocks (I, J), I <= J, on FP64 MFMA (v_mfma_f64_16x16x4f64):
    // lane l feeds X[r0 + l / 16][16 I + l % 16] as A[i][k] and
    // X[r0 + l / 16][16 J + l % 16] as B[k][j] (k: the row of the step);
    // D[i][j] lands in lane (i % 4) 16 + j, register i / 4.  Wave w takes
    // rows 16 w .. 16 w + 15 of each staged chunk.
    constexpr int NB = NP / 16, NBLK = NB * (NB + 1) / 2;
    const int lane = tid & 63, wave = tid >> 6;
    wf64x4 are[NBLK], aim[NBLK];
#pragma unroll
    for (int t = 0; t < NBLK; ++t) are[t] = aim[t] = (wf64x4){0.0, 0.0, 0.0, 0.0};
    {
        // staged columns past the system's order stay zero, and so do the
        // B_c x B_c form's rows past U
        const int c0 = bform ? nrows : U, nz = NP - c0;
        if (nz > 0)
            for (int e = tid; e < SR * nz; e += kWT) st[(e / nz) * NP + c0 + e % nz] = make_float2(0.f, 0.f);
        if (bform && nrows > 0)
            for (int e = tid; e < (SR - U) * nrows; e += kWT) st[(U + e / nrows) * NP + e % nrows] = make_float2(0.f, 0.f);
    }
    if (bform) {
        // X[u][i] = conj(H_c[i][u]): the whole cluster (nrows x U <= 64 x 64)
        const int ne = nrows * U;
        float2 v[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = tid + kWT * m;
            v[m] = e < ne ? Hs[e] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = tid + kWT * m;
            if (e < ne) st[(e % U) * NP + e / U] = make_float2(v[m].x, -v[m].y);
        }
    }
    bool ok = true;
    double scale = 1.0;
    float2 pre[PER];
    if (mode != kWSym) {
    const int nch = bform ? 1 : (nrows + SR - 1) / SR;
    if (!bform) {
        const int ne = min(SR, nrows) * U;
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = tid + kWT * m;
            pre[m] = e < ne ? Hs[e] : make_float2(0.f, 0.f);
        }
    }
    for (int q = 0; q < nch; ++q) {
        const int nr = bform ? U : min(SR, nrows - q * SR);
        if (!bform) {
            // rows nr..SR-1 of a short chunk are written as zeros
#pragma unroll
            for (int m = 0; m < PER; ++m) {
                const int e = tid + kWT * m;
                if (e < SR * U) st[(e / U) * NP + e % U] = e < nr * U ? pre[m] : make_float2(0.f, 0.f);
            }
        }
        __syncthreads();
        if (!bform && q + 1 < nch) {
            const float2 *src = Hs + (size_t)(q + 1) * SR * U;
            const int ne = min(SR, nrows - (q + 1) * SR) * U;
#pragma unroll
            for (int m = 0; m < PER; ++m) {
                const int e = tid + kWT * m;
                pre[m] = e < ne ? src[e] : make_float2(0.f, 0.f);
            }
        }
        // rows past nr in a step are zero
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
            const int rb4 = 16 * wave + 4 * qd;
            if (rb4 >= nr) break;  // wave-uniform: every lane stays active for the MFMA
            const float2 *row = st + (rb4 + (lane >> 4)) * NP + (lane & 15);
            double hr[NB], hi[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float2 v = row[16 * b];
                hr[b] = v.x;
                hi[b] = v.y;
            }
            int t = 0;
#pragma unroll
            for (int I = 0; I < NB; ++I)
#pragma unroll
                for (int J = I; J < NB; ++J, ++t) {
                    are[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(hr[I], hr[J], are[t], 0, 0, 0);
                    are[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(hi[I], hi[J], are[t], 0, 0, 0);
                    aim[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(hr[I], hi[J], aim[t], 0, 0, 0);
                    aim[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-hi[I], hr[J], aim[t], 0, 0, 0);
                }
        }
        __syncthreads();  // the staging area is rewritten by the next chunk
    }
    // the four waves' partial blocks summed in wave order into G (the A^-1
    // area), then each thread takes its E x E block (below the block
    // diagonal from the conjugate of the block above it)
    cx<double> *Gm = ainv;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
            int t = 0;
#pragma unroll
            for (int I = 0; I < NB; ++I)
#pragma unroll
                for (int J = I; J < NB; ++J, ++t)
#pragma unroll
                    for (int rg = 0; rg < 4; ++rg) {
                        cx<double> &g = Gm[(16 * I + 4 * rg + (lane >> 4)) * NP + 16 * J + (lane & 15)];
                        if (w == 0) {
                            g = {are[t][rg], aim[t][rg]};
                        } else {
                            g.re += are[t][rg];
                            g.im += aim[t][rg];
                        }
                    }
        }
        __syncthreads();
    }
    double gr[E][E], gi[E][E];
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) {
            const int i = E * bi + a, j = E * bj + b;
            if ((i >> 4) <= (j >> 4)) {
                const cx<double> g = Gm[i * NP + j];
                gr[a][b] = g.re;
                gi[a][b] = g.im;
            } else {
                const cx<double> g = Gm[j * NP + i];
                gr[a][b] = g.re;
                gi[a][b] = -g.im;
            }
        }

    // ---- A = G + kappa I, identity past N; 2^-e scaling
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) {
            const int i = E * bi + a, j = E * bj + b;
            if (i >= N || j >= N) {
                gr[a][b] = i == j ? 1.0 : 0.0;
                gi[a][b] = 0.0;
            } else if (i == j) {
                gr[a][b] += kap;
                gi[a][b] = 0.0;
            }
        }
    if (bi == bj)
#pragma unroll
        for (int a = 0; a < E; ++a) dg[E * bi + a] = gr[a][a];
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < N; ++i) dmax = fmax(dmax, dg[i]);
    int ex = 0;
    if (dmax > 0.0 && dmax < (double)INFINITY) ex = ilogb(dmax) + 1;
    const double sc = ldexp(1.0, -ex);
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b)
            if (E * bi + a < N && E * bj + b < N) {
                gr[a][b] *= sc;
                gi[a][b] *= sc;
            }

    // ---- Gauss-Jordan, steps k < N (the identity past N is its own inverse)
    cx<double> *rb = ainv;  // two row buffers [2][NP]
    for (int k = 0; k < N; ++k) {
        cx<double> *buf = rb + (k & 1) * NP;
        if (bi == k / E) {
            const int ak = k - E * bi;
#pragma unroll
            for (int a = 0; a < E; ++a)
                if (a == ak)
#pragma unroll
                    for (int b = 0; b < E; ++b) buf[E * bj + b] = {gr[a][b], gi[a][b]};
        }
        __syncthreads();
        const double piv = buf[k].re;
        const double inv = rcp_nr(piv);
        ok = ok && piv > kRelPivot64 * (dg[k] * sc) && piv < (double)INFINITY;
        cx<double> rj[E], ri[E];
#pragma unroll
        for (int b = 0; b < E; ++b) rj[b] = buf[E * bj + b];
#pragma unroll
        for (int a = 0; a < E; ++a) ri[a] = buf[E * bi + a];
#pragma unroll
        for (int a = 0; a < E; ++a) {
            const int i = E * bi + a;
            // column k at row i: conj(a_ki), negated for i < k
            const double sg = i < k ? -1.0 : 1.0;
            const double akr = sg * ri[a].re, aki = -sg * ri[a].im;
#pragma unroll
            for (int b = 0; b < E; ++b) {
                const bool iscol = E * bj + b == k;
                // multiplier a_kj / a_kk; 1 + 1 / a_kk in column k turns it into -a_ik / a_kk
                const double mr = iscol ? 1.0 + inv : rj[b].re * inv;
                const double mi = iscol ? 0.0 : rj[b].im * inv;
                const double xr = fma(-akr, mr, fma(aki, mi, gr[a][b]));
                const double xi = fma(-akr, mi, fma(-aki, mr, gi[a][b]));
                if (i == k) {
                    gr[a][b] = iscol ? inv : mr;
                    gi[a][b] = mi;
                } else {
                    gr[a][b] = xr;
                    gi[a][b] = xi;
                }
            }
        }
        // no second barrier: the next step writes the other buffer
    }

    // ---- Lemma 1 on A^-1 = 2^-e (2^-e A)^-1
    double tr = 0.0, fro = 0.0;
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) {
            const int i = E * bi + a, j = E * bj + b;
            if (i < N && j < N) {
                gr[a][b] *= sc;
                gi[a][b] *= sc;
                fro += gr[a][b] * gr[a][b] + gi[a][b] * gi[a][b];
                if (i == j) tr += gr[a][b];
            }
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tr += __shfl_xor(tr, o);
        fro += __shfl_xor(fro, o);
    }
    if ((tid & 63) == 0) {
        red[tid >> 6] = tr;
        red[4 + (tid >> 6)] = fro;
    }
    __syncthreads();  // also ends every read of the row buffers
    tr = red[0] + red[1] + red[2] + red[3];
    fro = red[4] + red[5] + red[6] + red[7];
    const double t = tr - kap * fro;
    ok = ok && t > 0.0 && t < (double)INFINITY;
    double out = 0.0;
    scale = 0.0;
    if (ok) {
        if (pd) {
            out = sqrt((double)pk->Es / (double)pk->power * t);  // beta
            scale = 1.0 / out;
        } else {
            out = sqrt(fd_power_c_d(pk, cl) / (t * (double)pk->Es));  // w_c
            scale = out;
        }
    }
    if (tid == 0) {
        if (scale_out) scale_out[sys] = (float)out;
        if (status) status[sys] = (ok ? PRECODE_ST_OK : PRECODE_ST_FAIL) | PRECODE_ST_FP64;
    }
    if (mode == kWPrep) {
        // scale A^-1 to the system's slot for the symbol passes
        cx<double> *f = fac + (size_t)sys * NP * NP;
#pragma unroll
        for (int a = 0; a < E; ++a)
#pragma unroll
            for (int b = 0; b < E; ++b)
                f[(E * bi + a) * NP + E * bj + b] = {ok ? scale * gr[a][b] : 0.0, ok ? scale * gi[a][b] : 0.0};
        return;
    }
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) ainv[(E * bi + a) * NP + E * bj + b] = {gr[a][b], gi[a][b]};
    } else {
        // a symbol pass: scale A^-1 and the status from the prepare pass
        const cx<double> *f = fac + (size_t)sys * NP * NP;
        for (int e = tid; e < NP * NP; e += kWT) ainv[e] = f[e];
        ok = !status || !(status[sys] & PRECODE_ST_FAIL);
        scale = 1.0;
    }

    // ---- symbols, KC at a time
    // solve: system row si, symbol group sg (symbols sg + G m < KC; threads
    // past G NP take none)
    const int si = tid % NP, sg = tid / NP;
    bool kv[MS];
    int kr[MS];
#pragma unroll
    for (int m = 0; m < MS; ++m) {
        kv[m] = sg < G && sg + G * m < KC;
        kr[m] = kv[m] ? sg + G * m : 0;
    }
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kc = min(KC, K - k0);
        if (!bform) {
            for (int e = tid; e < KC * NP; e += kWT) {
                const int k = e / NP, j = e % NP;
                const float2 v = k < kc && j < U ? s[((size_t)(k0 + k) * n_sc + n) * U + j] : make_float2(0.f, 0.f);
                vb[e] = {(double)v.x, (double)v.y};
            }
        } else {
            for (int e = tid; e < KC * 64; e += kWT) {
                const int k = e >> 6, u = e & 63;
                sy[e] = k < kc && u < U ? s[((size_t)(k0 + k) * n_sc + n) * U + u] : make_float2(0.f, 0.f);
            }
            __syncthreads();
            // v[k][i] = sum_u H_c[i][u] s_k[u], H_c[i][u] = conj(X[u][i])
            double vr[MS], vi[MS];
#pragma unroll
            for (int m = 0; m < MS; ++m) vr[m] = vi[m] = 0.0;
            for (int u = 0; u < U; ++u) {
                const float2 h = st[u * NP + si];
                const double hr = h.x, hm = -h.y;
#pragma unroll
                for (int m = 0; m < MS; ++m) {
                    const float2 sv = sy[kr[m] * 64 + u];
                    vr[m] = fma(hr, (double)sv.x, fma(-hm, (double)sv.y, vr[m]));
                    vi[m] = fma(hr, (double)sv.y, fma(hm, (double)sv.x, vi[m]));
                }
            }
#pragma unroll
            for (int m = 0; m < MS; ++m)
                if (kv[m]) vb[kr[m] * NP + si] = {vr[m], vi[m]};
        }
        __syncthreads();
        // z[k][i] = scale sum_j conj(A^-1[j][i]) v[k][j]  (A^-1 Hermitian)
        {
            double zr[MS], zi[MS];
#pragma unroll
            for (int m = 0; m < MS; ++m) zr[m] = zi[m] = 0.0;
            for (int j = 0; j < N; ++j) {
                const cx<double> a = ainv[j * NP + si];
#pragma unroll
                for (int m = 0; m < MS; ++m) {
                    const cx<double> v = vb[kr[m] * NP + j];
                    zr[m] = fma(a.re, v.re, fma(a.im, v.im, zr[m]));
                    zi[m] = fma(a.re, v.im, fma(-a.im, v.re, zi[m]));
                }
            }
#pragma unroll
            for (int m = 0; m < MS; ++m) {
                if (!kv[m]) continue;
                const int k = kr[m];
                const bool live = ok && si < N && k < kc;
                const double a = live ? scale * zr[m] : 0.0, b = live ? scale * zi[m] : 0.0;
                if (!bform)
                    zb[k * NP + si] = {a, b};
                else if (si < N && k < kc)
                    __builtin_nontemporal_store((wfloat2){(float)a, (float)b},
                                                (wfloat2 *)(x + ((size_t)(k0 + k) * n_sc + n) * B + r0 + si));
            }
        }
        if (!bform) {
            // x_c = H_c z, rows 64 at a time staged as [user][row]; thread (row
            // r, group g) takes symbols g, g + 4, ..
            constexpr int XS = KC / 4;
            const int r = tid & 63, g = tid >> 6;
            const int nrc = (nrows + 63) / 64;
            {
                const int ne = min(64, nrows) * U;
#pragma unroll
                for (int m = 0; m < PER; ++m) {
                    const int e = tid + kWT * m;
                    pre[m] = e < ne ? Hs[e] : make_float2(0.f, 0.f);
                }
            }
            __syncthreads();  // Z complete
            for (int c = 0; c < nrc; ++c) {
                const int nr = min(64, nrows - 64 * c);
#pragma unroll
                for (int m = 0; m < PER; ++m) {
                    const int e = tid + kWT * m;
                    if (e < nr * U) st[(e % U) * (kWSR + 1) + e / U] = pre[m];
                }
                __syncthreads();
                if (c + 1 < nrc) {
                    const float2 *src = Hs + (size_t)(c + 1) * 64 * U;
                    const int ne = min(64, nrows - 64 * (c + 1)) * U;
#pragma unroll
                    for (int m = 0; m < PER; ++m) {
                        const int e = tid + kWT * m;
                        pre[m] = e < ne ? src[e] : make_float2(0.f, 0.f);
                    }
                }
                double xr[XS], xi[XS];
#pragma unroll
                for (int m = 0; m < XS; ++m) xr[m] = xi[m] = 0.0;
                for (int i = 0; i < U; ++i) {
                    const float2 h = st[i * (kWSR + 1) + r];
                    const double hr = h.x, hm = h.y;
#pragma unroll
                    for (int m = 0; m < XS; ++m) {
                        const cx<double> z = zb[(g + 4 * m) * NP + i];
                        xr[m] = fma(hr, z.re, fma(-hm, z.im, xr[m]));
                        xi[m] = fma(hr, z.im, fma(hm, z.re, xi[m]));
                    }
                }
                if (r < nr)
#pragma unroll
                    for (int m = 0; m < XS; ++m) {
                        const int k = g + 4 * m;
                        if (k < kc)
                            __builtin_nontemporal_store(
                                (wfloat2){(float)xr[m], (float)xi[m]},
                                (wfloat2 *)(x + ((size_t)(k0 + k) * n_sc + n) * B + r0 + 64 * c + r));
                    }
                __syncthreads();  // the staging area is rewritten by the next chunk
            }
        }
        __syncthreads();  // the chunk buffers are rewritten by the next chunk
    }
}

template <int NP>
constexpr int wide_min_waves() { return NP == 16 ? 4 : (NP == 32 || NP == 48 ? 2 : 1); }

template <int NP>
__global__ void __launch_bounds__(kWT, (wide_min_waves<NP>()))
    wide_k(Prob p, int K, int mode, const float2 *__restrict__ H, const float2 *__restrict__ s,
           float2 *__restrict__ x, float *__restrict__ scale_out, int *__restrict__ status,
           cx<double> *__restrict__ fac) {
    extern __shared__ float4 smem_wide[];
    const Prob *pk = (const Prob *)__builtin_amdgcn_kernarg_segment_ptr();  // p: the first argument
    (void)p;
    wide_system<NP>(pk, blockIdx.x, K, mode, H, s, x, scale_out, status, fac, (char *)smem_wide);
}

template <int NP>
__global__ void __launch_bounds__(kWT, (wide_min_waves<NP>()))
    wide_batch_k(const BatchEntry *__restrict__ tab, int n) {
    extern __shared__ float4 smem_wide[];
    const int b = blockIdx.x;
    int lo = 0, hi = n - 1;  // last problem with block0 <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const BatchEntry &en = tab[lo];
    // an entry holds every system of its problem, or (cl >= 0) cluster cl of every subcarrier
    const int lb = b - en.block0;
    const int sys = en.cl < 0 ? lb : lb * en.p.C + en.cl;
    wide_system<NP>(&en.p, sys, en.K, kWFull, en.H, en.s, en.x, en.scale_out, en.status, nullptr, (char *)smem_wide);
}

template <typename F>
hipError_t set_lds(F fn, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int NP>
hipError_t launch_wide(const Prob &p, int K, int mode, const float2 *H, const float2 *s, float2 *x, float *scale_out,
                       int *status, cx<double> *fac, hipStream_t st) {
    const size_t lds = WideL<NP>::bytes;
    hipError_t e = set_lds(wide_k<NP>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((wide_k<NP>), dim3((unsigned)n_inst(p)), dim3(kWT), lds, st, p, K, mode, H, s, x, scale_out,
                       status, fac);
    return hipGetLastError();
}

hipError_t wide_dispatch(const Prob &p, int K, int mode, const float2 *H, const float2 *s, float2 *x,
                         float *scale_out, int *status, cx<double> *fac, hipStream_t st) {
    if (n_inst(p) == 0) return hipSuccess;
    switch (wide_order(p)) {
        case 16: return launch_wide<16>(p, K, mode, H, s, x, scale_out, status, fac, st);
        case 32: return launch_wide<32>(p, K, mode, H, s, x, scale_out, status, fac, st);
        case 48: return launch_wide<48>(p, K, mode, H, s, x, scale_out, status, fac, st);
        default: return launch_wide<64>(p, K, mode, H, s, x, scale_out, status, fac, st);
    }
}

template <int NP>
hipError_t launch_wide_batch(const BatchEntry *tab, int n, int blocks, hipStream_t st) {
    const size_t lds = WideL<NP>::bytes;
    hipError_t e = set_lds(wide_batch_k<NP>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((wide_batch_k<NP>), dim3((unsigned)blocks), dim3(kWT), lds, st, tab, n);
    return hipGetLastError();
}

}  // namespace

bool wide_supported(const Prob &p, int K) { return K >= 1 && p.U >= 1 && p.U <= 64 && n_inst(p) > 0; }

int wide_class(int n) { return n <= 16 ? 16 : (n <= 32 ? 32 : (n <= 48 ? 48 : 64)); }

int wide_cluster_order(const Prob &p, int c) {
    if (p.arch == kPD) return wide_class(p.U);
    const int bc = p.off[c + 1] - p.off[c];
    return wide_class(bc < p.U ? bc : p.U);
}

int wide_order(const Prob &p) {
    int m = 0;
    for (int c = 0; c < (p.arch == kPD ? 1 : p.C); ++c) m = std::max(m, wide_cluster_order(p, c));
    return m;
}

hipError_t wide_run(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *scale_out, int *status,
                    hipStream_t st) {
    return wide_dispatch(p, p.K, kWFull, H, s, x, scale_out, status, nullptr, st);
}

size_t wide_factor_bytes(const Prob &p) {
    const size_t np = (size_t)wide_order(p);
    return (size_t)n_inst(p) * np * np * sizeof(cx<double>);
}

hipError_t wide_prepare(const Prob &p, const float2 *H, void *fac, float *scale_out, int *status, hipStream_t st) {
    return wide_dispatch(p, 0, kWPrep, H, nullptr, nullptr, scale_out, status, (cx<double> *)fac, st);
}

hipError_t wide_symbols(const Prob &p, int nk, const float2 *H, const void *fac, const int *status, const float2 *s,
                        float2 *x, hipStream_t st) {
    if (nk == 0) return hipSuccess;
    return wide_dispatch(p, nk, kWSym, H, s, x, nullptr, (int *)status, (cx<double> *)fac, st);
}

hipError_t wide_batch_launch(int order, const BatchEntry *tab, int n, int blocks, hipStream_t st) {
    if (n == 0 || blocks == 0) return hipSuccess;
    switch (order) {
        case 16: return launch_wide_batch<16>(tab, n, blocks, st);
        case 32: return launch_wide_batch<32>(tab, n, blocks, st);
        case 48: return launch_wide_batch<48>(tab, n, blocks, st);
        default: return launch_wide_batch<64>(tab, n, blocks, st);
    }
}

}  // namespace pc
