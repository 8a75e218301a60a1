// ue.hip -- the user-equipment side of the uncoded-BER link (Sec. III-D),
// with the downlink model of Sec. II-A and the UE scaling of Sec. II-B.
//
//   qam_map     label l in [0, order) -> unit-energy square QAM point: the
//               upper half of l's bits is the binary-reflected Gray code of
//               the in-phase level, the lower half that of the quadrature
//               level; level i of m = sqrt(order) sits at (2 i - (m - 1)) d,
//               d = sqrt(3 / (2 (order - 1)))
//   receive     s_hat[k][n][u] = scale[n] (sum_b conj(H[n][b][u]) x[k][n][b]
//               + sqrt(N0) w[k][n][u])   (y = H_dl x + n, H_dl = H^H)
//   gain        the UE factor minimizing the MSE of Sec. II-B for the
//               precoder in use, from the noise-free responses to U pilots
//               s = e_v: beta = Es Re(tr E) / (Es ||E||_F^2 + U N0), E = H_dl P
//   errors      nearest-point decision per axis, Gray label, differing bits
//               counted into a 64-bit device counter
#include "common.h"

namespace pc {
namespace {

__device__ __forceinline__ int gray_to_index(int g) {
    int i = g;
    for (int sh = 1; sh < 16; sh <<= 1) i ^= i >> sh;
    return i;
}

__global__ void __launch_bounds__(256) qam_map_k(const int *__restrict__ labels, long long n, int half_bits,
                                                float d, float2 *__restrict__ s) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const int m = 1 << half_bits;
    const int l = labels[e] & ((1 << (2 * half_bits)) - 1);
    const int ir = gray_to_index(l >> half_bits), ii = gray_to_index(l & (m - 1));
    s[e] = make_float2((float)(2 * ir - (m - 1)) * d, (float)(2 * ii - (m - 1)) * d);
}

// One workgroup (256 threads) per subcarrier.  The outputs come in blocks of
// 4 users x 4 symbols (nbu = ceil(U / 4) by nbk = ceil(K / 4) blocks, at most
// 256); thread t takes block t % nblk for the antenna rows t / nblk, + G, ..
// of each staged chunk (G = 256 / nblk row groups), so each row's 4 channel
// entries and 4 precoded entries (8 LDS reads) feed 16 complex
// multiply-adds.  Rows are staged RC at a time: H rows [RC][U + 1] and x
// [K][XS] (XS = 1 mod 4), padded so that a wave's row groups and symbol
// blocks fall in different banks.  The row groups' partial sums are added
// within each wave by shuffles when nblk divides 64 (then per wave through
// LDS), otherwise through LDS per row group.
__host__ __device__ inline int ue_xs(int rc) { return rc + ((1 - rc) & 3); }

__global__ void __launch_bounds__(256) ue_receive_k(const float2 *__restrict__ H, const float2 *__restrict__ x,
                                                   const float2 *__restrict__ noise, float sq_n0,
                                                   const float *__restrict__ scale, int B, int U, int n_sc, int K,
                                                   int RC, float2 *__restrict__ y) {
    extern __shared__ float2 smem_ue[];
    const int HS = U + 1, XS = ue_xs(RC);
    float2 *Hs = smem_ue;            // [RC][HS]
    float2 *Xs = smem_ue + RC * HS;  // [K][XS]
    const int n = blockIdx.x, tid = threadIdx.x;
    const float2 *Hn = H + (size_t)n * B * U;
    const int nbu = (U + 3) >> 2, nbk = (K + 3) >> 2, nblk = nbu * nbk, G = 256 / nblk;
    const int blk = tid % nblk, grp = tid / nblk;
    const int u0 = 4 * (blk % nbu), k0 = 4 * (blk / nbu);
    const int hq = 256 / U, hr = 256 - hq * U;
    float2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = make_float2(0.f, 0.f);
    for (int b0 = 0; b0 < B; b0 += RC) {
        const int nb = min(RC, B - b0);
        __syncthreads();  // the previous chunk is consumed
        // element e = tid + 256 i of the chunk: (row, user) and (symbol, row)
        // stepped without a division per element
        for (int e = tid, r = tid / U, c = tid - (tid / U) * U; e < nb * U; e += 256) {
            Hs[r * HS + c] = Hn[(size_t)b0 * U + e];
            r += hq;
            c += hr;
            if (c >= U) {
                c -= U;
                ++r;
            }
        }
        {
            const int q = 256 / nb, qr = 256 - q * nb;
            for (int e = tid, kk = tid / nb, bb = tid - (tid / nb) * nb; e < K * nb; e += 256) {
                Xs[kk * XS + bb] = x[((size_t)kk * n_sc + n) * B + b0 + bb];
                kk += q;
                bb += qr;
                if (bb >= nb) {
                    bb -= nb;
                    ++kk;
                }
            }
        }
        __syncthreads();
        if (grp < G)
            for (int r = grp; r < nb; r += G) {
                float2 h[4], v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    h[i] = u0 + i < U ? Hs[r * HS + u0 + i] : make_float2(0.f, 0.f);
                    v[i] = k0 + i < K ? Xs[(k0 + i) * XS + r] : make_float2(0.f, 0.f);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c)  // acc += conj(h) v
                        acc[a][c] = make_float2(fmaf(h[a].x, v[c].x, fmaf(h[a].y, v[c].y, acc[a][c].x)),
                                                fmaf(h[a].x, v[c].y, fmaf(-h[a].y, v[c].x, acc[a][c].y)));
            }
    }
    // partial sums [ng][nblk][16] in the staging area
    const bool in_wave = (64 % nblk) == 0;  // then every thread is in a row group
    int ng = G, slot = grp;
    if (in_wave) {
        // lanes l and l ^ nblk ^ 2 nblk .. of a wave hold the same block
        for (int off = nblk; off < 64; off <<= 1)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    acc[a][c].x += __shfl_xor(acc[a][c].x, off);
                    acc[a][c].y += __shfl_xor(acc[a][c].y, off);
                }
        ng = 4;
        slot = (tid & 63) < nblk ? tid >> 6 : ng;  // one lane per block and wave writes
    }
    __syncthreads();  // the staging area becomes the partial sums
    float2 *part = smem_ue;
    if (slot < ng)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) part[(slot * nblk + blk) * 16 + 4 * a + c] = acc[a][c];
    __syncthreads();
    const float sc = scale ? scale[n] : 1.f;
    for (int o = tid; o < U * K; o += 256) {
        const int u = o % U, k = o / U;
        const int ob = (u >> 2) + (k >> 2) * nbu, oi = 4 * (u & 3) + (k & 3);
        float2 t = make_float2(0.f, 0.f);
        for (int g = 0; g < ng; ++g) {
            const float2 v = part[(g * nblk + ob) * 16 + oi];
            t = make_float2(t.x + v.x, t.y + v.y);
        }
        const size_t e = ((size_t)k * n_sc + n) * U + u;
        if (noise) {
            const float2 w = noise[e];
            t = make_float2(fmaf(sq_n0, w.x, t.x), fmaf(sq_n0, w.y, t.y));
        }
        y[e] = make_float2(t.x * sc, t.y * sc);
    }
}

// y_pilot [U][n_sc][U]: response of the U users (last index) to pilot v
// (first index), so E[n][u][v] = y_pilot[v][n][u].
__global__ void __launch_bounds__(256) ue_gain_k(const float2 *__restrict__ yp, float n0, float Es, int U, int n_sc,
                                                float *__restrict__ beta) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= n_sc) return;
    float tr = 0.f, fro = 0.f;
    for (int v = 0; v < U; ++v) {
        const float2 *col = yp + ((size_t)v * n_sc + n) * U;
        tr += col[v].x;
        for (int u = 0; u < U; ++u) fro = fmaf(col[u].x, col[u].x, fmaf(col[u].y, col[u].y, fro));
    }
    beta[n] = Es * tr / (Es * fro + (float)U * n0);
}

__device__ __forceinline__ int axis_code(float v, float inv_d, int m) {
    int i = (int)floorf((v * inv_d + (float)(m - 1)) * 0.5f + 0.5f);
    i = min(max(i, 0), m - 1);
    return i ^ (i >> 1);
}

__global__ void __launch_bounds__(256) qam_errors_k(const float2 *__restrict__ s_hat, const int *__restrict__ labels,
                                                   long long n, int half_bits, float inv_d, int *__restrict__ out,
                                                   unsigned long long *__restrict__ count) {
    __shared__ unsigned red[4];
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    unsigned errs = 0;
    if (e < n) {
        const int m = 1 << half_bits;
        const float2 v = s_hat[e];
        const int l = (axis_code(v.x, inv_d, m) << half_bits) | axis_code(v.y, inv_d, m);
        if (out) out[e] = l;
        errs = (unsigned)__popc((unsigned)(l ^ (labels[e] & ((1 << (2 * half_bits)) - 1))));
    }
    for (int o = 32; o > 0; o >>= 1) errs += __shfl_xor(errs, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = errs;
    __syncthreads();
    if (threadIdx.x == 0 && count) {
        const unsigned long long t = (unsigned long long)red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd(count, t);
    }
}

unsigned grid_of(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

float qam_spacing(int order) { return sqrtf(3.f / (2.f * (float)(order - 1))); }

hipError_t qam_map_run(const int *labels, long long n, int half_bits, float2 *s, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(qam_map_k, dim3(grid_of(n)), dim3(256), 0, st, labels, n, half_bits,
                       qam_spacing(1 << (2 * half_bits)), s);
    return hipGetLastError();
}

// Symbols per receive launch (at most 16 x 16 output blocks of 4 x 4).
constexpr int kUeSyms = 64;

// Rows per staged chunk: the chunk takes at most 16 KiB, so that at 16 users
// and 14 symbols nine workgroups share a CU (a frame's 1200 subcarriers are
// resident together); a multiple of 16 rows, so that each symbol's part of a
// chunk starts on a 128-byte line (66 rows at 256 antennas took 35.8 us per
// frame, 64 rows 33.5 us; 512 antennas / 32 users: 204 and 194 us).
int ue_rows(int B, int U, int K) {
    int rc = 2048 / (U + 1 + K);  // at least 15 (U, K <= 64)
    rc = rc > 128 ? 128 : rc >= 16 ? rc / 16 * 16 : rc;
    return rc < B ? rc : B;
}

hipError_t ue_receive_run(const float2 *H, const float2 *x, const float2 *noise, float N0, const float *scale, int B,
                          int U, int n_sc, int K, float2 *y, hipStream_t st) {
    if (n_sc == 0 || K == 0) return hipSuccess;
    for (int k0 = 0; k0 < K; k0 += kUeSyms) {
        const int kc = K - k0 < kUeSyms ? K - k0 : kUeSyms;
        const int rc = ue_rows(B, U, kc);
        const size_t nblk = (size_t)((U + 3) / 4) * ((kc + 3) / 4);
        const size_t stage = (size_t)rc * (U + 1) + (size_t)kc * ue_xs(rc);
        const size_t part = (64 % nblk == 0 ? 4 : 256 / nblk) * nblk * 16;
        const size_t lds = (stage > part ? stage : part) * sizeof(float2);
        const size_t xo = (size_t)k0 * n_sc * B, yo = (size_t)k0 * n_sc * U;
        hipLaunchKernelGGL(ue_receive_k, dim3(n_sc), dim3(256), lds, st, H, x + xo, noise ? noise + yo : nullptr,
                           sqrtf(N0), scale, B, U, n_sc, kc, rc, y + yo);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t ue_gain_run(const float2 *y_pilot, float N0, float Es, int U, int n_sc, float *beta, hipStream_t st) {
    if (n_sc == 0) return hipSuccess;
    hipLaunchKernelGGL(ue_gain_k, dim3(grid_of(n_sc)), dim3(256), 0, st, y_pilot, N0, Es, U, n_sc, beta);
    return hipGetLastError();
}

hipError_t qam_errors_run(const float2 *s_hat, const int *labels, long long n, int half_bits, int *out,
                          unsigned long long *count, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(qam_errors_k, dim3(grid_of(n)), dim3(256), 0, st, s_hat, labels, n, half_bits,
                       1.f / qam_spacing(1 << (2 * half_bits)), out, count);
    return hipGetLastError();
}

}  // namespace pc
