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

constexpr int kUeRows = 32;  // antenna rows staged per step of the receive kernel

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

// One workgroup per subcarrier; thread t owns outputs (u, k) = (o % U, o / U)
// for o = t, t + 256, ...; antenna rows are staged 32 at a time in LDS
// (H rows [32][U], x [K][32]).
__global__ void __launch_bounds__(256) ue_receive_k(const float2 *__restrict__ H, const float2 *__restrict__ x,
                                                   const float2 *__restrict__ noise, float sq_n0,
                                                   const float *__restrict__ scale, int B, int U, int n_sc, int K,
                                                   float2 *__restrict__ y) {
    extern __shared__ float2 smem_ue[];
    float2 *Hs = smem_ue;                 // [32][U]
    float2 *Xs = smem_ue + kUeRows * U;  // [K][32]
    const int n = blockIdx.x, tid = threadIdx.x;
    const float2 *Hn = H + (size_t)n * B * U;
    const float sc = scale ? scale[n] : 1.f;
    for (int o0 = 0; o0 < U * K; o0 += 256) {
        const int o = o0 + tid;
        const int u = o % U, k = o / U;
        float2 acc = make_float2(0.f, 0.f);
        for (int b0 = 0; b0 < B; b0 += kUeRows) {
            const int nb = min(kUeRows, B - b0);
            __syncthreads();
            for (int e = tid; e < nb * U; e += 256) Hs[e] = Hn[(size_t)b0 * U + e];
            for (int e = tid; e < K * kUeRows; e += 256) {
                const int kk = e / kUeRows, bb = e % kUeRows;
                Xs[e] = bb < nb ? x[((size_t)kk * n_sc + n) * B + b0 + bb] : make_float2(0.f, 0.f);
            }
            __syncthreads();
            if (o < U * K)
                for (int bb = 0; bb < nb; ++bb) {
                    const float2 h = Hs[bb * U + u], v = Xs[k * kUeRows + bb];
                    acc = make_float2(fmaf(h.x, v.x, fmaf(h.y, v.y, acc.x)), fmaf(h.x, v.y, fmaf(-h.y, v.x, acc.y)));
                }
        }
        if (o < U * K) {
            const size_t e = ((size_t)k * n_sc + n) * U + u;
            if (noise) {
                const float2 w = noise[e];
                acc = make_float2(fmaf(sq_n0, w.x, acc.x), fmaf(sq_n0, w.y, acc.y));
            }
            y[e] = make_float2(acc.x * sc, acc.y * sc);
        }
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

// Symbols per receive launch: a launch stages [32][U] channel rows and
// [kUeSyms][32] precoded entries in LDS (at most 48 KiB for U <= 64).
constexpr int kUeSyms = 64;

hipError_t ue_receive_run(const float2 *H, const float2 *x, const float2 *noise, float N0, const float *scale, int B,
                          int U, int n_sc, int K, float2 *y, hipStream_t st) {
    if (n_sc == 0 || K == 0) return hipSuccess;
    for (int k0 = 0; k0 < K; k0 += kUeSyms) {
        const int kc = K - k0 < kUeSyms ? K - k0 : kUeSyms;
        const size_t lds = (size_t)(kUeRows * U + kc * kUeRows) * sizeof(float2);
        const size_t xo = (size_t)k0 * n_sc * B, yo = (size_t)k0 * n_sc * U;
        hipLaunchKernelGGL(ue_receive_k, dim3(n_sc), dim3(256), lds, st, H, x + xo, noise ? noise + yo : nullptr,
                           sqrtf(N0), scale, B, U, n_sc, kc, y + yo);
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
