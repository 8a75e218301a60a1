// compare.hip -- the comparison precoders of the paper's evaluation (Sec. III-D):
// centralized WF in the B x B form of Theorem 1 and maximum ratio transmission.
//
// Centralized WF, one workgroup (4 waves) per subcarrier, FP32.  With this
// library's H = H_dl^H (B x U):
//
//   M    = H H^H + kappa I_B           (eq. originalQmatrix: B x B, Hermitian PD)
//   M    = L L^H                       tiled left-looking Cholesky, 32 x 32 tiles
//   Q    = L^-H L^-1 H                 forward / back substitution by tile rows
//   beta = sqrt(tr(Q^H Q) Es / rho^2)  (eq. precodingfactor)
//   x_k  = Q s_k / beta
//
// The matrix is padded to Bp = 32 T rows with an identity block (decoupled,
// so the result is unchanged).  Per subcarrier a workspace holds the
// off-diagonal tiles of L and the inverses of the diagonal tiles; Y = L^-1 H
// and then Q (Bp x U) stay in LDS.  Per tile column j the waves form the
// tiles of column j (H_i H_j^H - sum_{l<j} L_il L_jl^H), wave 0 factors the
// diagonal tile and inverts its factor, and the waves multiply the tiles
// below by that inverse (the triangular solve as a product) while one wave
// advances the forward substitution by one tile row.
//
// MRT is in mrt.hip.
#include <algorithm>

#include "common.h"

namespace pc {
namespace {

constexpr int TE = 32;          // tile edge
constexpr int TC = TE * TE;     // complex entries per tile
constexpr int kCenWaves = 4;
constexpr int kCenThreads = 64 * kCenWaves;
constexpr size_t kCenMaxLds = 160 * 1024;

struct Cen {
    int B, U, n_sc, K, T;  // T tiles per dimension (Bp = 32 T)
    int n0;                // first subcarrier of the launch
    float kappa, Es, power;
};

__device__ __forceinline__ int lane_of() { return threadIdx.x & 63; }

__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc + a b, acc + a conj(b), acc - a conj(b)
__device__ __forceinline__ float2 mac(float2 acc, float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
__device__ __forceinline__ float2 macc(float2 acc, float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x)), fmaf(a.y, b.x, fmaf(-a.x, b.y, acc.y)));
}
__device__ __forceinline__ float2 msc(float2 acc, float2 a, float2 b) {
    return make_float2(fmaf(-a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(-a.y, b.x, fmaf(a.x, b.y, acc.y)));
}
// acc - a b
__device__ __forceinline__ float2 msub(float2 acc, float2 a, float2 b) {
    return make_float2(fmaf(-a.x, b.x, fmaf(a.y, b.y, acc.x)), fmaf(-a.x, b.y, fmaf(-a.y, b.x, acc.y)));
}
// acc + conj(a) b, acc - conj(a) b
__device__ __forceinline__ float2 cmac(float2 acc, float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(-a.y, b.x, acc.y)));
}
__device__ __forceinline__ float2 cmsub(float2 acc, float2 a, float2 b) {
    return make_float2(fmaf(-a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(-a.x, b.y, fmaf(a.y, b.x, acc.y)));
}

// Workspace tiles of one subcarrier: off-diagonal L_ij (i > j) at
// i (i - 1) / 2 + j, then the T inverse diagonal tiles L_jj^-1; row-major.
__host__ __device__ __forceinline__ size_t off_tile(int i, int j) { return (size_t)(i * (i - 1) / 2 + j) * TC; }
__host__ __device__ __forceinline__ size_t inv_tile(int T, int j) { return (size_t)(T * (T - 1) / 2 + j) * TC; }
__host__ __device__ __forceinline__ size_t cen_ws_per_sc(int T) { return (size_t)(T * (T + 1) / 2) * TC * sizeof(float2); }

// LDS of the central kernel: Y / Q [Bp][U + 1] (padded rows against bank
// conflicts), the diagonal tile and its inverse [32][32], the solve's
// staging tile row [32][U + 1], the original diagonal, the reduction.
struct CenLds {
    int ys;  // row stride of Y and R (complex)
    size_t y, d, dinv, r, dorig, red, bytes;
    __host__ __device__ CenLds(int T, int U) {
        ys = U + 1;
        y = 0;
        d = y + (size_t)TE * T * ys * sizeof(float2);
        dinv = d + TC * sizeof(float2);
        r = dinv + TC * sizeof(float2);
        dorig = r + (size_t)TE * ys * sizeof(float2);
        red = dorig + TE * sizeof(float);
        bytes = red + 8 * sizeof(float);
    }
};

// One 32 x 32 tile of the left-looking step, wave-local: lane (lr, lc) holds
// rows 4 lr + q, columns 4 lc + t of  H_i H_j^H (+ the diagonal of M on tile
// (j, j)) - sum_{l<j} L_il L_jl^H.
__device__ void tile_column_entry(const Cen &c, const float2 *__restrict__ Hn, const float2 *ws, int i, int j,
                                  float2 (&acc)[4][4], float *dorig_lds) {
    const int lane = lane_of();
    const int lr = lane >> 3, lc = lane & 7;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[q][t] = make_float2(0.f, 0.f);
    for (int u = 0; u < c.U; ++u) {
        float2 a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = TE * i + 4 * lr + q;
            a[q] = r < c.B ? Hn[(size_t)r * c.U + u] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int r = TE * j + 4 * lc + t;
            b[t] = r < c.B ? Hn[(size_t)r * c.U + u] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[q][t] = macc(acc[q][t], a[q], b[t]);
    }
    if (i == j) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (4 * lr + q == 4 * lc + t) {
                    const int r = TE * i + 4 * lr + q;
                    acc[q][t].x += r < c.B ? c.kappa : 1.f;  // padded rows: identity block
                    dorig_lds[4 * lr + q] = acc[q][t].x;
                }
    }
    for (int l = 0; l < j; ++l) {
        const float2 *A = ws + off_tile(i, l);
        const float2 *Bt = ws + off_tile(j, l);
        // four steps' loads in flight at a time (the tiles come from L2):
        // 5.2 -> 4.3 ms per frame at 256 antennas; a full unroll (one wave
        // per SIMD) took 7.1 ms
#pragma unroll 4
        for (int m = 0; m < TE; m += 2) {
            float4 a2[4], b2[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) a2[q] = *(const float4 *)(A + (4 * lr + q) * TE + m);
#pragma unroll
            for (int t = 0; t < 4; ++t) b2[t] = *(const float4 *)(Bt + (4 * lc + t) * TE + m);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    acc[q][t] = msc(acc[q][t], make_float2(a2[q].x, a2[q].y), make_float2(b2[t].x, b2[t].y));
                    acc[q][t] = msc(acc[q][t], make_float2(a2[q].z, a2[q].w), make_float2(b2[t].z, b2[t].w));
                }
        }
    }
}

// Wave 0: Cholesky of the diagonal tile D (LDS) and the inverse of its
// factor.  Returns false (wave-uniform) on a pivot not above 2^-20 of the
// entry of M it started from.
__device__ bool factor_diag_tile(float2 *D, float2 *Dinv, const float *dorig) {
    const int lane = lane_of();
    const int col = lane & 31, h = lane >> 5;
    bool ok = true;
    // Schur elimination: D[r][c] -= D[r][k] conj(D[c][k]) / D[k][k], r >= c > k
    for (int k = 0; k < TE; ++k) {
        const float dkk = D[k * TE + k].x;
        if (!(dkk > kRelPivot32 * dorig[k]) || !(dkk - dkk == 0.f)) {
            ok = false;
            break;
        }
        const float inv = 1.f / dkk;
        if (col > k) {
            const float2 lck = D[col * TE + k];
            const float2 sc = make_float2(lck.x * inv, lck.y * inv);
            for (int q = 0; q < TE / 2; ++q) {
                const int r = h + 2 * q;
                if (r >= col) D[r * TE + col] = msc(D[r * TE + col], D[r * TE + k], sc);
            }
        }
        wsync();
    }
    if (!ok) return false;
    // column scaling: L[r][c] = D[r][c] / sqrt(D[c][c]), L[c][c] = sqrt(D[c][c])
    {
        const float dcc = D[col * TE + col].x;
        const float sq = sqrtf(dcc), isq = 1.f / sq;
        for (int q = 0; q < TE / 2; ++q) {
            const int r = h + 2 * q;
            if (r > col) {
                const float2 v = D[r * TE + col];
                D[r * TE + col] = make_float2(v.x * isq, v.y * isq);
            } else if (r == col) {
                D[r * TE + col] = make_float2(sq, 0.f);
            }
        }
    }
    wsync();
    // L^-1 by forward substitution, lane c < 32 owns column c
    if (h == 0) {
        for (int i = 0; i < TE; ++i) {
            if (i < col) {
                Dinv[i * TE + col] = make_float2(0.f, 0.f);
                continue;
            }
            float2 acc = make_float2(i == col ? 1.f : 0.f, 0.f);
            for (int m = col; m < i; ++m) acc = msub(acc, D[i * TE + m], Dinv[m * TE + col]);
            const float il = 1.f / D[i * TE + i].x;
            Dinv[i * TE + col] = make_float2(acc.x * il, acc.y * il);
        }
    }
    wsync();
    return true;
}

__global__ void __launch_bounds__(kCenThreads) central_k(Cen c, const float2 *__restrict__ H,
                                                        const float2 *__restrict__ s, float2 *__restrict__ x,
                                                        float *__restrict__ beta_out, int *__restrict__ status,
                                                        float2 *__restrict__ ws_all) {
    extern __shared__ float4 smem_cen[];
    char *lds = (char *)smem_cen;
    const CenLds L(c.T, c.U);
    float2 *Y = (float2 *)(lds + L.y);
    float2 *D = (float2 *)(lds + L.d);
    float2 *Dinv = (float2 *)(lds + L.dinv);
    float2 *R = (float2 *)(lds + L.r);
    float *dorig = (float *)(lds + L.dorig);
    float *red = (float *)(lds + L.red);
    const int tid = threadIdx.x, lane = lane_of();
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane >> 3, lc = lane & 7;
    const int nl = blockIdx.x, n = c.n0 + nl;
    const int T = c.T, U = c.U, ys = L.ys;
    const float2 *Hn = H + (size_t)n * c.B * U;
    float2 *ws = ws_all + (size_t)nl * (cen_ws_per_sc(T) / sizeof(float2));
    if (tid == 0) red[4] = 1.f;  // factorization ok
    __syncthreads();

    for (int j = 0; j < T; ++j) {
        // tiles (i, j), i >= j: the diagonal one to LDS, the others to the workspace
        for (int i = j + wave; i < T; i += kCenWaves) {
            float2 acc[4][4];
            tile_column_entry(c, Hn, ws, i, j, acc, dorig);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int e = (4 * lr + q) * TE + 4 * lc + t;
                    if (i == j)
                        D[e] = acc[q][t];
                    else
                        ws[off_tile(i, j) + e] = acc[q][t];
                }
        }
        __syncthreads();
        if (wave == 0) {
            const bool ok = factor_diag_tile(D, Dinv, dorig);
            if (!ok && lane == 0) red[4] = 0.f;
            for (int e = lane; e < TC; e += 64) ws[inv_tile(T, j) + e] = Dinv[e];
        }
        __syncthreads();
        if (red[4] == 0.f) break;  // uniform: read after the barrier
        // L_ij = (tile i, j) L_jj^-H, i > j
        for (int i = j + 1 + wave; i < T; i += kCenWaves) {
            float2 *Ti = ws + off_tile(i, j);
            float2 out[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int t = 0; t < 4; ++t) out[q][t] = make_float2(0.f, 0.f);
            for (int m = 0; m < TE; ++m) {
                float2 a[4], b[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) a[q] = Ti[(4 * lr + q) * TE + m];
#pragma unroll
                for (int t = 0; t < 4; ++t) b[t] = Dinv[(4 * lc + t) * TE + m];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int t = 0; t < 4; ++t) out[q][t] = macc(out[q][t], a[q], b[t]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int t = 0; t < 4; ++t) Ti[(4 * lr + q) * TE + 4 * lc + t] = out[q][t];
        }
        // forward substitution of tile row j: Y_j = L_jj^-1 (H_j - sum_{l<j} L_jl Y_l)
        if (wave == (T - 1 - j) % kCenWaves) {
            const int r = lane & 31, h = lane >> 5;
            const int row = TE * j + r;
            for (int u = h; u < U; u += 2) {
                float2 acc = row < c.B ? Hn[(size_t)row * U + u] : make_float2(0.f, 0.f);
                for (int l = 0; l < j; ++l) {
                    const float2 *Ljl = ws + off_tile(j, l) + r * TE;
                    for (int m = 0; m < TE; ++m) {
                        acc = msub(acc, Ljl[m], Y[(TE * l + m) * ys + u]);
                    }
                }
                R[r * ys + u] = acc;
            }
            wsync();
            for (int u = h; u < U; u += 2) {
                float2 acc = make_float2(0.f, 0.f);
                for (int m = 0; m <= r; ++m) acc = mac(acc, Dinv[r * TE + m], R[m * ys + u]);
                Y[row * ys + u] = acc;
            }
        }
        __syncthreads();
    }
    const bool ok = red[4] != 0.f;
    float bw = 0.f;
    if (ok) {
        // back substitution by tile rows: Q_i = L_ii^-H (Y_i - sum_{l>i} L_li^H Q_l)
        const int r = tid & 31, g = tid >> 5;
        for (int i = T - 1; i >= 0; --i) {
            for (int u = g; u < U; u += kCenThreads / 32) {
                float2 acc = Y[(TE * i + r) * ys + u];
                for (int l = i + 1; l < T; ++l) {
                    const float2 *Lli = ws + off_tile(l, i);
                    for (int m = 0; m < TE; ++m) {
                        // - conj(L_li[m][r]) Q_l[m][u]
                        acc = cmsub(acc, Lli[m * TE + r], Y[(TE * l + m) * ys + u]);
                    }
                }
                R[r * ys + u] = acc;
            }
            __syncthreads();
            const float2 *Di = ws + inv_tile(T, i);
            for (int u = g; u < U; u += kCenThreads / 32) {
                float2 acc = make_float2(0.f, 0.f);
                for (int m = r; m < TE; ++m) acc = cmac(acc, Di[m * TE + r], R[m * ys + u]);
                Y[(TE * i + r) * ys + u] = acc;
            }
            __syncthreads();
        }
        // tr(Q^H Q)
        float t = 0.f;
        for (int e = tid; e < c.B * U; e += kCenThreads) {
            const float2 v = Y[(e / U) * ys + e % U];
            t = fmaf(v.x, v.x, fmaf(v.y, v.y, t));
        }
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) red[wave] = t;
        __syncthreads();
        const float tr = red[0] + red[1] + red[2] + red[3];
        if (tr > 0.f && tr - tr == 0.f) bw = sqrtf(tr * c.Es / c.power);
    }
    if (tid == 0) {
        if (beta_out) beta_out[n] = bw;
        if (status) status[n] = bw > 0.f ? PRECODE_ST_OK : PRECODE_ST_FAIL;
    }
    const float ib = bw > 0.f ? 1.f / bw : 0.f;
    for (int b = tid; b < c.B; b += kCenThreads) {
        for (int k = 0; k < c.K; ++k) {
            const float2 *sk = s + ((size_t)k * c.n_sc + n) * U;
            float2 acc = make_float2(0.f, 0.f);
            if (bw > 0.f)
                for (int u = 0; u < U; ++u) acc = mac(acc, Y[b * ys + u], sk[u]);
            x[((size_t)k * c.n_sc + n) * c.B + b] = make_float2(acc.x * ib, acc.y * ib);
        }
    }
}

}  // namespace

size_t central_lds_bytes(int B, int U) { return CenLds((B + TE - 1) / TE, U).bytes; }
bool central_supported(int B, int U) { return B >= 1 && U >= 1 && central_lds_bytes(B, U) <= kCenMaxLds; }
size_t central_ws_bytes(int B, int n_chunk) { return cen_ws_per_sc((B + TE - 1) / TE) * (size_t)n_chunk; }

hipError_t central_run(int B, int U, int n_sc, int K, float kappa, float Es, float power, const float2 *H,
                       const float2 *s, float2 *x, float *beta, int *status, void *ws, size_t ws_bytes,
                       hipStream_t st) {
    if (!central_supported(B, U)) return hipErrorNotSupported;
    Cen c;
    c.B = B;
    c.U = U;
    c.n_sc = n_sc;
    c.K = K;
    c.T = (B + TE - 1) / TE;
    c.kappa = kappa;
    c.Es = Es;
    c.power = power;
    const size_t per = cen_ws_per_sc(c.T);
    const int chunk = (int)std::min<size_t>((size_t)n_sc, ws_bytes / per);
    if (chunk < 1) return hipErrorInvalidValue;
    const size_t lds = central_lds_bytes(B, U);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)central_k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    for (int n0 = 0; n0 < n_sc; n0 += chunk) {
        c.n0 = n0;
        const int nb = std::min(chunk, n_sc - n0);
        hipLaunchKernelGGL(central_k, dim3(nb), dim3(kCenThreads), lds, st, c, H, s, x, beta, status, (float2 *)ws);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pc
