// plain.hip -- the plain batched form: separate FP32 (or FP64-route) kernels
// with no MFMA, no fusion and no graph capture.  Steps, per instance:
//
//   gram      A = sum_c H_c^H H_c + kappa I        (PD, Sec. III-B)
//             A_c = H_c^H H_c + kappa_c I_U        (FD, B_c >= U, Sec. III-C)
//             M_c = H_c H_c^H + kappa_c I_{B_c}    (FD, B_c <  U)
//   factor    Cholesky A = L L^H, W = L^-1, A^-1 = W^H W,
//             t = tr A^-1 - kappa ||A^-1||_F^2     (Lemma 1)
//             PD: beta = sqrt(Es/rho^2 t), scale = 1/beta
//             FD: w_c = sqrt(rho_c^2/(t Es)), scale = w_c
//   solve     z = scale A^-1 s                     (per symbol)
//   refine    (optional) z += sc A^-1 (s - A z / sc), residual in FP64
//             from the complex64 channel (U x U systems)
//   precode   x_c = H_c z                          (per symbol)
//             (FD, B_c < U: x_c = w_c M_c^-1 (H_c s), done in `solve`)
//   retry     an FP32-route instance whose factorization failed is solved
//             on the FP64 route instead (retry_f64.h): its factors and
//             status at prepare, its symbols after the precode
//
// The whole instance runs in T = float, or T = double on the FP64 route
// (inputs widened exactly), with complex64 results.
#include "common.h"
#include "retry_f64.h"

#include <algorithm>

namespace pc {

namespace {

template <typename T>
constexpr bool is64() { return sizeof(T) == 8; }

// FP32 and FP64-route instances share the workspace, so every instance slot
// has the size of its FP64 form: kW elements of T per complex<double> slot.
template <typename T>
constexpr int kW() { return (int)(sizeof(double) / sizeof(T)); }

struct InstInfo {
    int n, c, row0, rows, m;  // subcarrier, cluster, first row, rows, system order
    bool big;                 // FD: B_c >= U (U x U system) ; PD: true
    bool r64;                 // on the FP64 route
    float kap;
};

__device__ inline InstInfo inst_info(const Prob &p, int inst) {
    InstInfo q;
    if (p.arch == kPD) {
        q.n = inst;
        q.c = -1;
        q.row0 = 0;
        q.rows = p.B;
        q.m = p.U;
        q.big = true;
        q.r64 = p.pd_fp64 != 0;
        q.kap = pd_kappa(p);
    } else {
        q.n = inst / p.C;
        q.c = inst % p.C;
        q.row0 = p.off[q.c];
        q.rows = p.off[q.c + 1] - q.row0;
        q.big = q.rows >= p.U;
        q.m = q.big ? p.U : q.rows;
        q.r64 = p.fp64[q.c] != 0;
        q.kap = fd_kappa_c(&p, q.c);
    }
    return q;
}

// --------------------------------------------------------------------------
// gram: one block per instance, threads over the m x m entries.
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) plain_gram_k(Prob p, const float2 *__restrict__ H,
                                                    cx<T> *__restrict__ A) {
    const int inst = blockIdx.x;
    const InstInfo q = inst_info(p, inst);
    if (q.r64 != is64<T>()) return;
    const float2 *Hn = H + (size_t)q.n * p.B * p.U;
    cx<T> *An = A + (size_t)inst * p.U * p.U * kW<T>();
    const int m = q.m;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int i = e / m, j = e % m;
        cx<T> g = {0, 0};
        if (p.arch == kPD) {
            // local Gram per cluster, then the cluster sum (adder tree)
            for (int c = 0; c < p.C; ++c) {
                cx<T> gc = {0, 0};
                for (int b = p.off[c]; b < p.off[c + 1]; ++b)
                    gc = cadd(gc, ccmul(ld_c64<T>(Hn + (size_t)b * p.U + i), ld_c64<T>(Hn + (size_t)b * p.U + j)));
                g = cadd(g, gc);
            }
        } else if (q.big) {
            for (int b = q.row0; b < q.row0 + q.rows; ++b)
                g = cadd(g, ccmul(ld_c64<T>(Hn + (size_t)b * p.U + i), ld_c64<T>(Hn + (size_t)b * p.U + j)));
        } else {
            for (int u = 0; u < p.U; ++u)
                g = cadd(g, cmulc(ld_c64<T>(Hn + (size_t)(q.row0 + i) * p.U + u),
                                  ld_c64<T>(Hn + (size_t)(q.row0 + j) * p.U + u)));
        }
        if (i == j) g.re += (T)q.kap;
        An[i * m + j] = g;
    }
}

// --------------------------------------------------------------------------
// factor: one 64-thread block per instance, in place on global memory.
//   A (lower) -> L (lower) ; L^H copied to the strict upper triangle ;
//   W = L^-1 into the lower triangle (one thread per column) ;
//   A^-1 = W^H W into Ainv ; t, scale, status.
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) plain_factor_k(Prob p, cx<T> *__restrict__ A, cx<T> *__restrict__ Ainv,
                                                    T *__restrict__ scale_ws, float *__restrict__ scale_out,
                                                    int *__restrict__ status) {
    const int inst = blockIdx.x;
    const InstInfo q = inst_info(p, inst);
    if (q.r64 != is64<T>()) return;
    const int m = q.m;
    const int tid = threadIdx.x;
    cx<T> *a = A + (size_t)inst * p.U * p.U * kW<T>();
    cx<T> *ai = Ainv + (size_t)inst * p.U * p.U * kW<T>();
    __shared__ T diag[kMaxU];
    __shared__ T diag0[kMaxU];
    __shared__ T red[2][64];
    bool ok = true;
    const T rel = is64<T>() ? (T)kRelPivot64 : (T)kRelPivot32;
    for (int i = tid; i < m; i += 64) diag0[i] = a[i * m + i].re;
    __syncthreads();
    // Cholesky, right-looking; a pivot not above rel * original diagonal marks
    // the system numerically singular
    for (int k = 0; k < m && ok; ++k) {
        const T akk = a[k * m + k].re;
        ok = (akk > rel * diag0[k]) && finite_f((double)akk);
        __syncthreads();
        if (!ok) break;
        const T d = sqrt(akk);
        for (int i = k + 1 + tid; i < m; i += 64) a[i * m + k] = cscale(a[i * m + k], (T)1 / d);
        if (tid == 0) {
            a[k * m + k] = {d, 0};
            diag[k] = d;
        }
        __syncthreads();
        const int w = m - k - 1;
        for (int e = tid; e < w * w; e += 64) {
            const int i = k + 1 + e / w, j = k + 1 + e % w;
            if (j <= i) a[i * m + j] = csub(a[i * m + j], cmulc(a[i * m + k], a[j * m + k]));
        }
        __syncthreads();
    }
    T t = 0;
    if (ok) {
        // L^H into the strict upper triangle
        for (int e = tid; e < m * m; e += 64) {
            const int i = e / m, j = e % m;
            if (j > i) a[i * m + j] = {a[j * m + i].re, -a[j * m + i].im};
        }
        __syncthreads();
        // W = L^-1, column `tid` by forward substitution; L[i][p] = conj(a[p][i]) (p < i)
        if (tid < m) {
            const int j = tid;
            a[j * m + j] = {(T)1 / diag[j], 0};
            for (int i = j + 1; i < m; ++i) {
                cx<T> acc = {0, 0};
                for (int pp = j; pp < i; ++pp) {
                    const cx<T> lip = {a[pp * m + i].re, -a[pp * m + i].im};
                    acc = cadd(acc, cmul(lip, a[pp * m + j]));
                }
                a[i * m + j] = cscale(acc, -(T)1 / diag[i]);
            }
        }
        __syncthreads();
        // A^-1 = W^H W ; W[p][i] = a[p][i] for p >= i
        T tr = 0, fro = 0;
        for (int e = tid; e < m * m; e += 64) {
            const int i = e / m, j = e % m;
            cx<T> acc = {0, 0};
            for (int pp = (i > j ? i : j); pp < m; ++pp) acc = cadd(acc, ccmul(a[pp * m + i], a[pp * m + j]));
            ai[i * m + j] = acc;
            if (i == j) tr += acc.re;
            fro += cabs2(acc);
        }
        red[0][tid] = tr;
        red[1][tid] = fro;
        __syncthreads();
        for (int sh = 32; sh > 0; sh >>= 1) {
            if (tid < sh) {
                red[0][tid] += red[0][tid + sh];
                red[1][tid] += red[1][tid + sh];
            }
            __syncthreads();
        }
        t = red[0][0] - (T)q.kap * red[1][0];
        ok = (t > (T)0) && finite_f((double)t);
    }
    if (tid == 0) {
        T sc = 0, out = 0;
        if (ok) {
            if (p.arch == kPD) {
                const T beta = sqrt((T)p.Es / (T)p.power * t);
                sc = (T)1 / beta;
                out = beta;
            } else {
                const T rho_c2 = sizeof(T) == sizeof(double) ? (T)fd_power_c_d(&p, q.c) : (T)fd_power_c(&p, q.c);
                const T w = sqrt(rho_c2 / (t * (T)p.Es));
                sc = w;
                out = w;
            }
        }
        scale_ws[inst * kW<T>()] = sc;
        if (scale_out) scale_out[inst] = (float)out;
        if (status) status[inst] = (ok ? PRECODE_ST_OK : PRECODE_ST_FAIL) | (q.r64 ? PRECODE_ST_FP64 : 0);
    }
}

// --------------------------------------------------------------------------
// solve: thread per (k, inst, row of the local system)
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) plain_solve_k(Prob p, int K, const float2 *__restrict__ H,
                                                     const float2 *__restrict__ s, const cx<T> *__restrict__ Ainv,
                                                     const T *__restrict__ scale_ws, float2 *__restrict__ z,
                                                     float2 *__restrict__ x) {
    const size_t ni = (size_t)n_inst(p);
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)K * ni * p.U) return;
    const int r = (int)(gid % p.U);
    const size_t inst = (gid / p.U) % ni;
    const int k = (int)(gid / ((size_t)p.U * ni));
    const InstInfo q = inst_info(p, (int)inst);
    if (q.r64 != is64<T>()) return;
    const T sc = scale_ws[inst * kW<T>()];  // 0 marks a failed instance: its output is 0
    if (sc < (T)0) return;                  // on the FP64 retry (plain_retry_k writes x)
    const cx<T> *ai = Ainv + inst * p.U * p.U * kW<T>();
    const float2 *sk = s + ((size_t)k * p.n_sc + q.n) * p.U;
    if (q.big) {
        if (r >= q.m) return;
        cx<T> acc = {0, 0};
        if (sc != (T)0)
            for (int v = 0; v < q.m; ++v) acc = cadd(acc, cmul(ai[r * q.m + v], ld_c64<T>(sk + v)));
        acc = cscale(acc, sc);
        z[((size_t)k * ni + inst) * p.U + r] = make_float2((float)acc.re, (float)acc.im);
    } else {
        // FD, B_c < U:  x_c = w_c M_c^-1 (H_c s)
        if (r >= q.m) return;
        const float2 *Hn = H + (size_t)q.n * p.B * p.U;
        cx<T> acc = {0, 0};
        for (int bb = 0; bb < q.m && sc != (T)0; ++bb) {
            cx<T> hs = {0, 0};
            for (int u = 0; u < p.U; ++u)
                hs = cadd(hs, cmul(ld_c64<T>(Hn + (size_t)(q.row0 + bb) * p.U + u), ld_c64<T>(sk + u)));
            acc = cadd(acc, cmul(ai[r * q.m + bb], hs));
        }
        acc = cscale(acc, sc);
        x[((size_t)k * p.n_sc + q.n) * p.B + q.row0 + r] = make_float2((float)acc.re, (float)acc.im);
    }
}

// --------------------------------------------------------------------------
// refine: one step of iterative refinement of z = sc A^-1 s for U x U systems
// (PD, and FD clusters with B_c >= U).  With y = z / sc the solution of
// A y = s, the residual r = s - (kappa y + H_c^H (H_c y)) is accumulated in
// FP64 straight from the complex64 channel (never from the stored Gram), and
// z += sc A^-1 r.  One 64-thread block per (symbol, instance); the H_c y
// vector is staged in LDS in chunks of kRefChunk rows.
// --------------------------------------------------------------------------
constexpr int kRefChunk = 512;

template <typename T>
__global__ void __launch_bounds__(64) plain_refine_k(Prob p, int K, const float2 *__restrict__ H,
                                                     const float2 *__restrict__ s, const cx<T> *__restrict__ Ainv,
                                                     const T *__restrict__ scale_ws, float2 *__restrict__ z) {
    const size_t ni = (size_t)n_inst(p);
    const size_t inst = blockIdx.x % ni;
    const int k = (int)(blockIdx.x / ni);
    const InstInfo q = inst_info(p, (int)inst);
    if (q.r64 != is64<T>() || !q.big) return;
    const T sc = scale_ws[inst * kW<T>()];
    if (sc <= (T)0) return;  // failed instance (z stays 0) or on the FP64 retry
    const int tid = threadIdx.x, U = p.U;
    __shared__ cx<double> zy[kMaxU], hz[kRefChunk], acc[kMaxU];
    __shared__ cx<double> r[kMaxU];
    float2 *zk = z + ((size_t)k * ni + inst) * U;
    const float2 *sk = s + ((size_t)k * p.n_sc + q.n) * U;
    const float2 *Hn = H + (size_t)q.n * p.B * U;
    for (int u = tid; u < U; u += 64) {
        zy[u] = {(double)zk[u].x, (double)zk[u].y};
        acc[u] = {0, 0};
    }
    __syncthreads();
    for (int b0 = q.row0; b0 < q.row0 + q.rows; b0 += kRefChunk) {
        const int nb = min(kRefChunk, q.row0 + q.rows - b0);
        for (int i = tid; i < nb; i += 64) {
            cx<double> w = {0, 0};
            const float2 *hb = Hn + (size_t)(b0 + i) * U;
            for (int u = 0; u < U; ++u) w = cadd(w, cmul(ld_c64<double>(hb + u), zy[u]));
            hz[i] = w;
        }
        __syncthreads();
        for (int u = tid; u < U; u += 64) {
            cx<double> a = acc[u];
            for (int i = 0; i < nb; ++i) a = cadd(a, ccmul(ld_c64<double>(Hn + (size_t)(b0 + i) * U + u), hz[i]));
            acc[u] = a;
        }
        __syncthreads();
    }
    // r = s - (kappa z + H^H H z) / sc
    const double inv = 1.0 / (double)sc;
    for (int u = tid; u < U; u += 64) {
        const cx<double> az = cadd(cscale(zy[u], (double)q.kap), acc[u]);
        r[u] = csub(ld_c64<double>(sk + u), cscale(az, inv));
    }
    __syncthreads();
    const cx<T> *ai = Ainv + inst * U * U * kW<T>();
    for (int u = tid; u < U; u += 64) {
        cx<double> d = {0, 0};
        for (int v = 0; v < U; ++v) {
            const cx<T> a = ai[u * U + v];
            d = cadd(d, cmul(cx<double>{(double)a.re, (double)a.im}, r[v]));
        }
        const cx<double> zn = cadd(zy[u], cscale(d, (double)sc));
        zk[u] = make_float2((float)zn.re, (float)zn.im);
    }
}

// --------------------------------------------------------------------------
// precode: thread per (k, n, b)
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) plain_precode_k(Prob p, int K, const float2 *__restrict__ H,
                                                       const float2 *__restrict__ z, const float *__restrict__ scale32,
                                                       float2 *__restrict__ x) {
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)K * p.n_sc * p.B) return;
    const int b = (int)(gid % p.B);
    const int n = (int)((gid / p.B) % p.n_sc);
    const int k = (int)(gid / ((size_t)p.B * p.n_sc));
    const size_t ni = (size_t)n_inst(p);
    size_t inst = n;
    bool r64 = p.pd_fp64 != 0;
    if (p.arch == kFD) {
        int c = 0;
        while (p.off[c + 1] <= b) ++c;
        if (p.off[c + 1] - p.off[c] < p.U) return;  // written by the solve step
        inst = (size_t)n * p.C + c;
        r64 = p.fp64[c] != 0;
    }
    // an FP32-route instance on the FP64 retry: plain_retry_k writes its x
    if (!r64 && scale32[inst * kW<float>()] < 0.f) return;
    const float2 *hb = H + ((size_t)n * p.B + b) * p.U;
    const float2 *zk = z + ((size_t)k * ni + inst) * p.U;
    float2 out;
    if (r64) {
        cx<double> acc = {0, 0};
        for (int u = 0; u < p.U; ++u) acc = cadd(acc, cmul(ld_c64<double>(hb + u), ld_c64<double>(zk + u)));
        out = make_float2((float)acc.re, (float)acc.im);
    } else {
        cx<float> acc = {0, 0};
        for (int u = 0; u < p.U; ++u) acc = cadd(acc, cmul(ld_c64<float>(hb + u), ld_c64<float>(zk + u)));
        out = make_float2(acc.re, acc.im);
    }
    x[gid] = out;
}

// zero x for failed instances (scale == 0) is automatic: z = 0 => x = 0.

// --------------------------------------------------------------------------
// retry: one wave per instance of the FP32 route.  factors: an instance whose
// FP32 factorization failed (scale 0) is factored on the FP64 route
// (f64r::instance writes its scale output and status) and marked with scale
// -1; symbols: every marked instance is solved and precoded on the FP64 route
// (after the FP32 precode, which skips it).
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(64) plain_retry_k(Prob p, int K, int factors, const float2 *__restrict__ H,
                                                    const float2 *__restrict__ s, float2 *__restrict__ x,
                                                    float *__restrict__ scale_ws, float *__restrict__ scale_out,
                                                    int *__restrict__ status) {
    extern __shared__ double retry_lds[];
    const int inst = blockIdx.x;
    const InstInfo q = inst_info(p, inst);
    if (q.r64) return;
    float *sc = scale_ws + (size_t)inst * kW<float>();
    const float v = *sc;
    if (factors ? v != 0.f : v >= 0.f) return;
    // the problem read in place from the kernel arguments (p first)
    const Prob *pk = (const Prob *)__builtin_amdgcn_kernarg_segment_ptr();
    f64r::instance(f64r::shape_of(p), pk, inst, K, factors != 0, H, s, x, scale_out, status, (char *)retry_lds);
    if (factors && threadIdx.x == 0) *sc = -1.f;
}

bool any_route(const Prob &p, bool want64) {
    if (p.arch == kPD) return (p.pd_fp64 != 0) == want64;
    for (int c = 0; c < p.C; ++c)
        if ((p.fp64[c] != 0) == want64) return true;
    return false;
}

}  // namespace

size_t plain_ws_bytes_A(const Prob &p) { return (size_t)n_inst(p) * p.U * p.U * sizeof(cx<double>); }
size_t plain_ws_bytes_scale(const Prob &p) { return (size_t)n_inst(p) * sizeof(double); }
size_t plain_ws_bytes_z(const Prob &p, int K) { return (size_t)K * n_inst(p) * p.U * sizeof(float2); }

hipError_t plain_prepare(const Prob &p, const float2 *H, float *scale_out, int *status, void *ws_A,
                         void *ws_Ainv, void *ws_scale, hipStream_t st) {
    const int ni = n_inst(p);
    if (ni == 0) return hipSuccess;
    if (any_route(p, false)) {
        hipLaunchKernelGGL(plain_gram_k<float>, dim3(ni), dim3(256), 0, st, p, H, (cx<float> *)ws_A);
        hipLaunchKernelGGL(plain_factor_k<float>, dim3(ni), dim3(64), 0, st, p, (cx<float> *)ws_A,
                           (cx<float> *)ws_Ainv, (float *)ws_scale, scale_out, status);
        hipLaunchKernelGGL(plain_retry_k, dim3(ni), dim3(64), f64r::lds_bytes(p.U), st, p, 0, 1, H,
                           (const float2 *)nullptr, (float2 *)nullptr, (float *)ws_scale, scale_out, status);
    }
    if (any_route(p, true)) {
        hipLaunchKernelGGL(plain_gram_k<double>, dim3(ni), dim3(256), 0, st, p, H, (cx<double> *)ws_A);
        hipLaunchKernelGGL(plain_factor_k<double>, dim3(ni), dim3(64), 0, st, p, (cx<double> *)ws_A,
                           (cx<double> *)ws_Ainv, (double *)ws_scale, scale_out, status);
    }
    return hipGetLastError();
}

hipError_t plain_symbols(const Prob &p, int K, const float2 *H, const float2 *s, float2 *x, void *ws_Ainv,
                         void *ws_scale, void *ws_z, hipStream_t st, int refine_steps) {
    const size_t ni = (size_t)n_inst(p);
    if (ni == 0 || K == 0) return hipSuccess;
    const size_t nsolve = (size_t)K * ni * p.U;
    const unsigned gs = (unsigned)((nsolve + 255) / 256);
    if (any_route(p, false))
        hipLaunchKernelGGL(plain_solve_k<float>, dim3(gs), dim3(256), 0, st, p, K, H, s,
                           (const cx<float> *)ws_Ainv, (const float *)ws_scale, (float2 *)ws_z, x);
    if (any_route(p, true))
        hipLaunchKernelGGL(plain_solve_k<double>, dim3(gs), dim3(256), 0, st, p, K, H, s,
                           (const cx<double> *)ws_Ainv, (const double *)ws_scale, (float2 *)ws_z, x);
    if (refine_steps > 0) {
        const unsigned gr = (unsigned)((size_t)K * ni);
        if (any_route(p, false))
            hipLaunchKernelGGL(plain_refine_k<float>, dim3(gr), dim3(64), 0, st, p, K, H, s,
                               (const cx<float> *)ws_Ainv, (const float *)ws_scale, (float2 *)ws_z);
        if (any_route(p, true))
            hipLaunchKernelGGL(plain_refine_k<double>, dim3(gr), dim3(64), 0, st, p, K, H, s,
                               (const cx<double> *)ws_Ainv, (const double *)ws_scale, (float2 *)ws_z);
    }
    const size_t nx = (size_t)K * p.n_sc * p.B;
    hipLaunchKernelGGL(plain_precode_k, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, p, K, H,
                       (const float2 *)ws_z, (const float *)ws_scale, x);
    if (any_route(p, false))
        hipLaunchKernelGGL(plain_retry_k, dim3((unsigned)ni), dim3(64), f64r::lds_bytes(p.U), st, p, K, 0, H, s, x,
                           (float *)ws_scale, (float *)nullptr, (int *)nullptr);
    return hipGetLastError();
}

}  // namespace pc
