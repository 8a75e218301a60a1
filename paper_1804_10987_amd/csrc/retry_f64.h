// retry_f64.h -- one local system solved entirely in FP64 by one wave, from
// the complex64 channel and symbols in global memory.
//
// This is the FP64 route taken by an instance whose FP32 factorization
// failed (a pivot not above kRelPivot32 times its original diagonal entry,
// or a non-finite value).  Theorem 1 only needs A invertible; an FP32
// factorization cannot tell an ill-conditioned system from a singular one,
// so such an instance is solved again with the Gram accumulated in FP64
// (complex64 products are exact there), an FP64 Cholesky factorization
// A = L L^H, W = L^-1 and the Lemma-1 quantities from W, the solve
// z = scale W^H (W s) and the precode x_c = H_c z accumulated in FP64.  Only
// when a pivot is not above kRelPivot64 times its original diagonal entry
// (the oracle's test), or t <= 0, is the instance marked FAIL (x = 0).
//
// Both forms of a local system (Sec. III-C case split):
//   big   (PD, FD with B_c >= U): A = H_c^H H_c + kappa I_U, z = scale A^-1 s,
//         x_c = H_c z
//   small (FD with B_c < U):      M = H_c H_c^H + kappa I_{B_c},
//         x_c = w_c M^-1 (H_c s)
//
// Cold path: one Gram entry per lane, read straight from global memory
// (served by the cache), the factor as a packed lower triangle in the
// wave's LDS area (lds_bytes(m)).  Used by the fused kernels in place of the
// failed FP32 result (same wave, same launch) and by the plain kernels' retry
// launch.
#pragma once

#include "common.h"

namespace pc {
namespace f64r {

__device__ __forceinline__ int lane() { return threadIdx.x & 63; }

// Orders one wave's LDS accesses across this point.
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

// Packed lower triangle: entry (i, j), i >= j.
__host__ __device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Row i of packed entry e (the largest i with tri(i, 0) <= e).
__device__ __forceinline__ int tri_row(int e) {
    int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while (tri(i + 1, 0) <= e) ++i;
    while (tri(i, 0) > e) --i;
    return i;
}

// LDS bytes of one wave for a system of order m: the packed factor, the
// original diagonal and two work vectors.
__host__ __device__ constexpr size_t lds_bytes(int m) {
    return (size_t)m * (m + 1) / 2 * 16 + (size_t)m * 8 + 2 * (size_t)m * 16;
}

__device__ __forceinline__ cx<double> ld64(const float2 *p) {
    const float2 v = *p;
    return {(double)v.x, (double)v.y};
}

// The scalars of a problem the FP64 route needs (passed by value, so that a
// kernel's by-value problem description stays in registers).
struct Shape64 {
    int pd, U, B, C, n_sc;
    float kap, Es, power;
};

__device__ __forceinline__ Shape64 shape_of(const Prob &p) {
    Shape64 q;
    q.pd = p.arch == kPD;
    q.U = p.U;
    q.B = p.B;
    q.C = p.C;
    q.n_sc = p.n_sc;
    q.kap = q.pd ? pd_kappa(p) : 0.f;  // FD: per cluster (fd_kappa_c)
    q.Es = p.Es;
    q.power = p.power;
    return q;
}

// Local system `sys` of problem p (PD: subcarrier sys over all rows; FD:
// cluster sys % C of subcarrier sys / C).  pk: the problem in memory the
// kernel can index (cluster offsets, kappa_c and rho_c^2; read for FD only).  K symbols s[k][n_sc][U] -> x[k][n_sc][B], k < K (K = 0: the
// factorization only).  factors: write scale_out[sys] (beta for PD, w_c for
// FD; 0 on failure) and status[sys] (PRECODE_ST_FP64, plus PRECODE_ST_FAIL
// when the FP64 factorization fails too); either pointer may be NULL.
// lds: lds_bytes(m) bytes of this wave's LDS, m = U (big) or B_c (small).
__device__ __forceinline__ void instance(Shape64 p, const Prob *__restrict__ pk, int sys, int K, bool factors,
                                             const float2 *__restrict__ H, const float2 *__restrict__ s,
                                             float2 *__restrict__ x, float *__restrict__ scale_out,
                                             int *__restrict__ status, char *lds) {
    const int ln = lane();
    const bool pd = p.pd != 0;
    const int U = p.U, B = p.B, C = p.C, n_sc = p.n_sc;
    const int n = pd ? sys : sys / C;
    const int c = pd ? 0 : sys - n * C;
    const int r0 = pd ? 0 : pk->off[c];
    const int rows = pd ? B : pk->off[c + 1] - r0;
    const bool big = rows >= U;
    const int m = big ? U : rows;
    const int nt = tri(m, 0);
    const double kap = pd ? (double)p.kap : (double)fd_kappa_c(pk, c);
    const float2 *Hn = H + (size_t)n * B * U;
    cx<double> *L = (cx<double> *)lds;
    double *d0 = (double *)(L + nt);
    cx<double> *y = (cx<double> *)(d0 + m);
    cx<double> *z = y + m;

    // regularized Gram, lower triangle
    for (int e = ln; e < nt; e += 64) {
        const int i = tri_row(e), j = e - tri(i, 0);
        cx<double> g = {0.0, 0.0};
        if (big) {
            for (int b = r0; b < r0 + rows; ++b)
                g = cadd(g, ccmul(ld64(Hn + (size_t)b * U + i), ld64(Hn + (size_t)b * U + j)));
        } else {
            for (int u = 0; u < U; ++u)
                g = cadd(g, cmulc(ld64(Hn + (size_t)(r0 + i) * U + u), ld64(Hn + (size_t)(r0 + j) * U + u)));
        }
        if (i == j) {
            g.re += kap;
            g.im = 0.0;
            d0[i] = g.re;
        }
        L[e] = g;
    }
    wsync();
    // Cholesky A = L L^H (right-looking); every lane reads the same pivot,
    // so `ok` and the early exit are uniform
    bool ok = true;
    for (int k = 0; k < m; ++k) {
        const double akk = L[tri(k, k)].re;
        ok = akk > kRelPivot64 * d0[k] && finite_f(akk);
        if (!ok) break;
        const double dk = sqrt(akk), inv = 1.0 / dk;
        wsync();
        for (int i = k + 1 + ln; i < m; i += 64) L[tri(i, k)] = cscale(L[tri(i, k)], inv);
        if (ln == 0) L[tri(k, k)] = {dk, 0.0};
        wsync();
        const int w = m - k - 1;
        for (int e = ln; e < tri(w, 0); e += 64) {
            const int ii = tri_row(e), jj = e - tri(ii, 0);
            const int i = k + 1 + ii, j = k + 1 + jj;
            L[tri(i, j)] = csub(L[tri(i, j)], cmulc(L[tri(i, k)], L[tri(j, k)]));
        }
        wsync();
    }
    double t = 0.0;
    if (ok) {
        // W = L^-1 row by row, in place (row i of L is read before it is
        // overwritten; rows < i already hold W); lane j forms W[i][j]
        for (int i = 0; i < m; ++i) {
            const double lii = L[tri(i, i)].re;
            cx<double> wij = {0.0, 0.0};
            if (ln < i) {
                cx<double> acc = {0.0, 0.0};
                for (int q = ln; q < i; ++q) acc = cadd(acc, cmul(L[tri(i, q)], L[tri(q, ln)]));
                wij = cscale(acc, -1.0 / lii);
            } else if (ln == i) {
                wij = {1.0 / lii, 0.0};
            }
            wsync();
            if (ln <= i) L[tri(i, ln)] = wij;
            wsync();
        }
        // Lemma 1: A^-1 = W^H W, tr A^-1 = ||W||_F^2,
        // ||A^-1||_F^2 = sum_ij |sum_{q >= max(i,j)} conj(W_qi) W_qj|^2
        double tr = 0.0, fro = 0.0;
        for (int e = ln; e < nt; e += 64) tr += cabs2(L[e]);
        for (int e = ln; e < m * m; e += 64) {
            const int i = e / m, j = e - (e / m) * m;
            cx<double> acc = {0.0, 0.0};
            for (int q = i > j ? i : j; q < m; ++q) acc = cadd(acc, ccmul(L[tri(q, i)], L[tri(q, j)]));
            fro += cabs2(acc);
        }
        t = wsum(tr) - kap * wsum(fro);
        ok = t > 0.0 && finite_f(t);
    }
    double out = 0.0, scale = 0.0;
    if (ok) {
        if (pd) {
            out = sqrt((double)p.Es / (double)p.power * t);  // beta
            scale = 1.0 / out;
        } else {
            out = sqrt(fd_power_c_d(pk, c) / (t * (double)p.Es));  // w_c
            scale = out;
        }
    }
    if (factors && ln == 0) {
        if (scale_out) scale_out[sys] = (float)out;
        if (status) status[sys] = PRECODE_ST_FP64 | (ok ? 0 : PRECODE_ST_FAIL);
    }
    wsync();
    for (int k = 0; k < K; ++k) {
        const float2 *sk = s + ((size_t)k * n_sc + n) * U;
        float2 *xk = x + ((size_t)k * n_sc + n) * B + r0;
        if (!ok) {
            for (int b = ln; b < rows; b += 64) xk[b] = make_float2(0.f, 0.f);
            continue;
        }
        // v = s (big) or H_c s (small), into z
        if (ln < m) {
            cx<double> v;
            if (big) {
                v = ld64(sk + ln);
            } else {
                v = {0.0, 0.0};
                for (int u = 0; u < U; ++u) v = cadd(v, cmul(ld64(Hn + (size_t)(r0 + ln) * U + u), ld64(sk + u)));
            }
            z[ln] = v;
        }
        wsync();
        // y = W v
        if (ln < m) {
            cx<double> acc = {0.0, 0.0};
            for (int q = 0; q <= ln; ++q) acc = cadd(acc, cmul(L[tri(ln, q)], z[q]));
            y[ln] = acc;
        }
        wsync();
        // z = scale W^H y = scale A^-1 v
        if (ln < m) {
            cx<double> acc = {0.0, 0.0};
            for (int q = ln; q < m; ++q) acc = cadd(acc, ccmul(L[tri(q, ln)], y[q]));
            z[ln] = cscale(acc, scale);
        }
        wsync();
        if (big) {
            // x_c = H_c z
            for (int b = ln; b < rows; b += 64) {
                cx<double> acc = {0.0, 0.0};
                const float2 *hb = Hn + (size_t)(r0 + b) * U;
                for (int u = 0; u < U; ++u) acc = cadd(acc, cmul(ld64(hb + u), z[u]));
                xk[b] = make_float2((float)acc.re, (float)acc.im);
            }
        } else if (ln < m) {
            xk[ln] = make_float2((float)z[ln].re, (float)z[ln].im);
        }
        wsync();
    }
}

}  // namespace f64r
}  // namespace pc
