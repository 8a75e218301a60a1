// fused_f64.hip -- the FP64 route in one fused launch: local systems whose
// conditioning calls for FP64 (U / B_eff >= fp64_ratio; precision FP64, with
// its precode in FP64 throughout, runs on the wide FP64 kernel) with U <= 32
// users and U <= B_eff <= 64 rows.
//
// One wave per local system (FD cluster c of subcarrier n, or a PD subcarrier
// of at most 64 antennas), four systems per workgroup, no workgroup barrier.
// Register layout of the UP x UP system (UP = 16 or 32): lane (r, c) =
// (lane / UP, lane % UP) holds column c of rows s R + r, s < NS (R = 64 / UP
// row groups, NS = UP / R slots), in FP64.
//
//   Gram      G_c = H_c^H H_c in FP64 on FP64 MFMA from coalesced loads:
//             at 16 users straight into the register layout (gram_mfma16);
//             at 32 its blocks (0,0), (0,1), (1,1) per 32-row tile
//             (gram_mfma32_tile), then through LDS into the register layout;
//             complex64 products are exact in FP64
//   invert    A_c = G_c + kappa_c I (scaled by a power of two, as the FP32
//             inversion) inverted by Gauss-Jordan without pivoting (Hermitian
//             positive definite).  Before step k the matrix is
//             [[A11^-1, A11^-1 A12], [-A21 A11^-1, S]]: its column k equals
//             row k conjugated, negated above the diagonal, so one staged
//             copy of row k in LDS gives every lane both its multiplier and
//             its column-k entries
//   factor    t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1) in FP64; PD beta,
//             FD w_c = sqrt(rho_c^2 / (t Es)) (Sec. III-C)
//   solve     Z = scale A^-1 S in FP64 per chunk of 16 symbols: at 16 users
//             on FP64 MFMA (Z^T = S^T conj(A^-1), the inverse's register
//             layout is the B operand); at 32, A^-1 being Hermitian, lane
//             (r, c) forms the part of Z[c][k] over its own rows from its
//             column and the row groups add their parts
//   precode   X_c = H_c Z (Sec. III-B/C) from register tiles loaded again
//             after the inversion: accumulated in FP64 for ZF and for local
//             systems with U / B_eff > 3/4 (precode_in_fp64), otherwise on
//             FP32 MFMA from Z rounded to complex64
//
// Status of every instance: PRECODE_ST_FP64, plus PRECODE_ST_FAIL when a
// pivot is not above kRelPivot64 times its original diagonal entry or t is
// not positive (then x = 0 and the scale output is 0).
#include "f64_common.h"

namespace pc {
namespace {

constexpr int kF64Waves = 4;

// Gauss-Jordan inversion in FP64 of the system in registers (rows / columns
// >= m hold the identity).  Step k: the lanes of row k's group write row k to
// LDS (as [upos(c)] complex FP64), every lane reads its column's entry (the
// multiplier) and the entries at its rows' positions (its column-k entries,
// by the block structure above), then updates its slots.  Returns whether
// every pivot is finite and above kRelPivot64 times its original diagonal
// entry d0.
template <int UP>
__device__ __forceinline__ bool gj_f64(double (&re)[F64L<UP>::NS], double (&im)[F64L<UP>::NS], double d0,
                                       cx<double> *row) {
    constexpr int R = F64L<UP>::R, NS = F64L<UP>::NS;
    const int lane = lane_id();
    const int r = lane / UP, c = lane % UP;
    const int pc = upos<UP>(c);
    double pv = 1.0;
#pragma unroll
    for (int k = 0; k < UP; ++k) {
        const int sk = k / R, rk = k % R;
        if (r == rk) row[pc] = {re[sk], im[sk]};
        wave_sync();
        // multiplier row: a_kc / a_kk, and 1 + 1/a_kk in the pivot column so
        // that one update also turns column k into -a_ik / a_kk; row k
        // itself becomes a_kc / a_kk (pivot 1/a_kk)
        const cx<double> akc = row[pc];
        const double piv = row[upos<UP>(k)].re;
        const bool iscol = c == k;
        pv = iscol ? piv : pv;
        // 1 / piv: hardware reciprocal and two Newton steps
        double inv = __builtin_amdgcn_rcp(piv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        const double mre = iscol ? 1.0 + inv : akc.re * inv;
        const double mim = iscol ? 0.0 : akc.im * inv;
        const bool isrow = r == rk;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            // column k at row i = s R + r: conj(a_ki), negated for i < k
            const cx<double> ak = row[r * NS + s];
            const double sg = s * R + r < k ? -1.0 : 1.0;
            const double ar = sg * ak.re, ai = -sg * ak.im;
            const double xr = fma(-ar, mre, fma(ai, mim, re[s]));
            const double xi = fma(-ar, mim, fma(-ai, mre, im[s]));
            if (s == sk) {
                re[s] = isrow ? (iscol ? inv : mre) : xr;
                im[s] = isrow ? mim : xi;
            } else {
                re[s] = xr;
                im[s] = xi;
            }
        }
        wave_sync();  // the row buffer is rewritten by the next step
        __builtin_amdgcn_sched_barrier(0);
    }
    return __all((pv > kRelPivot64 * d0) && (pv < (double)INFINITY));
}

template <int UP, int NT, int KU, bool P64>
__device__ __forceinline__ void f64_system(const Prob &p, const Prob *__restrict__ pk, int sys, int K,
                                           const float2 *__restrict__ H, const float2 *__restrict__ s,
                                           float2 *__restrict__ x, float *__restrict__ scale_out,
                                           int *__restrict__ status, char *wb) {
    constexpr int R = F64L<UP>::R, NS = F64L<UP>::NS;
    const int lane = lane_id();
    const int r = lane / UP, c = lane % UP;
    const bool pd = p.arch == kPD;
    const int B = p.B, U = p.U, C = p.C, n_sc = p.n_sc;
    const int n = pd ? sys : sys / C;
    const int cl = pd ? 0 : sys - n * C;
    const int r0 = pd ? 0 : pk->off[cl], r1 = pd ? B : pk->off[cl + 1];
    const int nrows = r1 - r0;
    const float2 *Hn = H + (size_t)n * B * U;
    float2 *rowsL = (float2 *)wb;                                         // [32][UP] staged rows
    cx<float> *sb = (cx<float> *)wb;                                     // [KC][UP] symbols (upos order)
    cx<float> *zb32 = (cx<float> *)(wb + F64L<UP>::s_bytes);             // [UP][KC] Z chunk (FP32 precode)
    cx<double> *zb = (cx<double> *)(wb + F64L<UP>::rows_bytes);          // [KC][UP] Z chunk (FP64 precode)
    cx<double> *rowbuf = (cx<double> *)(wb + F64L<UP>::base_bytes(P64));
    const double kap = pd ? (double)pd_kappa(p) : (double)fd_kappa_c(pk, cl);

    // Gram in FP64, tile by tile through the staged rows (no tile is held in
    // registers across the inversion: the precode loads the rows again)
    double gre[NS], gim[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) gre[q] = gim[q] = 0.0;
    if constexpr (UP == 16) {
        gram_mfma16<NT>(Hn, U, r0, nrows, gre, gim);
    } else {
        f64x4 acc[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) acc[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < NT; ++q)
            if (32 * q < nrows) gram_mfma32_tile(Hn, U, r0 + 32 * q, min(32, nrows - 32 * q), acc);
        gram32_to_regs(acc, (cx<double> *)wb, gre, gim);
        (void)rowsL;
    }
    // the first symbol chunk, in flight during the inversion
    float2 sym[F64L<UP>::SPL];
    if (K > 0) load_syms<UP>(s, 0, min(KC, K), n, n_sc, U, sym);
    // A = G + kappa I, identity past U; d0 = original diagonal entry of column c
    double dloc = 0.0;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int i = q * R + r;
        const bool in = i < U && c < U;
        if (i == c) {
            gre[q] = in ? gre[q] + kap : 1.0;
            dloc = gre[q];
        } else if (!in) {
            gre[q] = 0.0;
        }
        gim[q] = in && i != c ? gim[q] : 0.0;
    }
    // the diagonal entry of column c sits in row group c % R: to every lane of the column
    double d0 = group_sum_d<UP>(r == c % R ? dloc : 0.0);
    // invert 2^-e A with its largest diagonal entry in [0.5, 1) (no pivot
    // above 1, so 1 + 1/pivot keeps 1/pivot to an ulp); A^-1 = 2^-e (2^-e A)^-1
    const double dmax = wave_max_d(c < U ? d0 : 0.0);
    int e = 0;
    if (dmax > 0.0 && dmax < (double)INFINITY) e = ilogb(dmax) + 1;
    const double sc = ldexp(1.0, -e);
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const bool in = q * R + r < U && c < U;
        gre[q] = in ? gre[q] * sc : gre[q];
        gim[q] = in ? gim[q] * sc : gim[q];
    }
    d0 = c < U ? d0 * sc : d0;
    bool ok = gj_f64<UP>(gre, gim, d0, rowbuf);
    // the rows again for the precode (in flight during the Lemma-1 sums)
    Tile<UP, kF32> tl[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const bool v = 32 * q < nrows;
        load_tile<UP, kF32, false>(Hn, U, v ? r0 + 32 * q : r0, v ? min(32, nrows - 32 * q) : 0, tl[q]);
    }
    double tr = 0.0, fro = 0.0;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int i = q * R + r;
        gre[q] *= sc;
        gim[q] *= sc;
        if (i < U && c < U) {
            fro += gre[q] * gre[q] + gim[q] * gim[q];
            if (i == c) tr += gre[q];
        }
    }
    tr = wave_sum_d(tr);
    fro = wave_sum_d(fro);
    const double t = tr - kap * fro;
    ok = ok && t > 0.0 && t < (double)INFINITY;
    double out = 0.0, scale = 0.0;
    if (ok) {
        if (pd) {
            out = sqrt((double)p.Es / (double)p.power * t);  // beta
            scale = 1.0 / out;
        } else {
            out = sqrt(fd_power_c_d(pk, cl) / (t * (double)p.Es));  // w_c
            scale = out;
        }
    }
    if (lane == 0) {
        if (scale_out) scale_out[sys] = (float)out;
        if (status) status[sys] = (ok ? PRECODE_ST_OK : PRECODE_ST_FAIL) | PRECODE_ST_FP64;
    }
    const int j = lane & 31, g = lane >> 5;
    for (int k0 = 0; k0 < K; k0 += KC) {
        const int kc = min(KC, K - k0);
        if (k0 > 0) load_syms<UP>(s, k0, kc, n, n_sc, U, sym);
        stage_syms<UP>(sym, kc, U, sb);
        wave_sync();
        // Z[c][k] = scale sum_i conj(A^-1[i][c]) S[i][k] (A^-1 Hermitian)
        if constexpr (UP == 16) {
            // Z^T = S^T conj(A^-1) on FP64 MFMA, K step q over users 4 q ..
            // 4 q + 3: lane (r, c) feeds S[4 q + r][c] (user 4 q + r, symbol
            // c) as A[c][r] and its slot q, conj(A^-1[4 q + r][c]), as B[r][c];
            // D[k][c] = Z[c][k] lands in lane (k % 4, c), register k / 4
            f64x4 dre = {0.0, 0.0, 0.0, 0.0}, dim = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const cx<float> sv = sb[c * UP + upos<UP>(q * R + r)];
                const double sr = sv.re, si = sv.im;
                dre = __builtin_amdgcn_mfma_f64_16x16x4f64(sr, gre[q], dre, 0, 0, 0);
                dre = __builtin_amdgcn_mfma_f64_16x16x4f64(si, gim[q], dre, 0, 0, 0);
                dim = __builtin_amdgcn_mfma_f64_16x16x4f64(si, gre[q], dim, 0, 0, 0);
                dim = __builtin_amdgcn_mfma_f64_16x16x4f64(-sr, gim[q], dim, 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = 4 * t + r;
                const bool live = ok && c < U && k < kc;
                const double a = live ? scale * dre[t] : 0.0, b = live ? scale * dim[t] : 0.0;
                if constexpr (P64)
                    zb[k * UP + c] = {a, b};
                else
                    zb32[c * KC + k] = {(float)a, (float)b};
            }
        }
        // this lane's rows i = q R + r, then the row groups' parts added; KU
        // symbols per pass (independent accumulation chains)
        for (int k4 = 0; k4 < (UP == 16 ? 0 : KC); k4 += KU) {
            double zr[KU], zi[KU];
#pragma unroll
            for (int u = 0; u < KU; ++u) zr[u] = zi[u] = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < NS / 2; ++q2) {
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    const float4 v = ((const float4 *)(sb + (k4 + u) * UP + r * NS))[q2];
                    const double s0r = v.x, s0i = v.y, s1r = v.z, s1i = v.w;
                    zr[u] = fma(gre[2 * q2], s0r, fma(gim[2 * q2], s0i, zr[u]));
                    zi[u] = fma(gre[2 * q2], s0i, fma(-gim[2 * q2], s0r, zi[u]));
                    zr[u] = fma(gre[2 * q2 + 1], s1r, fma(gim[2 * q2 + 1], s1i, zr[u]));
                    zi[u] = fma(gre[2 * q2 + 1], s1i, fma(-gim[2 * q2 + 1], s1r, zi[u]));
                }
            }
#pragma unroll
            for (int u = 0; u < KU; ++u) {
                const double a = group_sum_d<UP>(zr[u]), b = group_sum_d<UP>(zi[u]);
                if (r == 0) {
                    const bool live = ok && c < U && k4 + u < kc;
                    if constexpr (P64)
                        zb[(k4 + u) * UP + c] = {live ? scale * a : 0.0, live ? scale * b : 0.0};
                    else
                        zb32[c * KC + k4 + u] = {live ? (float)(scale * a) : 0.f, live ? (float)(scale * b) : 0.f};
                }
            }
        }
        wave_sync();
        if constexpr (!P64) {
            // precode X_c = H_c Z on FP32 MFMA from the register tiles
            ZOp<UP, kF32> z;
            make_zop<UP, kF32>(zb32, KC, 1, kc, z);
#pragma unroll
            for (int q = 0; q < NT; ++q)
                if (32 * q < nrows)
                    store_x(mfma_apply_packed<UP, kF32>(tl[q], z), r0 + 32 * q, min(32, nrows - 32 * q), k0, kc, n,
                            n_sc, B, x);
        } else {
            // precode accumulated in FP64: lane (j, g) takes row j, users
            // g UP/2 .. of each tile and adds its half of the sum to its
            // partner's
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                if (32 * q >= nrows) continue;
                const int nq = min(32, nrows - 32 * q);
                float2 *xq = x + ((size_t)k0 * n_sc + n) * B + r0 + 32 * q + j;
                for (int k4 = 0; k4 < KC; k4 += KU) {
                    double xr[KU], xi[KU];
#pragma unroll
                    for (int u = 0; u < KU; ++u) xr[u] = xi[u] = 0.0;
#pragma unroll
                    for (int m2 = 0; m2 < UP / 2; ++m2) {
                        const double hr = tl[q].f[2 * m2], hi = tl[q].f[2 * m2 + 1];
#pragma unroll
                        for (int u = 0; u < KU; ++u) {
                            const cx<double> zz = zb[(k4 + u) * UP + g * (UP / 2) + m2];
                            xr[u] = fma(hr, zz.re, fma(-hi, zz.im, xr[u]));
                            xi[u] = fma(hr, zz.im, fma(hi, zz.re, xi[u]));
                        }
                    }
#pragma unroll
                    for (int u = 0; u < KU; ++u) {
                        const int k = k4 + u;
                        const double a = xr[u] + swap32_d(xr[u], g == 0), b = xi[u] + swap32_d(xi[u], g == 0);
                        if ((k & 1) == g && k < kc && j < nq)
                            __builtin_nontemporal_store((floatx2){(float)a, (float)b}, (floatx2 *)(xq + (size_t)k * n_sc * B));
                    }
                }
            }
        }
        wave_sync();  // the chunks are rewritten by the next one
    }
}

// Symbols per pass of the solve and the precode (independent chains), and
// the waves per SIMD the register allocation targets.
template <int UP, int NT>
struct F64Cfg {
    static constexpr int KU = UP == 16 ? 2 : 1;
    static constexpr int min_waves = UP == 16 ? 3 : 2;
};

template <int UP, int NT, bool P64>
__global__ void __launch_bounds__(64 * kF64Waves, (F64Cfg<UP, NT>::min_waves))
    fused_f64_k(Prob p, int K, const float2 *__restrict__ H, const float2 *__restrict__ s, float2 *__restrict__ x,
                float *__restrict__ scale_out, int *__restrict__ status) {
    extern __shared__ float4 smem_f64[];
    const Prob *pk = (const Prob *)__builtin_amdgcn_kernarg_segment_ptr();  // p: the first argument
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sys = blockIdx.x * kF64Waves + wave;
    if (sys >= n_inst(p)) return;
    f64_system<UP, NT, F64Cfg<UP, NT>::KU, P64>(p, pk, sys, K, H, s, x, scale_out, status,
                                                (char *)smem_f64 + (size_t)wave * F64L<UP>::per_wave(P64));
}

// Rows of the largest local system of a problem.
int max_rows(const Prob &p) {
    if (p.arch == kPD) return p.B;
    int m = 0;
    for (int c = 0; c < p.C; ++c) m = p.off[c + 1] - p.off[c] > m ? p.off[c + 1] - p.off[c] : m;
    return m;
}

template <int UP, int NT, bool P64>
hipError_t launch_f64(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *scale_out, int *status,
                      hipStream_t st) {
    const int ni = n_inst(p);
    const unsigned blocks = (unsigned)((ni + kF64Waves - 1) / kF64Waves);
    const size_t lds = F64L<UP>::per_wave(P64) * kF64Waves;
    hipLaunchKernelGGL((fused_f64_k<UP, NT, P64>), dim3(blocks), dim3(64 * kF64Waves), lds, st, p, p.K, H, s, x,
                       scale_out, status);
    return hipGetLastError();
}

template <int UP, int NT>
hipError_t launch_f64_p(bool p64, const Prob &p, const float2 *H, const float2 *s, float2 *x, float *scale_out,
                        int *status, hipStream_t st) {
    return p64 ? launch_f64<UP, NT, true>(p, H, s, x, scale_out, status, st)
               : launch_f64<UP, NT, false>(p, H, s, x, scale_out, status, st);
}

// Whether the precode of the FP64 route accumulates in FP64.  Its FP32
// accumulation errs by about u |H_c| |z| / |x_c| (u = 2^-24), which grows
// with the condition number of H_c: ZF (no regularization) and local
// systems with U / B_eff > 3/4 (cond(H_c) of an i.i.d. channel grows
// without bound as B_eff approaches U; at 3/4 it is about
// (1 + sqrt(3/4)) / (1 - sqrt(3/4)) = 14) accumulate in FP64, the others
// take the FP32 MFMA precode of the FP64 solve (a relative error of about
// 1e-6 at U / B_eff = 1/2).
bool precode_in_fp64(const Prob &p) {
    if (p.zf) return true;
    if (p.arch == kPD) return 4 * p.U > 3 * p.B;
    for (int c = 0; c < p.C; ++c)
        if (4 * p.U > 3 * (p.off[c + 1] - p.off[c])) return true;
    return false;
}

}  // namespace

bool fused_f64_supported(const Prob &p, int precision, int K) {
    if (K < 1 || p.U > 32 || precision == PRECODE_PREC_FP64) return false;
    if (p.arch == kPD) return p.pd_fp64 && p.B >= p.U && p.B <= 64;
    for (int c = 0; c < p.C; ++c) {
        const int bc = p.off[c + 1] - p.off[c];
        if (!p.fp64[c] || bc < p.U || bc > 64) return false;
    }
    return true;
}

hipError_t fused_f64_run(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *scale_out, int *status,
                         hipStream_t st) {
    if (n_inst(p) == 0) return hipSuccess;
    const bool two = max_rows(p) > 32, p64 = precode_in_fp64(p);
    if (p.U <= 16)
        return two ? launch_f64_p<16, 2>(p64, p, H, s, x, scale_out, status, st)
                   : launch_f64_p<16, 1>(p64, p, H, s, x, scale_out, status, st);
    return two ? launch_f64_p<32, 2>(p64, p, H, s, x, scale_out, status, st)
               : launch_f64_p<32, 1>(p64, p, H, s, x, scale_out, status, st);
}

}  // namespace pc
