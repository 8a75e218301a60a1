// common.h -- shared device/host definitions of the precoding library.
//
// Layouts follow include/precode.h: H[n_sc][B][U], s[K][n_sc][U],
// x[K][n_sc][B], complex64 interleaved.  An "instance" is one small linear
// system: a subcarrier for PD (Sec. III-B), a (subcarrier, cluster) pair for
// FD (Sec. III-C).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "precode.h"

namespace pc {

constexpr int kMaxC = 256;   // clusters per cell
constexpr int kMaxU = 64;    // users
constexpr int kMaxB = 4096;  // antennas
constexpr int kMaxK = 4096;  // symbols per call
constexpr int kMaxCv = 64;   // clusters of a call with per-cluster tau_c / rho_c^2

enum Arch { kPD = 0, kFD = 1 };

// A Cholesky pivot that is not above this fraction of the original diagonal
// entry marks the system numerically singular (status PRECODE_ST_FAIL):
// about 16 units of roundoff in FP32, 2^-40 on the FP64 route.
constexpr float kRelPivot32 = 9.5367431640625e-07f;  // 2^-20
constexpr double kRelPivot64 = 9.094947017729282e-13;  // 2^-40

// Per-call problem description, passed to kernels by value.
struct Prob {
    int arch;       // kPD / kFD
    int zf;         // 1: kappa = 0
    int B, U, n_sc, K, C;
    float kappa;    // Theorem-1 regularizer (PD) / base regularizer (FD)
    float power;    // rho^2
    float Es;
    float tau;      // FD tau_c
    int off[kMaxC + 1];          // cluster row offsets, off[C] = B
    unsigned char fp64[kMaxC];   // FD: cluster solved on the FP64 route
    int pd_fp64;                 // PD: every subcarrier on the FP64 route
    int clvar;                   // FD: the call's per-cluster kappa_c / rho_c^2 below
    float clk[kMaxCv];           // kappa_c = tau_c U N0 / rho_c^2 (clvar)
    float clp[kMaxCv];           // rho_c^2 (clvar)
};

__host__ __device__ inline int n_inst(const Prob &p) { return p.arch == kPD ? p.n_sc : p.n_sc * p.C; }

__host__ __device__ inline float pd_kappa(const Prob &p) { return p.zf ? 0.f : p.kappa; }

// Regularizer and power budget of FD cluster c (eq. regularization and the
// power-allocation footnote of Sec. III-C): the call's per-cluster values when
// given, else kappa_c = tau_c U N0 / rho_c^2 = tau C kappa and rho_c^2 =
// rho^2 / C.  pk: the problem in memory a kernel can index (the
// kernarg segment or a table in device memory).
__host__ __device__ inline float fd_kappa_c(const Prob *pk, int c) {
    if (pk->zf) return 0.f;
    return pk->clvar ? pk->clk[c] : pk->tau * (float)pk->C * pk->kappa;
}
__host__ __device__ inline float fd_power_c(const Prob *pk, int c) {
    return pk->clvar ? pk->clp[c] : pk->power / (float)pk->C;
}
__host__ __device__ inline double fd_power_c_d(const Prob *pk, int c) {
    return pk->clvar ? (double)pk->clp[c] : (double)pk->power / (double)pk->C;
}

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> ccmul(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ T cabs2(cx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename T>
__device__ __forceinline__ cx<T> ld_c64(const float2 *p) {
    float2 v = *p;
    return {(T)v.x, (T)v.y};
}

__device__ __forceinline__ bool finite_f(double v) { return v == v && v - v == 0.0; }

// Argument validation shared by every entry point (api.hip): fills *out or
// returns the PRECODE_E* code.
int make_prob_checked(int arch, float rho, const int *sizes, int C, int mode, int B, int U, int n_sc, int K,
                      const precode_params *q, Prob *out);
// Device of a context (api.hip).
int ctx_device(const precode_ctx *ctx);
// precode_pd with every workspace the call needs carved from ws (cap bytes):
// no allocation, no event, no launch-shape timing; PRECODE_ENOMEM when the
// call needs more than cap (api.hip).
int pd_fixed_ws(precode_ctx *ctx, const void *H, const void *s, float rho, const int *sizes, int C, int mode, int B,
                int U, int n_sc, int K, const precode_params *params, void *x, float *beta, int *status, void *stream,
                void *ws, size_t cap);

// Plain kernels (plain.hip).  Workspace: A and Ainv hold n_inst U x U
// complex<double>-sized slots, scale n_inst doubles, z K * n_inst * U complex64.
hipError_t plain_prepare(const Prob &p, const float2 *H, float *scale_out, int *status, void *ws_A,
                         void *ws_Ainv, void *ws_scale, hipStream_t st);
hipError_t plain_symbols(const Prob &p, int K, const float2 *H, const float2 *s, float2 *x, void *ws_Ainv,
                         void *ws_scale, void *ws_z, hipStream_t st, int refine_steps = 0);
size_t plain_ws_bytes_A(const Prob &p);
size_t plain_ws_bytes_scale(const Prob &p);
size_t plain_ws_bytes_z(const Prob &p, int K);

// Fused single-launch kernel (fused.hip).  Returns hipErrorNotSupported if the
// shape is outside what it handles.
bool fused_supported(const Prob &p, int precision);
// *nw_used (may be NULL) receives the waves per workgroup the launch used.
hipError_t fused_run(const Prob &p, int precision, const float2 *H, const float2 *s, float2 *x,
                     float *scale_out, int *status, hipStream_t st, int *nw_used = nullptr);
// The FP64 route in one fused launch (fused_f64.hip), one wave per local
// system: every local system of the problem on the FP64 route, U <= 32 and
// U <= B_eff <= 64, K >= 1, not precision FP64 (which the wide FP64 kernel
// takes, its precode in FP64 throughout).
bool fused_f64_supported(const Prob &p, int precision, int K);
hipError_t fused_f64_run(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *scale_out, int *status,
                         hipStream_t st);
// Waves per workgroup of the batch launches.
int fused_default_waves();
// Launch-shape autotuning on the first call of a problem shape (on by
// default), per host thread.  A serving loop turns it off while it runs:
// timing the candidates synchronizes the stream, a stall its latency cannot
// absorb; calls then use a shape the process has already tuned, else the
// default shape.
void fused_set_autotune(bool on);
// Forgets every tuned shape of the process; the next untuned call reads the
// cache file again.
void fused_autotune_reset();
// Frame split of the fused kernel: prepare writes scale * A^-1 per instance
// (n_inst x U x U complex64, scale = 1/beta for PD, w_c for FD; zero for an
// instance on the FP64 route or failed) with beta / weights and status;
// symbols precodes nk symbols from it, reading prepare's status: an instance
// whose status is PRECODE_ST_FP64 (its FP32 factorization failed, the FP64
// one succeeded) is solved on the FP64 route again at every symbol pass.
hipError_t fused_prepare(const Prob &p, int precision, const float2 *H, float2 *ainv, float *scale_out, int *status,
                         hipStream_t st);
hipError_t fused_symbols(const Prob &p, int precision, int nk, const float2 *H, const float2 *ainv,
                         const int *status, const float2 *s, float2 *x, hipStream_t st);

// One step of iterative refinement fused after the factorization
// (refine.hip): fused_prepare at `precision` into the workspace ws
// (fused_refine_ws_bytes: factors, scale, status), then one wave per system
// forms the FP64 Gram, the FP32 solve, the FP64 residual, the corrected solve
// and the precode.  scale_out / status (may be NULL) receive the prepare
// pass's outputs.
size_t fused_refine_ws_bytes(const Prob &p);
hipError_t fused_refine_run(const Prob &p, int precision, const float2 *H, const float2 *s, float2 *x,
                            float *scale_out, int *status, void *ws, hipStream_t st);

// Heterogeneous batch of fused problems (batch.hip), each with K >= 1 and of
// its kind: kBatchTile problems fused_supported at `precision`, kBatchWide
// problems wide_supported, kBatchF64 problems fused_f64_supported.  Tile
// problems are grouped by tile width (U <= 16 or U <= 32) and register tiles,
// wide problems by system order; each group -- PD and FD alike -- runs as one
// launch over all its local systems, a block finding its problem by binary
// search in a table in device memory.
// kind: kBatchTile (the register-tile classes), kBatchWide (the wide FP64
// kernel, one launch per system order) or kBatchF64 (the one-wave FP64
// kernel, one launch per problem, no table entry).
enum BatchKind { kBatchTile = 0, kBatchWide = 1, kBatchF64 = 2 };
struct BatchProblem {
    Prob p;
    const float2 *H, *s;
    float2 *x;
    float *scale_out;
    int *status;
    int kind;
};
// One problem of a launch's device table: its systems are the launch's
// blocks block0 .. (blocks of the next entry) - 1.
struct BatchEntry {
    Prob p;
    const float2 *H, *s;
    float2 *x;
    float *scale_out;
    int *status;
    int K;       // symbols
    int block0;  // first block of this problem within its launch
    int cl;      // -1: every local system; >= 0: FD cluster cl of each subcarrier (wide kernel)
};
// Bytes of the device table fused_batch_launch reads.
size_t fused_batch_table_bytes(const BatchProblem *bp, int n);
// Builds the table into host memory `host` (table bytes) in launch order.
void fused_batch_fill(const BatchProblem *bp, int n, void *host);
// Enqueues the class launches reading the table at `dev` (already holding
// what fused_batch_fill wrote); *launches receives the number of launches.
hipError_t fused_batch_launch(const BatchProblem *bp, int n, int precision, const void *dev, hipStream_t st,
                              int *launches);

// Local systems of order up to 64 in one FP64 launch (wide.hip): one
// workgroup per system, U x U form (PD; FD with B_c >= U) or B_c x B_c form
// (FD with B_c < U); every system flagged PRECODE_ST_FP64.  Needs K >= 1 and
// U <= 64.  Launches come in classes of system order (16, 32, 48, 64):
// wide_cluster_order is the class of FD cluster c's systems (of every
// system for PD), wide_order the largest over the problem.
bool wide_supported(const Prob &p, int K);
int wide_cluster_order(const Prob &p, int c);
int wide_order(const Prob &p);
hipError_t wide_run(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *scale_out, int *status,
                    hipStream_t st);
hipError_t wide_batch_launch(int order, const BatchEntry *tab, int n, int blocks, hipStream_t st);
// Frame split of the wide kernel: prepare stores scale * A^-1 per system
// (wide_factor_bytes: n_inst slots of order^2 complex doubles, scale = 1/beta
// for PD, w_c for FD; zero for a failed system) with beta / weights and
// status; symbols precodes nk symbols from it, reading prepare's status.
size_t wide_factor_bytes(const Prob &p);
hipError_t wide_prepare(const Prob &p, const float2 *H, void *fac, float *scale_out, int *status, hipStream_t st);
hipError_t wide_symbols(const Prob &p, int nk, const float2 *H, const void *fac, const int *status, const float2 *s,
                        float2 *x, hipStream_t st);

// Comparison precoders (compare.hip).  Centralized WF in the B x B form of
// Theorem 1: FP32, one workgroup per subcarrier, ws holds ws_bytes of
// per-subcarrier factor tiles (central_ws_bytes(B, 1) each; launches are
// chunked to fit).  MRT with the per-cluster normalization of Sec. III-C.
bool central_supported(int B, int U);
size_t central_ws_bytes(int B, int n_chunk);
hipError_t central_run(int B, int U, int n_sc, int K, float kappa, float Es, float power, const float2 *H,
                       const float2 *s, float2 *x, float *beta, int *status, void *ws, size_t ws_bytes,
                       hipStream_t st);
hipError_t mrt_run(const Prob &p, const float2 *H, const float2 *s, float2 *x, float *wgt, int *status,
                   hipStream_t st);

// The UE side of the uncoded-BER link (ue.hip); half_bits = log2(order) / 2.
float qam_spacing(int order);
hipError_t qam_map_run(const int *labels, long long n, int half_bits, float2 *s, hipStream_t st);
hipError_t ue_receive_run(const float2 *H, const float2 *x, const float2 *noise, float N0, const float *scale, int B,
                          int U, int n_sc, int K, float2 *y, hipStream_t st);
hipError_t ue_gain_run(const float2 *y_pilot, float N0, float Es, int U, int n_sc, float *beta, hipStream_t st);
hipError_t qam_errors_run(const float2 *s_hat, const int *labels, long long n, int half_bits, int *out,
                          unsigned long long *count, hipStream_t st);

}  // namespace pc
