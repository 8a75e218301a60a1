// api.hip -- the C ABI declared in include/precode.h: argument validation,
// context workspace under an HBM budget, dispatch between the fused kernels
// (register tiles, refinement, one-wave FP64, wide FP64) and the plain
// kernels, the frame/symbol split and the heterogeneous batch call.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "common.h"

using namespace pc;

struct precode_frame {
    Prob prob;
    const float2 *H;
    int fused;      // state from the fused prepare pass (else from the plain kernels)
    int wide;       // state from the wide FP64 kernel's prepare pass
    int precision;
    int refine;     // refinement steps per symbol (plain kernels)
    void *ainv;     // fused: scale * A^-1 (n_inst x U x U complex64); wide: scale * A^-1 (complex FP64,
                    // wide_factor_bytes); plain: A^-1 slots (complex<T>)
    void *scale;    // plain-layout scale (T); unused when fused
    float *scale_out;
    int *status;
    size_t bytes;
    precode_frame *next;
};

struct precode_ctx {
    int device;
    size_t budget;
    size_t held;
    // plain-kernel workspace (grow-only), shared by every plain-path call of
    // the context: wsDone marks the end of the last call's use of it on
    // wsStream, and a call on another stream waits for it first
    void *wsA, *wsAinv, *wsScale, *wsZ;
    size_t capA, capAinv, capScale, capZ;
    hipEvent_t wsDone;
    hipStream_t wsStream;
    int wsUsed;
    // fused refinement workspace (factors, scale, status), ordered as the
    // plain workspace
    void *wsRef;
    size_t capRef;
    // centralized B x B WF factor tiles, ordered as the plain workspace
    void *wsCen;
    size_t capCen;
    precode_frame *frames;
    int last_impl;
    int last_waves;  // waves per workgroup of the last fused launch
    // fused batch slice table: device copy, pinned host staging, and events
    // marking the last copy out of the staging and the last batch reading it
    void *tab, *tabHost;
    size_t capTab, capTabHost;
    hipEvent_t tabCopied, tabRead;
};

struct precode_batch_plan {
    precode_ctx *ctx;
    void *tab;
    size_t tabBytes;
    void *wsA, *wsAinv, *wsScale, *wsZ;
    size_t bA, bS, bZ;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int launches;
    int fused_jobs;  // jobs with n_sc > 0 on the fused kernels
};

namespace {

int dev_err(hipError_t e) { return e == hipSuccess ? PRECODE_OK : PRECODE_EDEVICE; }

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

bool finite_nonneg(float v) { return isfinite(v) && v >= 0.f; }

int ctx_alloc(precode_ctx *ctx, void **ptr, size_t bytes) {
    if (ctx->budget && ctx->held + bytes > ctx->budget) return PRECODE_ENOMEM;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != ctx->device) (void)hipSetDevice(ctx->device);
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 1);
    if (cur >= 0 && cur != ctx->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? PRECODE_ENOMEM : PRECODE_EDEVICE;
    }
    ctx->held += bytes;
    return PRECODE_OK;
}

void ctx_free(precode_ctx *ctx, void *ptr, size_t bytes) {
    if (!ptr) return;
    (void)hipFree(ptr);
    ctx->held -= bytes;
}

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return cs != hipStreamCaptureStatusNone;
}

// Grow a workspace buffer to at least `need` bytes.  The caller's stream may
// still be using the old buffer, so the device is synchronized before a free.
// Under stream capture nothing may synchronize or allocate: the workspace
// must already be large enough (an earlier uncaptured call of the shape).
int grow(precode_ctx *ctx, void **buf, size_t *cap, size_t need, hipStream_t st) {
    if (*cap >= need) return PRECODE_OK;
    if (capturing(st)) return PRECODE_EUNSUPPORTED;
    if (*buf) {
        (void)hipDeviceSynchronize();
        ctx_free(ctx, *buf, *cap);
        *buf = nullptr;
        *cap = 0;
    }
    int rc = ctx_alloc(ctx, buf, need);
    if (rc == PRECODE_OK) *cap = need;
    return rc;
}

// Orders this call's use of the shared plain-path workspace after the last
// one, which may have been enqueued on another stream.  Inside a stream
// capture the captured stream's own order applies (no external wait).
int ws_acquire(precode_ctx *ctx, hipStream_t st) {
    if (!ctx->wsUsed || ctx->wsStream == st || capturing(st)) return PRECODE_OK;
    return hipStreamWaitEvent(st, ctx->wsDone, 0) == hipSuccess ? PRECODE_OK : PRECODE_EDEVICE;
}

int ws_release(precode_ctx *ctx, hipStream_t st) {
    if (capturing(st)) return PRECODE_OK;
    if (!ctx->wsDone && hipEventCreateWithFlags(&ctx->wsDone, hipEventDisableTiming) != hipSuccess)
        return PRECODE_EDEVICE;
    if (hipEventRecord(ctx->wsDone, st) != hipSuccess) return PRECODE_EDEVICE;
    ctx->wsStream = st;
    ctx->wsUsed = 1;
    return PRECODE_OK;
}

precode_params defaults() {
    precode_params d;
    d.power = 1.f;
    d.Es = 1.f;
    d.tau = 0.125f;
    d.precision = PRECODE_PREC_FP32;
    d.refine_steps = 0;
    d.fp64_ratio = 0.5f;
    d.impl = PRECODE_IMPL_AUTO;
    d.cluster_tau = nullptr;
    d.cluster_power = nullptr;
    return d;
}

int check_params(const precode_params &q) {
    if (!(isfinite(q.power) && q.power > 0.f)) return PRECODE_EINVAL;
    if (!(isfinite(q.Es) && q.Es > 0.f)) return PRECODE_EINVAL;
    if (!finite_nonneg(q.tau)) return PRECODE_EINVAL;
    if (q.precision < PRECODE_PREC_FP32 || q.precision > PRECODE_PREC_FP64) return PRECODE_EINVAL;
    if (q.refine_steps < 0 || q.refine_steps > 1) return PRECODE_EINVAL;
    if (!isfinite(q.fp64_ratio)) return PRECODE_EINVAL;
    if (q.impl < PRECODE_IMPL_AUTO || q.impl > PRECODE_IMPL_PLAIN) return PRECODE_EINVAL;
    return PRECODE_OK;
}

// Validates a call and fills the kernel problem description.
int make_prob(int arch, float rho, const int *sizes, int C, int mode, int B, int U, int n_sc, int K,
              const precode_params &q, Prob *out) {
    if (arch != kPD && arch != kFD) return PRECODE_EINVAL;
    if (mode != PRECODE_ZF && mode != PRECODE_WF) return PRECODE_EINVAL;
    if (U < 1 || B < 1 || n_sc < 0 || K < 0 || C < 1) return PRECODE_EINVAL;
    if (!sizes) return PRECODE_EINVAL;
    if (C > B) return PRECODE_EINVAL;
    if (U > kMaxU || B > kMaxB || K > kMaxK || C > kMaxC) return PRECODE_EUNSUPPORTED;
    if (mode == PRECODE_WF && !finite_nonneg(rho)) return PRECODE_EINVAL;
    int rc = check_params(q);
    if (rc) return rc;
    Prob &p = *out;
    memset(&p, 0, sizeof(p));
    p.arch = arch;
    p.zf = mode == PRECODE_ZF;
    p.B = B;
    p.U = U;
    p.n_sc = n_sc;
    p.K = K;
    p.C = C;
    p.kappa = p.zf ? 0.f : rho;
    p.power = q.power;
    p.Es = q.Es;
    p.tau = q.tau;
    long sum = 0;
    p.off[0] = 0;
    for (int c = 0; c < C; ++c) {
        if (sizes[c] < 1) return PRECODE_EINVAL;
        sum += sizes[c];
        if (sum > B) return PRECODE_EINVAL;
        p.off[c + 1] = (int)sum;
    }
    if (sum != B) return PRECODE_EINVAL;
    if (arch == kFD && (q.cluster_tau || q.cluster_power)) {
        // per-cluster tau_c / rho_c^2 (eq. regularization, Sec. III-C)
        if (C > kMaxCv) return PRECODE_EUNSUPPORTED;
        double total = 0.0;
        for (int c = 0; c < C; ++c) {
            const float pw = q.cluster_power ? q.cluster_power[c] : q.power / (float)C;
            const float tc = q.cluster_tau ? q.cluster_tau[c] : q.tau;
            if (!(isfinite(pw) && pw > 0.f) || !finite_nonneg(tc)) return PRECODE_EINVAL;
            total += pw;
            p.clp[c] = pw;
            p.clk[c] = p.zf ? 0.f : (float)((double)tc * (double)rho * (double)q.power / (double)pw);
        }
        if (q.cluster_power && fabs(total - (double)q.power) > 1e-5 * (double)q.power) return PRECODE_EINVAL;
        p.clvar = 1;
    }
    const bool all64 = q.precision == PRECODE_PREC_FP64;
    p.pd_fp64 = all64 || (double)U / (double)B >= (double)q.fp64_ratio;
    for (int c = 0; c < C; ++c)
        p.fp64[c] = all64 || (double)U / (double)sizes[c] >= (double)q.fp64_ratio;
    return PRECODE_OK;
}

// Validates every job of a batch and splits it into problems for the fused
// batch launches (each with its kind) and jobs for the plain kernels (those
// without symbols).  Nothing is launched unless the whole batch is valid.
int classify(const precode_job *jobs, int n_jobs, int precision, std::vector<BatchProblem> *fused,
             std::vector<std::pair<int, Prob>> *plain) {
    for (int i = 0; i < n_jobs; ++i) {
        const precode_job &j = jobs[i];
        precode_params q = defaults();
        q.power = j.power;
        q.Es = j.Es;
        q.tau = j.tau;
        q.precision = precision;
        Prob p;
        int rc = make_prob(j.arch, j.rho, j.cluster_sizes, j.C, j.mode, j.B, j.U, j.n_sc, j.K, q, &p);
        if (rc) return rc;
        if (j.n_sc == 0) continue;
        if (!j.H || (j.K > 0 && (!j.s || !j.x))) return PRECODE_EINVAL;
        if (!aligned8(j.H) || !aligned8(j.s) || !aligned8(j.x)) return PRECODE_EINVAL;
        // register tiles, else the one-wave FP64 kernel, else the wide FP64 kernel
        int kind = -1;
        if (j.K > 0 && fused_supported(p, precision)) kind = kBatchTile;
        else if (fused_f64_supported(p, precision, j.K)) kind = kBatchF64;
        else if (wide_supported(p, j.K)) kind = kBatchWide;
        if (kind < 0 && (precision == PRECODE_PREC_SPLIT_FP16 || precision == PRECODE_PREC_SPLIT_BF16))
            return PRECODE_EUNSUPPORTED;
        if (kind >= 0) {
            BatchProblem b;
            b.p = p;
            b.H = (const float2 *)j.H;
            b.s = (const float2 *)j.s;
            b.x = (float2 *)j.x;
            b.scale_out = j.scale;
            b.status = j.status;
            b.kind = kind;
            fused->push_back(b);
        } else {
            plain->push_back(std::make_pair(i, p));
        }
    }
    return PRECODE_OK;
}

// Plain-kernel path of one validated problem on caller-provided workspace.
int run_plain(const Prob &p, const precode_job &j, void *wsA, void *wsAinv, void *wsScale, void *wsZ,
              hipStream_t st) {
    int rc = dev_err(plain_prepare(p, (const float2 *)j.H, j.scale, j.status, wsA, wsAinv, wsScale, st));
    if (!rc && p.K > 0)
        rc = dev_err(plain_symbols(p, p.K, (const float2 *)j.H, (const float2 *)j.s, (float2 *)j.x, wsAinv, wsScale,
                                   wsZ, st));
    return rc;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// One PD / FD call.  Workspace: the context's (grown on demand, its uses
// ordered across streams) or, with fixed_ws, the fixed_cap bytes there (no
// allocation, no event, no launch-shape timing: PRECODE_ENOMEM when the call
// needs more).
int run(precode_ctx *ctx, int arch, const void *H, const void *s, float rho, const int *sizes, int C, int mode,
        int B, int U, int n_sc, int K, const precode_params *params, void *x, float *scale, int *status,
        void *stream, void *fixed_ws = nullptr, size_t fixed_cap = 0) {
    if (!ctx) return PRECODE_EINVAL;
    const precode_params q = params ? *params : defaults();
    Prob p;
    int rc = make_prob(arch, rho, sizes, C, mode, B, U, n_sc, K, q, &p);
    if (rc) return rc;
    if (n_sc == 0) return PRECODE_OK;
    if (!H || (K > 0 && (!s || !x))) return PRECODE_EINVAL;
    if (!aligned8(H) || !aligned8(s) || !aligned8(x)) return PRECODE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const bool can_fuse = K > 0 && q.refine_steps == 0 && fused_supported(p, q.precision);
    // one refinement step after the fused factorization (refine.hip)
    const bool can_refine = K > 0 && q.refine_steps == 1 && fused_supported(p, q.precision);
    // the FP64 route fused (its Gram, inversion and solve in FP64) when every
    // local system takes it and fits; its FP64 solve needs no refinement step
    const bool can_f64 = !can_fuse && !can_refine && fused_f64_supported(p, q.precision, K);
    // everything else with U <= 64 on the wide FP64 kernel (its FP64 solve
    // needs no refinement step either)
    const bool can_wide = !can_fuse && !can_refine && !can_f64 && wide_supported(p, K);
    const bool any_fused = can_fuse || can_refine || can_f64 || can_wide;
    if (q.impl == PRECODE_IMPL_FUSED && !any_fused) return PRECODE_EUNSUPPORTED;
    if (q.precision == PRECODE_PREC_SPLIT_FP16 || q.precision == PRECODE_PREC_SPLIT_BF16) {
        if (!any_fused) return PRECODE_EUNSUPPORTED;
    }
    const bool fixed = fixed_ws != nullptr;
    // no launch-shape timing on a fixed workspace (it would create events)
    struct Tune {
        bool off;
        explicit Tune(bool o) : off(o) {
            if (off) fused_set_autotune(false);
        }
        ~Tune() {
            if (off) fused_set_autotune(true);
        }
    } tune(fixed);
    if (q.impl != PRECODE_IMPL_PLAIN && can_refine) {
        void *ws = fixed_ws;
        if (fixed) {
            if (fused_refine_ws_bytes(p) > fixed_cap) return PRECODE_ENOMEM;
        } else {
            rc = grow(ctx, &ctx->wsRef, &ctx->capRef, fused_refine_ws_bytes(p), st);
            if (!rc) rc = ws_acquire(ctx, st);
            if (rc) return rc;
            ws = ctx->wsRef;
        }
        rc = dev_err(fused_refine_run(p, q.precision, (const float2 *)H, (const float2 *)s, (float2 *)x, scale, status,
                                      ws, st));
        const int rr = fixed ? PRECODE_OK : ws_release(ctx, st);
        if (!rc) rc = rr;
        if (rc == PRECODE_OK) {
            ctx->last_impl = PRECODE_IMPL_FUSED;
            ctx->last_waves = 0;
        }
        return rc;
    }
    if (q.impl != PRECODE_IMPL_PLAIN && can_f64) {
        rc = dev_err(fused_f64_run(p, (const float2 *)H, (const float2 *)s, (float2 *)x, scale, status, st));
        if (rc == PRECODE_OK) {
            ctx->last_impl = PRECODE_IMPL_FUSED;
            ctx->last_waves = 4;
        }
        return rc;
    }
    if (q.impl != PRECODE_IMPL_PLAIN && can_wide) {
        rc = dev_err(wide_run(p, (const float2 *)H, (const float2 *)s, (float2 *)x, scale, status, st));
        if (rc == PRECODE_OK) {
            ctx->last_impl = PRECODE_IMPL_FUSED;
            ctx->last_waves = 4;
        }
        return rc;
    }
    if (q.impl != PRECODE_IMPL_PLAIN && can_fuse) {
        int nw = 0;
        rc = dev_err(
            fused_run(p, q.precision, (const float2 *)H, (const float2 *)s, (float2 *)x, scale, status, st, &nw));
        if (rc == PRECODE_OK) {
            ctx->last_impl = PRECODE_IMPL_FUSED;
            ctx->last_waves = nw;
        }
        return rc;
    }
    void *wA, *wAinv, *wScale, *wZ;
    if (fixed) {
        // the four plain workspaces carved from the fixed area
        const size_t bA = align256(plain_ws_bytes_A(p)), bS = align256(plain_ws_bytes_scale(p));
        const size_t bZ = align256(plain_ws_bytes_z(p, K > 0 ? K : 1));
        if (2 * bA + bS + bZ > fixed_cap) return PRECODE_ENOMEM;
        char *w = (char *)fixed_ws;
        wA = w;
        wAinv = w + bA;
        wScale = w + 2 * bA;
        wZ = w + 2 * bA + bS;
    } else {
        rc = grow(ctx, &ctx->wsA, &ctx->capA, plain_ws_bytes_A(p), st);
        if (!rc) rc = grow(ctx, &ctx->wsAinv, &ctx->capAinv, plain_ws_bytes_A(p), st);
        if (!rc) rc = grow(ctx, &ctx->wsScale, &ctx->capScale, plain_ws_bytes_scale(p), st);
        if (!rc) rc = grow(ctx, &ctx->wsZ, &ctx->capZ, plain_ws_bytes_z(p, K > 0 ? K : 1), st);
        if (!rc) rc = ws_acquire(ctx, st);
        if (rc) return rc;
        wA = ctx->wsA;
        wAinv = ctx->wsAinv;
        wScale = ctx->wsScale;
        wZ = ctx->wsZ;
    }
    rc = dev_err(plain_prepare(p, (const float2 *)H, scale, status, wA, wAinv, wScale, st));
    if (!rc && K > 0)
        rc = dev_err(plain_symbols(p, K, (const float2 *)H, (const float2 *)s, (float2 *)x, wAinv, wScale, wZ, st,
                                   q.refine_steps));
    const int rr = fixed ? PRECODE_OK : ws_release(ctx, st);
    if (!rc) rc = rr;
    if (rc == PRECODE_OK) ctx->last_impl = PRECODE_IMPL_PLAIN;
    return rc;
}

}  // namespace

namespace pc {
int make_prob_checked(int arch, float rho, const int *sizes, int C, int mode, int B, int U, int n_sc, int K,
                      const precode_params *q, Prob *out) {
    const precode_params qq = q ? *q : defaults();
    return make_prob(arch, rho, sizes, C, mode, B, U, n_sc, K, qq, out);
}
int ctx_device(const precode_ctx *ctx) { return ctx->device; }
int pd_fixed_ws(precode_ctx *ctx, const void *H, const void *s, float rho, const int *sizes, int C, int mode, int B,
                int U, int n_sc, int K, const precode_params *params, void *x, float *beta, int *status, void *stream,
                void *ws, size_t cap) {
    if (!ws) return PRECODE_EINVAL;
    return run(ctx, kPD, H, s, rho, sizes, C, mode, B, U, n_sc, K, params, x, beta, status, stream, ws, cap);
}
}  // namespace pc

extern "C" {

void precode_params_init(precode_params *p) {
    if (p) *p = defaults();
}

const char *precode_strerror(int code) {
    switch (code) {
        case PRECODE_OK: return "ok";
        case PRECODE_EINVAL: return "invalid argument";
        case PRECODE_EUNSUPPORTED: return "unsupported shape or option";
        case PRECODE_ENOMEM: return "out of device memory or over the context budget";
        case PRECODE_EDEVICE: return "HIP runtime error";
        default: return "unknown error";
    }
}

int precode_ctx_create(int device, size_t hbm_budget_bytes, precode_ctx **out) {
    if (!out) return PRECODE_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) {
        (void)hipGetLastError();
        return PRECODE_EDEVICE;
    }
    if (device < 0 || device >= ndev) return PRECODE_EINVAL;
    precode_ctx *c = new (std::nothrow) precode_ctx;
    if (!c) return PRECODE_ENOMEM;
    memset(c, 0, sizeof(*c));
    c->device = device;
    c->budget = hbm_budget_bytes;
    *out = c;
    return PRECODE_OK;
}

int precode_ctx_destroy(precode_ctx *ctx) {
    if (!ctx) return PRECODE_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    while (ctx->frames) {
        precode_frame *f = ctx->frames;
        ctx->frames = f->next;
        ctx_free(ctx, f->ainv, f->bytes);
        delete f;
    }
    ctx_free(ctx, ctx->wsA, ctx->capA);
    ctx_free(ctx, ctx->wsAinv, ctx->capAinv);
    ctx_free(ctx, ctx->wsScale, ctx->capScale);
    ctx_free(ctx, ctx->wsZ, ctx->capZ);
    ctx_free(ctx, ctx->wsRef, ctx->capRef);
    ctx_free(ctx, ctx->wsCen, ctx->capCen);
    ctx_free(ctx, ctx->tab, ctx->capTab);
    if (ctx->tabHost) (void)hipHostFree(ctx->tabHost);
    if (ctx->tabCopied) (void)hipEventDestroy(ctx->tabCopied);
    if (ctx->tabRead) (void)hipEventDestroy(ctx->tabRead);
    if (ctx->wsDone) (void)hipEventDestroy(ctx->wsDone);
    delete ctx;
    return PRECODE_OK;
}

int precode_validate(int arch, float rho, const int *cluster_sizes, int C, int mode, int B, int U, int n_sc, int K,
                     const precode_params *params) {
    const precode_params q = params ? *params : defaults();
    Prob p;
    return make_prob(arch, rho, cluster_sizes, C, mode, B, U, n_sc, K, q, &p);
}

size_t precode_ctx_bytes(const precode_ctx *ctx) { return ctx ? ctx->held : 0; }

int precode_ctx_last_impl(const precode_ctx *ctx) { return ctx ? ctx->last_impl : 0; }

int precode_ctx_last_waves(const precode_ctx *ctx) { return ctx ? ctx->last_waves : 0; }

int precode_pd(precode_ctx *ctx, const void *H, const void *s, float rho, const int *cluster_sizes, int C, int mode,
               int B, int U, int n_sc, int K, const precode_params *params, void *x, float *beta, int *status,
               void *stream) {
    return run(ctx, kPD, H, s, rho, cluster_sizes, C, mode, B, U, n_sc, K, params, x, beta, status, stream);
}

int precode_fd(precode_ctx *ctx, const void *H, const void *s, float rho, const int *cluster_sizes, int C, int mode,
               int B, int U, int n_sc, int K, const precode_params *params, void *x, float *weights, int *status,
               void *stream) {
    return run(ctx, kFD, H, s, rho, cluster_sizes, C, mode, B, U, n_sc, K, params, x, weights, status, stream);
}

int precode_central(precode_ctx *ctx, const void *H, const void *s, float rho, int B, int U, int n_sc, int K,
                    const precode_params *params, void *x, float *beta, int *status, void *stream) {
    if (!ctx) return PRECODE_EINVAL;
    const precode_params q = params ? *params : defaults();
    int rc = check_params(q);
    if (rc) return rc;
    if (U < 1 || B < 1 || n_sc < 0 || K < 0) return PRECODE_EINVAL;
    if (!isfinite(rho) || rho < 0.f) return PRECODE_EINVAL;
    // the B x B form needs kappa > 0 (H H^H is singular for B > U); FP32 only
    if (!(rho > 0.f) || q.precision != PRECODE_PREC_FP32) return PRECODE_EUNSUPPORTED;
    if (B > kMaxB || U > kMaxU || K > kMaxK || !central_supported(B, U)) return PRECODE_EUNSUPPORTED;
    if (n_sc == 0) return PRECODE_OK;
    if (!H || (K > 0 && (!s || !x))) return PRECODE_EINVAL;
    if (!aligned8(H) || !aligned8(s) || !aligned8(x)) return PRECODE_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    // factor tiles for up to 256 MiB of subcarriers per launch
    const size_t per = central_ws_bytes(B, 1);
    const size_t chunk = std::max<size_t>(1, std::min<size_t>((size_t)n_sc, (size_t(256) << 20) / per));
    rc = grow(ctx, &ctx->wsCen, &ctx->capCen, chunk * per, st);
    if (!rc) rc = ws_acquire(ctx, st);
    if (rc) return rc;
    rc = dev_err(central_run(B, U, n_sc, K, rho, q.Es, q.power, (const float2 *)H, (const float2 *)s, (float2 *)x,
                             beta, status, ctx->wsCen, chunk * per, st));
    const int rr = ws_release(ctx, st);
    return rc ? rc : rr;
}

int precode_mrt(precode_ctx *ctx, const void *H, const void *s, const int *cluster_sizes, int C, int B, int U,
                int n_sc, int K, const precode_params *params, void *x, float *weights, int *status, void *stream) {
    if (!ctx) return PRECODE_EINVAL;
    const precode_params q = params ? *params : defaults();
    Prob p;
    int rc = make_prob(kFD, 0.f, cluster_sizes, C, PRECODE_ZF, B, U, n_sc, K, q, &p);
    if (rc) return rc;
    if (q.precision != PRECODE_PREC_FP32) return PRECODE_EUNSUPPORTED;
    if (n_sc == 0) return PRECODE_OK;
    if (!H || (K > 0 && (!s || !x))) return PRECODE_EINVAL;
    if (!aligned8(H) || !aligned8(s) || !aligned8(x)) return PRECODE_EINVAL;
    return dev_err(mrt_run(p, (const float2 *)H, (const float2 *)s, (float2 *)x, weights, status, (hipStream_t)stream));
}

static int qam_half_bits(int order) {
    for (int hb = 1; hb <= 8; ++hb)
        if (order == 1 << (2 * hb)) return hb;
    return 0;
}

int precode_qam_map(const int *labels, long long n, int order, void *s, void *stream) {
    const int hb = qam_half_bits(order);
    if (!hb || n < 0) return PRECODE_EINVAL;
    if (n > 0 && (!labels || !s || !aligned8(s))) return PRECODE_EINVAL;
    return dev_err(qam_map_run(labels, n, hb, (float2 *)s, (hipStream_t)stream));
}

int precode_ue_receive(const void *H, const void *x, const void *noise, float N0, const float *scale, int B, int U,
                       int n_sc, int K, void *s_hat, void *stream) {
    if (B < 1 || U < 1 || U > kMaxU || n_sc < 0 || K < 0) return PRECODE_EINVAL;
    if (!isfinite(N0) || N0 < 0.f) return PRECODE_EINVAL;
    if (n_sc == 0 || K == 0) return PRECODE_OK;
    if (!H || !x || !s_hat) return PRECODE_EINVAL;
    if (!aligned8(H) || !aligned8(x) || !aligned8(noise) || !aligned8(s_hat)) return PRECODE_EINVAL;
    return dev_err(ue_receive_run((const float2 *)H, (const float2 *)x, (const float2 *)noise, N0, scale, B, U, n_sc,
                                  K, (float2 *)s_hat, (hipStream_t)stream));
}

int precode_ue_gain(const void *y_pilot, float N0, float Es, int U, int n_sc, float *beta, void *stream) {
    if (U < 1 || n_sc < 0 || !isfinite(N0) || N0 < 0.f || !isfinite(Es) || !(Es > 0.f)) return PRECODE_EINVAL;
    if (n_sc == 0) return PRECODE_OK;
    if (!y_pilot || !beta || !aligned8(y_pilot)) return PRECODE_EINVAL;
    return dev_err(ue_gain_run((const float2 *)y_pilot, N0, Es, U, n_sc, beta, (hipStream_t)stream));
}

int precode_qam_errors(const void *s_hat, const int *labels, long long n, int order, int *labels_out,
                       unsigned long long *bit_errors, void *stream) {
    const int hb = qam_half_bits(order);
    if (!hb || n < 0) return PRECODE_EINVAL;
    if (n > 0 && (!s_hat || !labels || !aligned8(s_hat))) return PRECODE_EINVAL;
    return dev_err(qam_errors_run((const float2 *)s_hat, labels, n, hb, labels_out, bit_errors, (hipStream_t)stream));
}

int precode_frame_prepare(precode_ctx *ctx, int arch, const void *H, float rho, const int *cluster_sizes, int C,
                          int mode, int B, int U, int n_sc, const precode_params *params, precode_frame **out,
                          void *stream) {
    if (!ctx || !out) return PRECODE_EINVAL;
    *out = nullptr;
    const precode_params q = params ? *params : defaults();
    Prob p;
    int rc = make_prob(arch, rho, cluster_sizes, C, mode, B, U, n_sc, 1, q, &p);
    if (rc) return rc;
    if (n_sc > 0 && (!H || !aligned8(H))) return PRECODE_EINVAL;
    const bool fuse = q.impl != PRECODE_IMPL_PLAIN && q.refine_steps == 0 && fused_supported(p, q.precision);
    // the shapes the register-tile kernels do not take (and refinement on
    // them: the FP64 solve needs none) on the wide FP64 kernel
    const bool wide = !fuse && q.impl != PRECODE_IMPL_PLAIN && !(q.refine_steps > 0 && fused_supported(p, q.precision)) &&
                      wide_supported(p, 1);
    if (q.impl == PRECODE_IMPL_FUSED && !fuse && !wide) return PRECODE_EUNSUPPORTED;
    if ((q.precision == PRECODE_PREC_SPLIT_FP16 || q.precision == PRECODE_PREC_SPLIT_BF16) && !fuse && !wide)
        return PRECODE_EUNSUPPORTED;
    // resident state: factors (fused / wide: scale * A^-1; plain: A^-1 slots
    // and scale), beta / weights and status
    const size_t ni = (size_t)n_inst(p);
    const size_t bA = fuse ? ni * p.U * p.U * sizeof(float2) : (wide ? wide_factor_bytes(p) : plain_ws_bytes_A(p));
    const size_t bS = fuse || wide ? 0 : plain_ws_bytes_scale(p);
    const size_t bytes = bA + bS + ni * sizeof(float) + ni * sizeof(int) + 64;
    precode_frame *f = new (std::nothrow) precode_frame;
    if (!f) return PRECODE_ENOMEM;
    memset(f, 0, sizeof(*f));
    rc = ctx_alloc(ctx, &f->ainv, bytes);
    if (rc) {
        delete f;
        return rc;
    }
    f->bytes = bytes;
    f->prob = p;
    f->H = (const float2 *)H;
    f->fused = fuse;
    f->wide = wide;
    f->precision = q.precision;
    f->refine = q.refine_steps;
    f->scale = (char *)f->ainv + bA;
    f->scale_out = (float *)((char *)f->scale + bS);
    f->status = (int *)((char *)f->scale_out + ((ni * sizeof(float) + 7) & ~(size_t)7));
    if (n_sc > 0) {
        if (fuse) {
            rc = dev_err(fused_prepare(p, q.precision, (const float2 *)H, (float2 *)f->ainv, f->scale_out, f->status,
                                       (hipStream_t)stream));
        } else if (wide) {
            rc = dev_err(wide_prepare(p, (const float2 *)H, f->ainv, f->scale_out, f->status, (hipStream_t)stream));
        } else {
            rc = grow(ctx, &ctx->wsA, &ctx->capA, bA, (hipStream_t)stream);
            if (!rc) rc = ws_acquire(ctx, (hipStream_t)stream);
            if (!rc) {
                rc = dev_err(plain_prepare(p, (const float2 *)H, f->scale_out, f->status, ctx->wsA, f->ainv,
                                           f->scale, (hipStream_t)stream));
                const int rr = ws_release(ctx, (hipStream_t)stream);
                if (!rc) rc = rr;
            }
        }
    }
    if (rc) {
        ctx_free(ctx, f->ainv, f->bytes);
        delete f;
        return rc;
    }
    if (rc == PRECODE_OK) ctx->last_impl = fuse || wide ? PRECODE_IMPL_FUSED : PRECODE_IMPL_PLAIN;
    f->next = ctx->frames;
    ctx->frames = f;
    *out = f;
    return PRECODE_OK;
}

int precode_frame_symbols(precode_ctx *ctx, precode_frame *f, const void *s, int nk, void *x, void *stream) {
    if (!ctx || !f) return PRECODE_EINVAL;
    if (nk < 0) return PRECODE_EINVAL;
    if (nk > kMaxK) return PRECODE_EUNSUPPORTED;
    if (nk == 0 || f->prob.n_sc == 0) return PRECODE_OK;
    if (!s || !x || !aligned8(s) || !aligned8(x)) return PRECODE_EINVAL;
    Prob p = f->prob;
    p.K = nk;
    if (f->fused)
        return dev_err(fused_symbols(p, f->precision, nk, f->H, (const float2 *)f->ainv, f->status,
                                     (const float2 *)s, (float2 *)x, (hipStream_t)stream));
    if (f->wide)
        return dev_err(wide_symbols(p, nk, f->H, f->ainv, f->status, (const float2 *)s, (float2 *)x,
                                    (hipStream_t)stream));
    hipStream_t st = (hipStream_t)stream;
    int rc = grow(ctx, &ctx->wsZ, &ctx->capZ, plain_ws_bytes_z(p, nk), st);
    if (!rc) rc = ws_acquire(ctx, st);
    if (rc) return rc;
    rc = dev_err(plain_symbols(p, nk, f->H, (const float2 *)s, (float2 *)x, f->ainv, f->scale, ctx->wsZ, st,
                               f->refine));
    const int rr = ws_release(ctx, st);
    return rc ? rc : rr;
}

int precode_frame_factors(precode_ctx *ctx, precode_frame *f, float *scale, int *status, void *stream) {
    if (!ctx || !f) return PRECODE_EINVAL;
    const size_t ni = (size_t)n_inst(f->prob);
    hipStream_t st = (hipStream_t)stream;
    if (ni == 0) return PRECODE_OK;
    hipError_t e = hipSuccess;
    if (scale) e = hipMemcpyAsync(scale, f->scale_out, ni * sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && status) e = hipMemcpyAsync(status, f->status, ni * sizeof(int), hipMemcpyDeviceToDevice, st);
    return dev_err(e);
}

int precode_frame_release(precode_ctx *ctx, precode_frame *f) {
    if (!ctx || !f) return PRECODE_EINVAL;
    precode_frame **pp = &ctx->frames;
    while (*pp && *pp != f) pp = &(*pp)->next;
    if (!*pp) return PRECODE_EINVAL;
    *pp = f->next;
    // work enqueued on any stream may still read the frame's state
    (void)hipDeviceSynchronize();
    ctx_free(ctx, f->ainv, f->bytes);
    delete f;
    return PRECODE_OK;
}

int precode_batch(precode_ctx *ctx, const precode_job *jobs, int n_jobs, int precision, void *stream) {
    if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs)) return PRECODE_EINVAL;
    std::vector<BatchProblem> fused;
    std::vector<std::pair<int, Prob>> plain;
    int rc = classify(jobs, n_jobs, precision, &fused, &plain);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = fused.empty() ? 0 : fused_batch_table_bytes(fused.data(), (int)fused.size());
    if (!fused.empty() && bytes == 0) {
        // one-wave FP64 problems only: no table
        if (hipSetDevice(ctx->device) != hipSuccess) return PRECODE_EDEVICE;
        int nl = 0;
        if (fused_batch_launch(fused.data(), (int)fused.size(), precision, nullptr, st, &nl) != hipSuccess)
            return PRECODE_EDEVICE;
        ctx->last_impl = PRECODE_IMPL_FUSED;
        ctx->last_waves = fused_default_waves();
    }
    if (bytes > 0) {
        if (hipSetDevice(ctx->device) != hipSuccess) return PRECODE_EDEVICE;
        if (!ctx->tabCopied) {
            if (hipEventCreateWithFlags(&ctx->tabCopied, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&ctx->tabRead, hipEventDisableTiming) != hipSuccess)
                return PRECODE_EDEVICE;
            if (hipEventRecord(ctx->tabCopied, st) != hipSuccess || hipEventRecord(ctx->tabRead, st) != hipSuccess)
                return PRECODE_EDEVICE;
        }
        // the staging buffer may still be the source of the previous copy
        if (hipEventSynchronize(ctx->tabCopied) != hipSuccess) return PRECODE_EDEVICE;
        if (ctx->capTabHost < bytes) {
            if (ctx->tabHost) (void)hipHostFree(ctx->tabHost);
            ctx->tabHost = nullptr;
            ctx->capTabHost = 0;
            if (hipHostMalloc(&ctx->tabHost, bytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return PRECODE_ENOMEM;
            }
            ctx->capTabHost = bytes;
        }
        rc = grow(ctx, &ctx->tab, &ctx->capTab, bytes, st);
        if (rc) return rc;
        fused_batch_fill(fused.data(), (int)fused.size(), ctx->tabHost);
        // the device table may still be read by the previous batch's launches
        hipError_t e = hipStreamWaitEvent(st, ctx->tabRead, 0);
        if (e == hipSuccess) e = hipMemcpyAsync(ctx->tab, ctx->tabHost, bytes, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(ctx->tabCopied, st);
        int nl = 0;
        if (e == hipSuccess) e = fused_batch_launch(fused.data(), (int)fused.size(), precision, ctx->tab, st, &nl);
        if (e == hipSuccess) e = hipEventRecord(ctx->tabRead, st);
        if (e != hipSuccess) return PRECODE_EDEVICE;
        ctx->last_impl = PRECODE_IMPL_FUSED;
        ctx->last_waves = fused_default_waves();
    }
    for (const auto &pp : plain) {
        const Prob &p = pp.second;
        rc = grow(ctx, &ctx->wsA, &ctx->capA, plain_ws_bytes_A(p), st);
        if (!rc) rc = grow(ctx, &ctx->wsAinv, &ctx->capAinv, plain_ws_bytes_A(p), st);
        if (!rc) rc = grow(ctx, &ctx->wsScale, &ctx->capScale, plain_ws_bytes_scale(p), st);
        if (!rc) rc = grow(ctx, &ctx->wsZ, &ctx->capZ, plain_ws_bytes_z(p, p.K > 0 ? p.K : 1), st);
        if (!rc) rc = ws_acquire(ctx, st);
        if (!rc) {
            rc = run_plain(p, jobs[pp.first], ctx->wsA, ctx->wsAinv, ctx->wsScale, ctx->wsZ, st);
            const int rr = ws_release(ctx, st);
            if (!rc) rc = rr;
        }
        if (rc) return rc;
        if (fused.empty()) ctx->last_impl = PRECODE_IMPL_PLAIN;
    }
    return PRECODE_OK;
}

int precode_batch_plan_create(precode_ctx *ctx, const precode_job *jobs, int n_jobs, int precision,
                              precode_batch_plan **out) {
    if (!ctx || !out || n_jobs < 0 || (n_jobs > 0 && !jobs)) return PRECODE_EINVAL;
    *out = nullptr;
    std::vector<BatchProblem> fused;
    std::vector<std::pair<int, Prob>> plain;
    int rc = classify(jobs, n_jobs, precision, &fused, &plain);
    if (rc) return rc;
    if (hipSetDevice(ctx->device) != hipSuccess) return PRECODE_EDEVICE;
    precode_batch_plan *pl = new (std::nothrow) precode_batch_plan;
    if (!pl) return PRECODE_ENOMEM;
    memset(pl, 0, sizeof(*pl));
    pl->ctx = ctx;
    auto fail = [&](int code) {
        precode_batch_plan_destroy(pl);
        return code;
    };
    // the slice table, uploaded once (synchronous copy)
    pl->tabBytes = fused.empty() ? 0 : fused_batch_table_bytes(fused.data(), (int)fused.size());
    if (pl->tabBytes > 0) {
        std::vector<char> host(pl->tabBytes);
        fused_batch_fill(fused.data(), (int)fused.size(), host.data());
        rc = ctx_alloc(ctx, &pl->tab, pl->tabBytes);
        if (rc) return fail(rc);
        if (hipMemcpy(pl->tab, host.data(), pl->tabBytes, hipMemcpyHostToDevice) != hipSuccess)
            return fail(PRECODE_EDEVICE);
    }
    // plain-kernel workspace of the plan (its jobs run one after another)
    for (const auto &pp : plain) {
        pl->bA = std::max(pl->bA, plain_ws_bytes_A(pp.second));
        pl->bS = std::max(pl->bS, plain_ws_bytes_scale(pp.second));
        pl->bZ = std::max(pl->bZ, plain_ws_bytes_z(pp.second, pp.second.K > 0 ? pp.second.K : 1));
    }
    if (!plain.empty()) {
        rc = ctx_alloc(ctx, &pl->wsA, pl->bA);
        if (!rc) rc = ctx_alloc(ctx, &pl->wsAinv, pl->bA);
        if (!rc) rc = ctx_alloc(ctx, &pl->wsScale, pl->bS);
        if (!rc) rc = ctx_alloc(ctx, &pl->wsZ, pl->bZ);
        if (rc) return fail(rc);
    }
    // record every launch into one graph
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(PRECODE_EDEVICE);
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int nl = 0;
    if (e == hipSuccess && !fused.empty())
        e = fused_batch_launch(fused.data(), (int)fused.size(), precision, pl->tab, cs, &nl);
    for (size_t i = 0; e == hipSuccess && i < plain.size(); ++i) {
        if (run_plain(plain[i].second, jobs[plain[i].first], pl->wsA, pl->wsAinv, pl->wsScale, pl->wsZ, cs))
            e = hipErrorUnknown;
        else
            nl += plain[i].second.K > 0 ? 4 : 2;
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = ee;
    (void)hipStreamDestroy(cs);
    pl->graph = g;
    if (e == hipSuccess && g) e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PRECODE_EDEVICE);
    }
    pl->launches = nl;
    for (const auto &b : fused)
        if (b.p.n_sc > 0) ++pl->fused_jobs;
    *out = pl;
    return PRECODE_OK;
}

int precode_batch_plan_launch(precode_batch_plan *plan, void *stream) {
    if (!plan) return PRECODE_EINVAL;
    if (!plan->exec) return PRECODE_OK;
    return dev_err(hipGraphLaunch(plan->exec, (hipStream_t)stream));
}

int precode_batch_plan_launches(const precode_batch_plan *plan) { return plan ? plan->launches : 0; }

int precode_batch_plan_fused_jobs(const precode_batch_plan *plan) { return plan ? plan->fused_jobs : 0; }

void precode_autotune_reset(void) { fused_autotune_reset(); }

int precode_batch_plan_destroy(precode_batch_plan *plan) {
    if (!plan) return PRECODE_EINVAL;
    precode_ctx *ctx = plan->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    ctx_free(ctx, plan->tab, plan->tabBytes);
    ctx_free(ctx, plan->wsA, plan->bA);
    ctx_free(ctx, plan->wsAinv, plan->bA);
    ctx_free(ctx, plan->wsScale, plan->bS);
    ctx_free(ctx, plan->wsZ, plan->bZ);
    delete plan;
    return PRECODE_OK;
}

}  // extern "C"
