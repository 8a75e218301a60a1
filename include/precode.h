/*
 * precode.h -- C ABI of the MI355X (gfx950) decentralized precoding library.
 *
 * Method: K. Li, C. Jeon, J. R. Cavallaro, C. Studer, "Feedforward
 * Architectures for Decentralized Precoding in Massive MU-MIMO Systems",
 * arXiv:1804.10987.  Partially decentralized (PD) Wiener-filter / ZF
 * precoding of Sec. III-B and fully decentralized (FD) precoding of
 * Sec. III-C, batched over OFDM subcarriers (Sec. IV-B) on one GPU: the
 * paper's antenna clusters (one per GPU there) are batch entries here.
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Complex values are complex64: interleaved {float re, float im}, 8 bytes.
 *  - The channel of subcarrier n is stored as H[n] = B x U, row-major
 *    (antenna rows, user columns).  This is the Hermitian transpose of the
 *    paper's U x B downlink matrix (downlink model, Sec. II-A), so the
 *    paper's local Gram H_c H_c^H is H_c^H H_c here and the per-cluster
 *    product H_c^H z is H_c z here.  Cluster c owns the contiguous antenna
 *    rows [o_c, o_c + B_c), o_c = B_0 + ... + B_{c-1} (Sec. III-A).
 *  - Tensors (all DEVICE pointers, owned by the caller, 8-byte aligned):
 *        H  [n_sc][B][U]      channel, constant over the K symbols of a frame
 *        s  [K][n_sc][U]      transmit symbols (symbol-major)
 *        x  [K][n_sc][B]      precoded vectors (output)
 *  - `rho` is the WF regularizer kappa = U N0 / rho^2 of Theorem 1
 *    (eq. precodingfactor); it is ignored for ZF (kappa = 0).
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL = the default stream) and return after enqueueing.  A context is
 *    not thread-safe: use one context per host thread.  The plain kernels'
 *    workspace is one per context: plain-path calls of one context on
 *    different streams are ordered by the library (each waits for the
 *    previous one's use of it), so they do not overlap on the device.  Under
 *    stream capture that workspace must already be large enough (an earlier
 *    uncaptured call of the same or a larger shape), else
 *    PRECODE_EUNSUPPORTED; a captured call is ordered by its capture only.
 *  - Errors detectable on the host are returned before anything is
 *    launched.  Per-instance numerical failures are reported asynchronously
 *    through `status` (see PRECODE_ST_*), never through the return code.
 */
#ifndef PRECODE_H
#define PRECODE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define PRECODE_OK 0
#define PRECODE_EINVAL (-1)       /* bad shape, pointer, size or parameter        */
#define PRECODE_EUNSUPPORTED (-2) /* U > 64, B > 4096, K > 4096, ...              */
#define PRECODE_ENOMEM (-3)       /* context workspace over its HBM budget        */
#define PRECODE_EDEVICE (-4)      /* a HIP runtime error                          */

/* ---- per-instance status values (bit flags, written asynchronously) ---- */
/* An instance whose FP32 factorization fails (a pivot not above 2^-20 of
 * its original diagonal entry, a non-finite value, or Lemma 1's t <= 0) is
 * solved again on the FP64 route in the same call: FP64 Gram, Cholesky
 * factorization, solve and precode (Theorem 1 only needs A invertible).  It
 * is flagged PRECODE_ST_FAIL only if the FP64 factorization fails as well
 * (a pivot not above 2^-40 of its original diagonal entry, or t <= 0). */
#define PRECODE_ST_OK 0   /* solved                                          */
#define PRECODE_ST_FAIL 1 /* numerically singular on the FP64 route as well  */
                          /* (always with PRECODE_ST_FP64): x is set to 0,   */
                          /* beta / weight to 0                              */
#define PRECODE_ST_FP64 2 /* solved on the FP64 route: routed there by       */
                          /* fp64_ratio / precision FP64, or retried there   */
                          /* after its FP32 factorization failed             */

/* ---- enums ---------------------------------------------------------------- */
enum precode_mode { PRECODE_ZF = 0, PRECODE_WF = 1 };
enum precode_arch { PRECODE_ARCH_PD = 0, PRECODE_ARCH_FD = 1 };
enum precode_prec {
    PRECODE_PREC_FP32 = 0,       /* FP32 MFMA Gram and precode, FP32 factorization   */
    PRECODE_PREC_SPLIT_FP16 = 1, /* Gram / precode as hi+lo FP16 MFMA, FP32 accum.   */
    PRECODE_PREC_SPLIT_BF16 = 2, /* Gram / precode as hi+lo BF16 MFMA, FP32 accum.   */
    PRECODE_PREC_FP64 = 3        /* every instance on the FP64 route                 */
};
enum precode_impl {
    PRECODE_IMPL_AUTO = 0,  /* fused single-launch kernel where supported, else plain */
                            /* (with K >= 1 every shape has one: the register-tile   */
                            /* kernels for U <= 32 on the FP32 route, the one-wave   */
                            /* FP64 kernel for FP64-route systems with U <= 32 and   */
                            /* U <= B_eff <= 64, else a wide FP64 kernel, one        */
                            /* workgroup per local system of order <= 64, that takes */
                            /* U in 33..64, FD clusters with B_c < U, mixed routes   */
                            /* and precision FP64, its systems flagged FP64)         */
    PRECODE_IMPL_FUSED = 1, /* fused kernel; PRECODE_EUNSUPPORTED if the shape is not */
    PRECODE_IMPL_PLAIN = 2  /* separate plain FP32/FP64 kernels (no MFMA, no fusion)  */
};

/* ---- optional parameters (NULL => defaults from precode_params_init) ---- */
typedef struct precode_params {
    float power;       /* rho^2, the power budget E||x||^2 <= rho^2 (Sec. II-A); 1 */
    float Es;          /* symbol energy E_s (Theorem 1, Lemma 1); 1                */
    float tau;         /* FD regularization factor tau_c (eq. regularization);     */
                       /* 0.125, the value the paper's simulations settle on       */
    int precision;     /* enum precode_prec; PRECODE_PREC_FP32                     */
    int refine_steps;  /* 0 or 1 steps of iterative refinement of the U x U solve */
                       /* (PD; FD clusters with B_c >= U): residual               */
                       /* s - (kappa y + H^H (H y)) accumulated in FP64 from the  */
                       /* complex64 channel, y += A^-1 r.  Shapes the fused      */
                       /* kernel takes run the fused factorization at the call's */
                       /* precision, then one fused refine-and-precode launch    */
                       /* (the FP64 Gram gives the exact residual); a call whose */
                       /* systems all take the fused FP64 route runs it (an FP64 */
                       /* solve needs no refinement); others run the plain       */
                       /* kernels.  beta / weights are not refined; 0            */
    float fp64_ratio;  /* an instance whose local system has U / B_eff >= ratio is */
                       /* solved on the FP64 route (B_eff = B for PD, B_c for FD); */
                       /* 0.5; a value > 1 disables the route                      */
    int impl;          /* enum precode_impl; PRECODE_IMPL_AUTO                     */
    /* FD and MRT only (PD ignores them); HOST arrays of C values read during  */
    /* the call, or NULL; either one needs C <= 64:                             */
    const float *cluster_tau;    /* tau_c >= 0 per cluster (eq. regularization); */
                                 /* NULL: tau for every cluster                  */
    const float *cluster_power;  /* budgets rho_c^2 > 0 summing to power       */
                                 /* (relative 1e-5), the unequal allocations the */
                                 /* power footnote of Sec. III-C considers;      */
                                 /* NULL: rho^2 / C each.  Then                  */
                                 /* kappa_c = tau_c U N0 / rho_c^2               */
                                 /*         = tau_c kappa rho^2 / rho_c^2 and    */
                                 /* w_c = sqrt(rho_c^2 / (t_c Es))               */
} precode_params;

typedef struct precode_ctx precode_ctx;
typedef struct precode_frame precode_frame;

/* Fills *p with the defaults listed above. */
void precode_params_init(precode_params *p);

/* Human-readable text for a return code (static storage). */
const char *precode_strerror(int code);

/* Checks a PD (arch = PRECODE_ARCH_PD) or FD call's scalar arguments exactly
 * as precode_pd / precode_fd do, without touching any device: returns the
 * code those calls would return for these arguments (pointer checks aside).
 * params may be NULL (defaults). */
int precode_validate(int arch, float rho, const int *cluster_sizes, int C, int mode, int B,
                     int U, int n_sc, int K, const precode_params *params);

/* Creates a context on HIP device `device`.  The context owns the workspace
 * used by the plain kernels, the refinement step and the resident state of
 * frames; its total device allocation never exceeds `hbm_budget_bytes`
 * (0 = unlimited).  *out receives the handle. */
int precode_ctx_create(int device, size_t hbm_budget_bytes, precode_ctx **out);

/* Frees the context's workspace (after synchronizing its device). */
int precode_ctx_destroy(precode_ctx *ctx);

/* Bytes of device memory the context currently holds. */
size_t precode_ctx_bytes(const precode_ctx *ctx);

/* Path taken by the most recent successful call on this context
 * (1 = fused, 2 = plain), or 0 if none. */
int precode_ctx_last_impl(const precode_ctx *ctx);

/* Waves per workgroup (1, 2 or 4) of the most recent fused precode_pd /
 * precode_fd / precode_batch call on this context, or 0 if none.  The
 * register-tile kernels' launch shape (waves per workgroup, and register
 * tiles or channel rows streamed twice) is chosen by an autotuner that times
 * every feasible shape on the first call of each problem shape (the call's
 * own launch, repeated on its stream, before the call returns; streamed
 * shapes only when the channel exceeds the 256 MB last-level cache or no
 * tiles fit) and reuses the fastest.  Tuned shapes are kept for the process
 * and appended to a cache file keyed by device (architecture, name, compute
 * units) and HIP runtime version, which later processes read instead of
 * timing again: PRECODE_TUNE_CACHE=path names it ("off": no file; unset:
 * $XDG_CACHE_HOME/precode/tune.txt, else $HOME/.cache/precode/tune.txt;
 * lines "<device> <problem shape> <waves> <streamed>").
 * PRECODE_FUSED_WAVES=1|2|4 in the environment forces the waves,
 * PRECODE_AUTOTUNE=0 keeps the default shape (the fewest waves per
 * workgroup that keep the rows in registers; at 17 to 32 users the fewest
 * that stream them, for PD systems whose rows need a whole workgroup);
 * PRECODE_FUSED_STREAM=1 makes every wave stream its channel rows twice
 * instead of keeping them in registers.  Calls made under stream capture
 * never tune.  Shapes differ only in the order of the cluster-sum rounding. */
int precode_ctx_last_waves(const precode_ctx *ctx);

/* Forgets every launch shape the process has tuned or read; the next call
 * of each problem shape reads the cache file again (then tunes if absent). */
void precode_autotune_reset(void);

/* ---------------------------------------------------------------------------
 * PD precoding of a frame (Sec. III-B; Theorem 1; Lemma 1).  Per subcarrier
 * n (n < n_sc):
 *     G = sum_c H_c^H H_c,   A = G + kappa I_U,
 *     beta = sqrt(Es / power * (tr A^-1 - kappa ||A^-1||_F^2)),
 *     z_k = A^-1 s_k / beta,  x_c,k = H_c z_k   for all K symbols k.
 * cluster_sizes: HOST array of C positive ints summing to B.
 * mode: PRECODE_ZF or PRECODE_WF.  beta: device [n_sc] or NULL.
 * status: device [n_sc] int or NULL.
 * Limits: 1 <= U <= 64, 1 <= B <= 4096, 1 <= C <= min(B, 256),
 * 0 <= K <= 4096, n_sc >= 0 (n_sc = 0 or K = 0 precodes nothing).
 * rho must be finite and >= 0 for WF.
 * ------------------------------------------------------------------------- */
int precode_pd(precode_ctx *ctx, const void *H, const void *s, float rho,
               const int *cluster_sizes, int C, int mode, int B, int U, int n_sc,
               int K, const precode_params *params, void *x, float *beta,
               int *status, void *stream);

/* ---------------------------------------------------------------------------
 * precode_pd without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Arguments, outputs and routing as precode_pd.  The
 * workspace a call needs (the fused refinement's factors, or the plain
 * kernels' workspace) comes from a fixed 64 MiB device array of the library,
 * one per GPU, held until the process ends; a call needing more returns
 * PRECODE_ENOMEM before anything is enqueued.  The call allocates nothing,
 * creates no event and times no launch shape (an untuned shape uses the
 * default launch shape).  All calls on one GPU share that array: calls that
 * overlap on one GPU race.
 * ------------------------------------------------------------------------- */
int precode_pd_noalloc(precode_ctx *ctx, const void *H, const void *s, float rho,
                       const int *cluster_sizes, int C, int mode, int B, int U, int n_sc,
                       int K, const precode_params *params, void *x, float *beta,
                       int *status, void *stream);

/* ---------------------------------------------------------------------------
 * Centralized WF precoding in the B x B form of Theorem 1 (Sec. II-B), the
 * reference the PD architecture must equal (Sec. III-D):
 *     M = H H^H + kappa I_B,  Q = M^-1 H  (eq. originalQmatrix),
 *     beta = sqrt(tr(Q^H Q) Es / rho^2)  (eq. precodingfactor),  x = Q s / beta,
 * with H = H_dl^H as everywhere in this library and kappa = rho (> 0: the
 * B x B form has no ZF case for B > U).  FP32 Cholesky of M by 32 x 32
 * tiles, one workgroup per subcarrier; the context holds the factor tiles
 * (up to 256 MiB, launches chunked).  Layouts, beta and status as precode_pd
 * (PRECODE_ST_FAIL with x = 0 on a pivot not above 2^-20 of its diagonal
 * entry; no FP64 route).  params: power and Es; precision must be FP32.
 * PRECODE_EUNSUPPORTED for kappa = 0 or shapes whose factor tiles and Q do
 * not fit (about (B + 32) (U + 1) <= 18000).
 * ------------------------------------------------------------------------- */
int precode_central(precode_ctx *ctx, const void *H, const void *s, float rho, int B, int U,
                    int n_sc, int K, const precode_params *params, void *x, float *beta,
                    int *status, void *stream);

/* ---------------------------------------------------------------------------
 * Maximum ratio transmission, the fully distributed comparison precoder of
 * Sec. I and Sec. III-D: the matched filter Q_c = H_c with the per-cluster
 * power normalization of Sec. III-C,
 *     x_c = sqrt(rho_c^2 / (||H_c||_F^2 Es)) H_c s,   rho_c^2 = rho^2 / C
 * (C = 1: centralized MRT).  weights [n_sc][C] receive the factors; a
 * cluster with a zero channel gets status PRECODE_ST_FAIL, weight 0, x_c = 0.
 * params: power and Es; precision must be FP32.
 * ------------------------------------------------------------------------- */
int precode_mrt(precode_ctx *ctx, const void *H, const void *s, const int *cluster_sizes,
                int C, int B, int U, int n_sc, int K, const precode_params *params, void *x,
                float *weights, int *status, void *stream);

/* ---------------------------------------------------------------------------
 * The UE side of the uncoded-BER link (Sec. III-D; downlink model of
 * Sec. II-A, UE scaling of Sec. II-B).  Device pointers, asynchronous on
 * `stream`, no context.
 *
 * precode_qam_map: labels [n] (int32 in [0, order); higher bits ignored) to
 * unit-energy square QAM points s [n] (complex64).  The upper half of a
 * label's log2(order) bits is the binary-reflected Gray code of the in-phase
 * level, the lower half that of the quadrature level; level i of
 * m = sqrt(order) sits at (2 i - (m - 1)) d, d = sqrt(3 / (2 (order - 1))).
 * order = 4, 16, 64, ..., 65536.
 *
 * precode_ue_receive: s_hat[k][n][u] = scale[n] (sum_b conj(H[n][b][u])
 * x[k][n][b] + sqrt(N0) noise[k][n][u]), i.e. y = H_dl x + n scaled by the
 * UE factor.  noise [K][n_sc][U] complex64 of unit variance per complex
 * entry, or NULL (noise-free); scale [n_sc] float or NULL (1).
 *
 * precode_ue_gain: the joint UE factor minimizing the MSE of Sec. II-B for
 * the precoder in use, from its noise-free responses to the U pilots
 * s = e_v: y_pilot [U][n_sc][U] = precode_ue_receive output for those
 * pilots (scale NULL), E[n][u][v] = y_pilot[v][n][u] = (H_dl P)[u][v],
 * beta[n] = Es Re(tr E) / (Es ||E||_F^2 + U N0).  For the WF precoder this
 * is beta_WF.
 *
 * precode_qam_errors: nearest-point decision of every s_hat (per axis,
 * clamped to the outer levels), its Gray label to labels_out [n] (or NULL),
 * and the number of bits that differ from labels [n] added to the 64-bit
 * device counter *bit_errors (or NULL); the caller clears the counter.
 * ------------------------------------------------------------------------- */
int precode_qam_map(const int *labels, long long n, int order, void *s, void *stream);
int precode_ue_receive(const void *H, const void *x, const void *noise, float N0,
                       const float *scale, int B, int U, int n_sc, int K, void *s_hat,
                       void *stream);
int precode_ue_gain(const void *y_pilot, float N0, float Es, int U, int n_sc, float *beta,
                    void *stream);
int precode_qam_errors(const void *s_hat, const int *labels, long long n, int order,
                       int *labels_out, unsigned long long *bit_errors, void *stream);

/* ---------------------------------------------------------------------------
 * FD precoding of a frame (Sec. III-C).  Per subcarrier and cluster c, with
 * rho_c^2 = power / C and kappa_c = tau C kappa (eq. regularization):
 *     B_c >= U:  A_c = H_c^H H_c + kappa_c I_U,   x_c = w_c H_c A_c^-1 s
 *     B_c <  U:  M_c = H_c H_c^H + kappa_c I_B_c, x_c = w_c M_c^-1 H_c s
 *     w_c = sqrt(rho_c^2 / (t_c Es)),  t_c = tr(Q_c^H Q_c)
 *         = tr X^-1 - kappa_c ||X^-1||_F^2   (X = A_c or M_c).
 * weights: device [n_sc][C] float or NULL.  status: device [n_sc][C] or NULL.
 * Limits as for precode_pd.
 * ------------------------------------------------------------------------- */
int precode_fd(precode_ctx *ctx, const void *H, const void *s, float rho,
               const int *cluster_sizes, int C, int mode, int B, int U, int n_sc,
               int K, const precode_params *params, void *x, float *weights,
               int *status, void *stream);

/* ---------------------------------------------------------------------------
 * Frame / symbol split (the channel is constant over a frame and A^-1, beta
 * are reused across its symbols, Sec. IV-B).  frame_prepare runs the
 * per-frame part (Gram, factorization, beta / weights) once and keeps the
 * result resident in context memory (counted against the budget);
 * frame_symbols precodes nk symbols s[nk][n_sc][U] -> x[nk][n_sc][B] with it.
 * H must stay valid and unchanged until frame_release (it is read by
 * frame_symbols).  arch: enum precode_arch.  The frame handle is owned by
 * the context and freed by frame_release or ctx_destroy.  Routing as for
 * precode_pd / precode_fd: the register-tile kernels keep scale * A^-1 in
 * complex64, the wide FP64 kernel (every other shape with U <= 64, unless
 * impl is PLAIN) in complex FP64 (up to 64 x 64 x 16 bytes per local
 * system), the plain kernels their A^-1 slots.
 * ------------------------------------------------------------------------- */
int precode_frame_prepare(precode_ctx *ctx, int arch, const void *H, float rho,
                          const int *cluster_sizes, int C, int mode, int B, int U,
                          int n_sc, const precode_params *params,
                          precode_frame **out, void *stream);
int precode_frame_symbols(precode_ctx *ctx, precode_frame *frame, const void *s,
                          int nk, void *x, void *stream);
/* Copies the frame's beta (PD, [n_sc]) or weights (FD, [n_sc][C]) and status
 * into caller device buffers (either may be NULL). */
int precode_frame_factors(precode_ctx *ctx, precode_frame *frame, float *scale,
                          int *status, void *stream);
int precode_frame_release(precode_ctx *ctx, precode_frame *frame);

/* ---------------------------------------------------------------------------
 * Heterogeneous batch: n_jobs independent frames (cells with different
 * B, C, U, n_sc, K, mode, regularizer; the batching of Sec. IV's per-
 * subcarrier independence across cells).  Every job is described by one
 * precode_job; pointers are device pointers with the layouts above and the
 * outputs are those of precode_pd / precode_fd for the same job.
 *   - jobs the register-tile kernels take (U <= 32, no FP64 route, FD
 *     clusters with B_c >= U) run as ONE launch per kernel shape class (tile
 *     width U <= 16 or U <= 32, times the channel tiles a wave keeps in
 *     registers: 1, 2, 4 or streamed, times the load width), PD and FD jobs
 *     together;
 *   - jobs whose every local system takes the FP64 route with U <= 32 and
 *     U <= B_eff <= 64 run on the one-wave FP64 kernel, one launch per job;
 *   - every other job with K >= 1 (U in 33..64, FD clusters with B_c < U,
 *     mixed routes, larger FP64-route systems, precision FP64) runs on the
 *     wide FP64 kernel: one launch per system-order class (16, 32, 48, 64;
 *     an FD job's clusters each in their own class) for all such jobs,
 *     every local system flagged PRECODE_ST_FP64;
 *   - the remaining jobs (K = 0) run on the plain kernels after them, on
 *     `stream`.
 * The whole batch is validated before anything is enqueued (first error
 * returned).  With SPLIT precision every job must take one of the fused
 * kernels (PRECODE_EUNSUPPORTED otherwise); jobs on the FP64 kernels compute
 * in FP64.  The slice table is staged through a pinned host buffer of the
 * context; a call may wait on the host for the previous call's table copy.
 * ------------------------------------------------------------------------- */
typedef struct precode_job {
    int arch;                 /* enum precode_arch                         */
    int mode;                 /* enum precode_mode                         */
    int B, U, n_sc, K, C;
    const int *cluster_sizes; /* HOST array of C ints                      */
    float rho;                /* kappa                                     */
    float power, Es, tau;     /* as in precode_params                      */
    const void *H;
    const void *s;
    void *x;
    float *scale;             /* beta [n_sc] (PD) / weights [n_sc][C] (FD) or NULL */
    int *status;              /* [n_sc] (PD) / [n_sc][C] (FD) or NULL      */
} precode_job;

int precode_batch(precode_ctx *ctx, const precode_job *jobs, int n_jobs,
                  int precision, void *stream);

/* Batch plan: the launches of one precode_batch recorded once into a HIP
 * graph, for replay each frame with the same buffers (a serving loop that
 * reuses its H / s / x ring).  create validates as precode_batch, uploads the
 * slice table, allocates the plan's own plain-kernel workspace (counted in
 * the context's budget) and instantiates the graph; every pointer in `jobs`
 * is baked in and must stay valid, with the same shapes, until destroy.
 * launch enqueues one replay on `stream` (asynchronous, no allocation, no
 * host copy).  launches returns the kernel launches one replay holds;
 * fused_jobs the jobs (with n_sc > 0) it runs on the fused kernels rather
 * than the plain ones.  destroy synchronizes the device and frees the plan. */
typedef struct precode_batch_plan precode_batch_plan;
int precode_batch_plan_create(precode_ctx *ctx, const precode_job *jobs, int n_jobs,
                              int precision, precode_batch_plan **out);
int precode_batch_plan_launch(precode_batch_plan *plan, void *stream);
int precode_batch_plan_launches(const precode_batch_plan *plan);
int precode_batch_plan_fused_jobs(const precode_batch_plan *plan);
int precode_batch_plan_destroy(precode_batch_plan *plan);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of per-frame jobs arriving over time.  Each
 * job is one frame of one cell (its precode_job holds all K symbols in s and
 * receives all K outputs in x).  Symbol k of a job is released at
 * arrival_s + k * symbol_period_s (seconds from the start of the call).
 * precode_serve replays the arrival trace in real time and returns when every
 * job has completed:
 *   - an arrived job is admitted (FIFO) when fewer than max_active jobs are in
 *     flight and its resident state (factors, beta / weights, status: scale
 *     A^-1 in complex64 for the register-tile kernels, in complex FP64 for
 *     the wide FP64 kernel, which takes every other job with symbols; the
 *     plain kernels' workspace for jobs without symbols or with impl PLAIN)
 *     fits the slab of slab_bytes of device memory (the HBM budget);
 *   - admission enqueues the per-frame part (Gram, factors, beta / weights,
 *     Sec. IV-B) on one of n_streams streams; released symbols are precoded
 *     from the resident factors as they are released, jobs overlapping on
 *     the device across streams; a job with symbol_period_s == 0 on the
 *     fused kernels is instead precoded in one launch from Gram to precode
 *     (its channel read once);
 *   - a job's state returns to the slab after its last symbol completes.
 * The call allocates the slab and streams once; the loop itself never
 * allocates, and runs no launch-shape timing (see precode_ctx_last_waves): a
 * shape the process has not tuned yet uses the default launch shape.
 * sym_latency (host array of sum_j K_j doubles, job-major, or
 * NULL) receives each symbol's latency: completion observed on the host minus
 * release.  The job's scale / status outputs are filled as for precode_pd /
 * precode_fd.  Returns PRECODE_ENOMEM if a job can never fit the slab.
 * ------------------------------------------------------------------------- */
typedef struct precode_serve_job {
    precode_job job;
    double arrival_s;       /* arrival time, seconds from the start of the call */
    double symbol_period_s; /* OFDM symbol period; 0 releases all K at arrival  */
} precode_serve_job;

typedef struct precode_serve_config {
    int max_active;    /* jobs admitted at once (slots)                        */
    int n_streams;     /* HIP streams the loop spreads jobs over (1..64)       */
    int precision;     /* enum precode_prec for every job                      */
    size_t slab_bytes; /* device memory for resident state (the HBM budget)    */
    int impl;          /* enum precode_impl for every job (AUTO, FUSED, PLAIN) */
} precode_serve_config;

typedef struct precode_serve_stats {
    int jobs_done;
    int peak_active;                   /* most jobs admitted at once            */
    long long symbols_done;            /* symbol vectors (all subcarriers)      */
    long long subcarrier_symbols_done; /* subcarrier-symbols precoded           */
    double wall_s;                     /* first arrival to last completion      */
    double throughput;                 /* subcarrier-symbols per second         */
    double lat_p50_s, lat_p99_s, lat_max_s; /* symbol latency                   */
    double wait_p50_s, wait_p99_s;     /* admission wait (arrival to admission) */
    size_t peak_bytes;                 /* peak slab use                         */
} precode_serve_stats;

int precode_serve(precode_ctx *ctx, const precode_serve_job *jobs, int n_jobs,
                  const precode_serve_config *cfg, double *sym_latency,
                  precode_serve_stats *stats);

#ifdef __cplusplus
}
#endif

#endif /* PRECODE_H */
