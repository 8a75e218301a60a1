// serve.hip -- continuous-batching serving loop for per-frame precoding jobs.
//
// Each job is one frame of one cell: a channel that stays constant over the
// frame's K OFDM symbols and K symbol vectors released one after another
// (the per-frame factors are computed once and reused for every symbol,
// Sec. IV-B).  The loop replays an arrival trace in real time:
//
//   admission  an arrived job is admitted (FIFO) when fewer than max_active
//              jobs are in flight and its resident state fits the HBM budget;
//              state comes from one device slab sub-allocated on the host, so
//              the loop never calls hipMalloc / hipFree
//   prepare    Gram + factorization + beta / weights of the frame, enqueued on
//              the job's stream as soon as it is admitted
//   symbols    symbols whose release time has passed are precoded from the
//              resident factors, all newly released symbols of a job in one
//              launch; jobs on different streams overlap on the device.  A
//              job with a zero symbol period (every symbol released at
//              arrival) on the fused kernels takes one launch from Gram to
//              precode instead of prepare + symbols.  Jobs the register-tile
//              kernels do not take run on the wide FP64 kernel (its factors
//              scale A^-1 in FP64), jobs without symbols on the plain ones
//   retire     when a job's last symbol completes its state returns to the slab
//              and waiting jobs can be admitted
//
// Latency of a symbol = time its precoded vector is observed complete - its
// release time (host steady clock; completions are polled with event queries).
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <vector>

#include "common.h"

namespace pc {
namespace {

// First-fit sub-allocator over one device slab (host-side bookkeeping only).
class Slab {
   public:
    bool init(size_t bytes) {
        cap_ = bytes;
        if (hipMalloc(&base_, bytes ? bytes : 1) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            return false;
        }
        free_[0] = bytes;
        return true;
    }
    ~Slab() {
        if (base_) (void)hipFree(base_);
    }
    void *alloc(size_t n) {
        n = (n + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                used_ += n;
                peak_ = std::max(peak_, used_);
                return (char *)base_ + off;
            }
        }
        return nullptr;
    }
    void release(void *p, size_t n) {
        n = (n + 255) & ~(size_t)255;
        size_t off = (char *)p - (char *)base_;
        used_ -= n;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + n == nx->first) {
            n += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t peak() const { return peak_; }
    size_t capacity() const { return cap_; }

   private:
    void *base_ = nullptr;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Launch {
    hipEvent_t ev;
    int k0, nk;
};

struct JobState {
    const precode_serve_job *src;
    Prob p;
    bool fused;  // register-tile kernels
    bool wide;   // the wide FP64 kernel (factors scale A^-1 in FP64)
    int precision;
    size_t n_inst;
    // device state from the slab
    void *mem = nullptr;
    size_t bytes = 0;
    float2 *ainv = nullptr;  // fused or wide factors, or plain A^-1 slots
    void *wsA = nullptr, *wsScale = nullptr, *wsZ = nullptr;
    float *scale_out = nullptr;
    int *status = nullptr;
    int stream = 0;
    int next = 0;       // next symbol to launch
    int done = 0;       // symbols completed
    double t_admit = 0;
    std::deque<Launch> inflight;
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

double pct(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace
}  // namespace pc

using namespace pc;

extern "C" int precode_serve(precode_ctx *ctx, const precode_serve_job *jobs, int n_jobs,
                             const precode_serve_config *cfg, double *sym_latency, precode_serve_stats *stats) {
    if (!ctx || n_jobs < 0 || (n_jobs > 0 && !jobs) || !cfg || !stats) return PRECODE_EINVAL;
    if (cfg->max_active < 1 || cfg->n_streams < 1 || cfg->n_streams > 64 || cfg->slab_bytes == 0 ||
        cfg->impl < PRECODE_IMPL_AUTO || cfg->impl > PRECODE_IMPL_PLAIN)
        return PRECODE_EINVAL;
    memset(stats, 0, sizeof(*stats));
    // no launch-shape timing inside the loop (it would synchronize a stream)
    struct NoTune {
        NoTune() { fused_set_autotune(false); }
        ~NoTune() { fused_set_autotune(true); }
    } no_tune;
    // validate every job and size its resident state before touching the device
    std::vector<JobState> st(n_jobs);
    std::vector<size_t> sym_off(n_jobs + 1, 0);
    size_t total_syms = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const precode_job &j = jobs[i].job;
        if (!(jobs[i].arrival_s >= 0) || !(jobs[i].symbol_period_s >= 0)) return PRECODE_EINVAL;
        precode_params q;
        precode_params_init(&q);
        q.power = j.power;
        q.Es = j.Es;
        q.tau = j.tau;
        q.precision = cfg->precision;
        JobState &s = st[i];
        s.src = &jobs[i];
        int rc = make_prob_checked(j.arch, j.rho, j.cluster_sizes, j.C, j.mode, j.B, j.U, j.n_sc, j.K, &q,
                                            &s.p);
        if (rc) return rc;
        if (j.n_sc > 0 && (!j.H || (j.K > 0 && (!j.s || !j.x)))) return PRECODE_EINVAL;
        s.fused = cfg->impl != PRECODE_IMPL_PLAIN && fused_supported(s.p, cfg->precision);
        // every other job with symbols on the wide FP64 kernel
        s.wide = !s.fused && cfg->impl != PRECODE_IMPL_PLAIN && wide_supported(s.p, j.K);
        if (!s.fused && !s.wide &&
            (cfg->impl == PRECODE_IMPL_FUSED || cfg->precision == PRECODE_PREC_SPLIT_FP16 ||
             cfg->precision == PRECODE_PREC_SPLIT_BF16))
            return PRECODE_EUNSUPPORTED;
        s.precision = cfg->precision;
        s.n_inst = (size_t)n_inst(s.p);
        const size_t ni = s.n_inst;
        const size_t aux = ni * sizeof(float) + ni * sizeof(int) + 512;
        if (s.fused)
            s.bytes = ni * j.U * j.U * sizeof(float2) + aux;
        else if (s.wide)
            s.bytes = wide_factor_bytes(s.p) + aux;
        else
            s.bytes = 2 * plain_ws_bytes_A(s.p) + plain_ws_bytes_scale(s.p) + plain_ws_bytes_z(s.p, j.K) + aux + 1024;
        if (s.bytes > cfg->slab_bytes) return PRECODE_ENOMEM;  // could never be admitted
        total_syms += (size_t)j.K;
        sym_off[i + 1] = total_syms;
    }
    int dev = 0;
    if (hipSetDevice(ctx_device(ctx)) != hipSuccess || hipGetDevice(&dev) != hipSuccess) return PRECODE_EDEVICE;
    if (n_jobs == 0) return PRECODE_OK;
    Slab slab;
    if (!slab.init(cfg->slab_bytes)) return PRECODE_ENOMEM;
    std::vector<hipStream_t> streams;
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (auto q : streams) (void)hipStreamDestroy(q);
            return PRECODE_EDEVICE;
        }
        streams.push_back(s);
    }
    std::vector<hipEvent_t> evpool;
    auto get_event = [&]() -> hipEvent_t {
        if (!evpool.empty()) {
            hipEvent_t e = evpool.back();
            evpool.pop_back();
            return e;
        }
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    };
    // pre-create events so the loop rarely creates any
    for (int i = 0; i < 4 * cfg->max_active + 16; ++i) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) evpool.push_back(e);
    }

    std::vector<int> order(n_jobs);
    for (int i = 0; i < n_jobs; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return jobs[a].arrival_s < jobs[b].arrival_s; });
    std::vector<double> lat, waits;
    lat.reserve(total_syms);
    size_t next_arrival = 0;
    std::deque<int> waiting;
    std::vector<int> active;
    int rr = 0, rc_out = PRECODE_OK;
    size_t syms_done = 0, subsyms_done = 0;
    int jobs_done = 0, peak_active = 0;
    const auto t0 = std::chrono::steady_clock::now();
    double t_last = 0;

    while (jobs_done < n_jobs && rc_out == PRECODE_OK) {
        const double t = now_s(t0);
        while (next_arrival < order.size() && jobs[order[next_arrival]].arrival_s <= t)
            waiting.push_back(order[next_arrival++]);
        // ---- admission (FIFO) -------------------------------------------------
        while (!waiting.empty() && (int)active.size() < cfg->max_active) {
            JobState &s = st[waiting.front()];
            s.mem = slab.alloc(s.bytes);
            if (!s.mem) break;  // over the HBM budget: wait for a retirement
            const precode_job &j = s.src->job;
            const size_t ni = s.n_inst;
            char *m = (char *)s.mem;
            hipStream_t stream = streams[rr];
            s.stream = rr;
            rr = (rr + 1) % cfg->n_streams;
            hipError_t e = hipSuccess;
            if (s.fused) {
                s.ainv = (float2 *)m;
                m += (ni * j.U * j.U * sizeof(float2) + 255) & ~(size_t)255;
            } else if (s.wide) {
                s.ainv = (float2 *)m;
                m += (wide_factor_bytes(s.p) + 255) & ~(size_t)255;
            } else {
                const size_t bA = plain_ws_bytes_A(s.p);
                s.wsA = m;
                m += (bA + 255) & ~(size_t)255;
                s.ainv = (float2 *)m;
                m += (bA + 255) & ~(size_t)255;
                s.wsScale = m;
                m += (plain_ws_bytes_scale(s.p) + 255) & ~(size_t)255;
                s.wsZ = m;
                m += (plain_ws_bytes_z(s.p, j.K) + 255) & ~(size_t)255;
            }
            s.scale_out = (float *)m;
            m += (ni * sizeof(float) + 255) & ~(size_t)255;
            s.status = (int *)m;
            // a job whose symbols are all released at arrival (zero symbol
            // period) is precoded in one launch that keeps the channel in
            // registers from the Gram to the precode, so the channel is read
            // once instead of once for the factors and again for the symbols
            const bool one_launch = (s.fused || s.wide) && j.n_sc > 0 && j.K > 0 && s.src->symbol_period_s <= 0;
            if (j.n_sc > 0) {
                if (one_launch && s.fused)
                    e = fused_run(s.p, s.precision, (const float2 *)j.H, (const float2 *)j.s, (float2 *)j.x,
                                  s.scale_out, s.status, stream);
                else if (one_launch)
                    e = wide_run(s.p, (const float2 *)j.H, (const float2 *)j.s, (float2 *)j.x, s.scale_out,
                                 s.status, stream);
                else if (s.fused)
                    e = fused_prepare(s.p, s.precision, (const float2 *)j.H, s.ainv, s.scale_out, s.status, stream);
                else if (s.wide)
                    e = wide_prepare(s.p, (const float2 *)j.H, s.ainv, s.scale_out, s.status, stream);
                else
                    e = plain_prepare(s.p, (const float2 *)j.H, s.scale_out, s.status, s.wsA, s.ainv, s.wsScale,
                                      stream);
                if (e == hipSuccess && j.scale)
                    e = hipMemcpyAsync(j.scale, s.scale_out, ni * sizeof(float), hipMemcpyDeviceToDevice, stream);
                if (e == hipSuccess && j.status)
                    e = hipMemcpyAsync(j.status, s.status, ni * sizeof(int), hipMemcpyDeviceToDevice, stream);
            }
            // a job with no symbols still retires only once its factors and
            // their copies are done (its slab region is written until then)
            if (e == hipSuccess && (one_launch || j.K == 0)) {
                Launch L;
                L.ev = get_event();
                L.k0 = 0;
                L.nk = j.K;
                e = L.ev ? hipEventRecord(L.ev, stream) : hipErrorOutOfMemory;
                if (e == hipSuccess) {
                    s.inflight.push_back(L);
                    s.next = j.K;
                } else if (L.ev) {
                    evpool.push_back(L.ev);
                }
            }
            if (e != hipSuccess) {
                rc_out = PRECODE_EDEVICE;
                break;
            }
            s.t_admit = t;
            waits.push_back(t - s.src->arrival_s);
            active.push_back(waiting.front());
            waiting.pop_front();
            peak_active = std::max(peak_active, (int)active.size());
        }
        // ---- symbol releases --------------------------------------------------
        for (int id : active) {
            JobState &s = st[id];
            const precode_job &j = s.src->job;
            if (s.next >= j.K) continue;
            const double per = s.src->symbol_period_s;
            int rel = j.K;
            if (per > 0) rel = std::min(j.K, (int)((t - s.src->arrival_s) / per) + 1);
            if (rel <= s.next) continue;
            const int k0 = s.next, nk = rel - s.next;
            hipStream_t stream = streams[s.stream];
            hipError_t e = hipSuccess;
            if (j.n_sc > 0) {
                const float2 *sk = (const float2 *)j.s + (size_t)k0 * j.n_sc * j.U;
                float2 *xk = (float2 *)j.x + (size_t)k0 * j.n_sc * j.B;
                Prob pk = s.p;
                pk.K = nk;
                if (s.fused)
                    e = fused_symbols(pk, s.precision, nk, (const float2 *)j.H, s.ainv, s.status, sk, xk, stream);
                else if (s.wide)
                    e = wide_symbols(pk, nk, (const float2 *)j.H, s.ainv, s.status, sk, xk, stream);
                else
                    e = plain_symbols(pk, nk, (const float2 *)j.H, sk, xk, s.ainv, s.wsScale, s.wsZ, stream);
            }
            Launch L;
            L.ev = get_event();
            L.k0 = k0;
            L.nk = nk;
            if (e == hipSuccess && L.ev) e = hipEventRecord(L.ev, stream);
            if (e != hipSuccess || !L.ev) {
                rc_out = PRECODE_EDEVICE;
                break;
            }
            s.inflight.push_back(L);
            s.next = rel;
        }
        // ---- completions ------------------------------------------------------
        const double tq = now_s(t0);
        for (size_t a = 0; a < active.size();) {
            JobState &s = st[active[a]];
            const precode_job &j = s.src->job;
            while (!s.inflight.empty()) {
                hipError_t q = hipEventQuery(s.inflight.front().ev);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    rc_out = PRECODE_EDEVICE;
                    break;
                }
                const Launch L = s.inflight.front();
                s.inflight.pop_front();
                evpool.push_back(L.ev);
                for (int k = L.k0; k < L.k0 + L.nk; ++k) {
                    const double release = s.src->arrival_s + k * s.src->symbol_period_s;
                    const double l = tq - release;
                    if (sym_latency) sym_latency[sym_off[active[a]] + k] = l;
                    lat.push_back(l);
                }
                s.done += L.nk;
                syms_done += L.nk;
                subsyms_done += (size_t)L.nk * j.n_sc;
            }
            if (s.done >= j.K && s.next >= j.K && s.inflight.empty()) {
                slab.release(s.mem, s.bytes);
                s.mem = nullptr;
                ++jobs_done;
                t_last = tq;
                active[a] = active.back();
                active.pop_back();
            } else {
                ++a;
            }
        }
    }
    for (auto &s : streams) (void)hipStreamSynchronize(s);
    for (auto &s : streams) (void)hipStreamDestroy(s);
    for (auto e : evpool) (void)hipEventDestroy(e);
    stats->jobs_done = jobs_done;
    stats->symbols_done = (long long)syms_done;
    stats->subcarrier_symbols_done = (long long)subsyms_done;
    const double first = n_jobs ? jobs[order[0]].arrival_s : 0.0;
    stats->wall_s = t_last - first;
    stats->throughput = stats->wall_s > 0 ? (double)subsyms_done / stats->wall_s : 0.0;
    stats->lat_p50_s = pct(lat, 0.50);
    stats->lat_p99_s = pct(lat, 0.99);
    stats->lat_max_s = lat.empty() ? 0.0 : *std::max_element(lat.begin(), lat.end());
    stats->wait_p50_s = pct(waits, 0.50);
    stats->wait_p99_s = pct(waits, 0.99);
    stats->peak_active = peak_active;
    stats->peak_bytes = slab.peak();
    return rc_out;
}
