// fused.hip -- single-problem dispatch of the fused PD / FD kernel on gfx950,
// with the launch-shape autotuner.
//
// One launch runs the whole per-system chain; only the precoded vectors,
// beta / weights and status are written back (the kernel body is in
// fused_kernel.h).  Every wave owns one local system -- a PD subcarrier over
// the whole array, or one FD cluster of a subcarrier -- and runs it without
// any workgroup barrier:
//
//   Gram        G_c = H_c^H H_c on MFMA over the real embedding
//               [Re h_u, Im h_u] of the columns: the 2U x 2U real Gram M
//               gives G = (M_rr + M_ii) + i (M_ri - M_ir) (local Gram,
//               Sec. III-B; for PD the accumulation over every cluster's
//               rows is the cluster sum of the adder tree).  Rows stream
//               from HBM in 32-row tiles loaded straight into the MFMA
//               operand layout, the next tile's loads in flight during the
//               current tile's MFMAs
//   regularize  A = G + kappa I (PD) / A_c = G_c + kappa_c I (FD,
//               kappa_c = tau_c C kappa, Sec. III-C)
//   invert      A^-1 in registers (Gauss-Jordan elimination; for Hermitian
//               positive-definite A its pivots are the squared diagonal of
//               the Cholesky factor)
//   factor      t = tr A^-1 - kappa ||A^-1||_F^2 (Lemma 1);
//               PD beta = sqrt(Es/rho^2 t); FD w_c = sqrt(rho_c^2/(t Es))
//   solve       Z = scale * A^-1 S for chunks of 16 symbols, on MFMA, with S
//               read from global memory
//   precode     X_c = H_c Z on MFMA (Sec. III-B; FD x_c = w_c H_c A_c^-1 s,
//               Sec. III-C): the rows are streamed a second time (served by
//               the cache) in the row layout of the product and the results
//               stored coalesced
//
// Launch shape: NW = 1, 2 or 4 waves per workgroup (fused_nw{1,2,4}.hip),
// each wave one system.  For PD with NW >= 2 whose rows do not fit one wave's
// registers, the NW waves instead share one subcarrier (split): each keeps
// its share of the channel tiles in registers from load to precode, the
// partial Grams are summed in LDS in fixed wave order, and one master wave
// factors and solves.  The autotuner times every feasible shape (NW, and
// register tiles or rows streamed twice) on the first call of each problem
// shape (the call itself, repeated) and caches the fastest for the process
// and in a file per device and HIP runtime.
//
// Modes: full (Gram to precode), prepare (per-frame factors scale * A^-1 to
// device memory for the frame API and serving) and symbols (precode released
// symbols from stored factors, re-reading only the channel).
//
// MFMA precision (PREC): FP32 (v_mfma_f32_32x32x2f32, exact FP32 products)
// or split 16-bit: every operand x is written as hi + lo with hi = f16(x),
// lo = f16(x - hi) (or bf16) and a product a b is accumulated as
// ah bh + ah bl + al bh in FP32 (v_mfma_f32_32x32x16_f16 / _bf16).  Each
// operand tile is scaled by a power of two into the FP16 range first and the
// FP32 result unscaled exactly.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <mutex>
#include <set>
#include <string>
#include <unordered_map>

#include "fused_kernel.h"
#include "fused_launch.h"

namespace pc {
namespace {

constexpr int kNWs[] = {1, 2, 4};
constexpr int kDefaultNW = 4;
// the last-level (Infinity) cache: a channel no larger stays resident across
// back-to-back calls on the same inputs
constexpr size_t kCacheBytes = size_t(256) << 20;

bool nw_feasible(const Prob &p, int nw) {
    const int up = pick_up(p.U);
    if (up == 0) return false;
    const size_t lds = up == 16 ? Lds<16>::bytes(nw) : Lds<32>::bytes(nw);
    return lds <= kLdsUsable;
}

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

hipError_t launch_nw(int nw, const Prob &p, int prec, const FusedCall &a, hipStream_t st) {
    switch (nw) {
        case 1: return fused_launch_nw1(p, prec, a, st);
        case 2: return fused_launch_nw2(p, prec, a, st);
        default: return fused_launch_nw4(p, prec, a, st);
    }
}

// One launch of a mode (all K symbols, in chunks of 16 inside the kernel).
// A launch shape: waves per workgroup, and whether every wave streams its
// rows twice instead of keeping them in register tiles.  Coded as
// nw | kStreamBit for the caches.
constexpr int kStreamBit = 16;

// Register tiles per wave and whether the waves share a PD subcarrier, for
// NW waves per workgroup (maxt 0: the rows are streamed twice).
void pick_tiles(const Prob &p, int nw, bool stream, int *maxt, bool *split) {
    stream = stream || env_int("PRECODE_FUSED_STREAM", 0);
    *maxt = stream ? 0 : pick_maxt(p);
    // a PD system too large for one wave's registers: the waves of a
    // workgroup share the subcarrier instead of streaming its rows
    *split = false;
    if (*maxt == 0 && nw >= 2 && !stream) {
        const int m = pick_split_maxt(p, nw);
        if (m > 0) {
            *split = true;
            *maxt = m;
        }
    }
}

hipError_t run_once(int shape, const Prob &p, int prec, int mode, int K, const float2 *H, const float2 *s, float2 *x,
                    cx<float> *ainv, float *scale_out, int *status, hipStream_t st) {
    const int nw = shape & ~kStreamBit;
    FusedCall a;
    a.K = mode == kPrepare ? 0 : K;
    a.mode = mode;
    pick_tiles(p, nw, (shape & kStreamBit) != 0, &a.maxt, &a.split);
    a.vec = pick_vec(p, H);
    a.H = H;
    a.s = s;
    a.x = x;
    a.ainv = ainv;
    a.scale_out = scale_out;
    a.status = status;
    return launch_nw(nw, p, prec, a, st);
}

// ---- autotuner ------------------------------------------------------------------
// Cache: (device, problem shape) -> launch shape, for the process and, unless
// disabled, persisted in a text file (one line per entry: device key,
// problem-shape key, waves per workgroup, streamed) so that later processes
// on the same device and HIP runtime skip the timing.  Environment:
// PRECODE_FUSED_WAVES=1|2|4 forces the waves (when feasible),
// PRECODE_AUTOTUNE=0 disables tuning (default shape), PRECODE_TUNE_CACHE=path
// names the file ("off": no file; unset: $XDG_CACHE_HOME/precode/tune.txt or
// $HOME/.cache/precode/tune.txt).
std::mutex g_tune_mu;
std::unordered_map<std::string, int> g_tuned;
std::set<std::string> g_loaded;  // cache files read into g_tuned
std::unordered_map<int, std::string> g_devkey;

std::string tune_key(const Prob &p, int prec, int mode, int K) {
    std::string k = std::to_string(p.arch) + "/" + std::to_string(p.U) + "/" + std::to_string(p.B) + "/" +
                    std::to_string(p.n_sc) + "/" + std::to_string(K) + "/" +
                    std::to_string(prec) + "/" + std::to_string(mode) + ":";
    if (p.arch == kFD)
        for (int c = 0; c < p.C; ++c) k += std::to_string(p.off[c + 1] - p.off[c]) + ",";
    return k;
}

// The current device and HIP runtime: "<arch>|<name>|<CUs>cu|hip<version>",
// spaces replaced (called with g_tune_mu held).
std::string device_key() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    auto it = g_devkey.find(dev);
    if (it != g_devkey.end()) return it->second;
    hipDeviceProp_t pr;
    int rt = 0;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess || hipRuntimeGetVersion(&rt) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    char buf[640];
    snprintf(buf, sizeof buf, "%s|%s|%dcu|hip%d", pr.gcnArchName, pr.name, pr.multiProcessorCount, rt);
    std::string k(buf);
    for (char &c : k)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    g_devkey[dev] = k;
    return k;
}

std::string cache_path() {
    const char *v = getenv("PRECODE_TUNE_CACHE");
    if (v) return (strcmp(v, "off") == 0 || strcmp(v, "0") == 0) ? std::string() : std::string(v);
    const char *x = getenv("XDG_CACHE_HOME");
    const char *h = getenv("HOME");
    if (x && *x) return std::string(x) + "/precode/tune.txt";
    if (h && *h) return std::string(h) + "/.cache/precode/tune.txt";
    return std::string();
}

bool valid_shape(int code) {
    const int nw = code & ~kStreamBit;
    return nw == 1 || nw == 2 || nw == 4;
}

// Reads the cache file's entries into g_tuned once per path (g_tune_mu held).
void load_cache(const std::string &path) {
    if (path.empty() || g_loaded.count(path)) return;
    g_loaded.insert(path);
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    char dk[640], tk[4096];
    int nw = 0, stream = 0;
    while (fscanf(f, "%639s %4095s %d %d", dk, tk, &nw, &stream) == 4) {
        const int code = nw | (stream ? kStreamBit : 0);
        if (valid_shape(code)) g_tuned[std::string(dk) + " " + tk] = code;
    }
    fclose(f);
}

// Appends one entry (g_tune_mu held); failures leave the process cache only.
void save_entry(const std::string &path, const std::string &dk, const std::string &tk, int code) {
    if (path.empty()) return;
    const size_t sl = path.rfind('/');
    if (sl != std::string::npos && sl > 0) {
        // the default location's directories
        const std::string dir = path.substr(0, sl);
        const size_t up = dir.rfind('/');
        if (up != std::string::npos && up > 0) (void)mkdir(dir.substr(0, up).c_str(), 0755);
        (void)mkdir(dir.c_str(), 0755);
    }
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;
    fprintf(f, "%s %s %d %d\n", dk.c_str(), tk.c_str(), code & ~kStreamBit, (code & kStreamBit) ? 1 : 0);
    fclose(f);
}

thread_local bool t_autotune = true;

bool shape_ok(const Prob &p, int code) {
    return valid_shape(code) && nw_feasible(p, code & ~kStreamBit);
}

// The shape of an untuned call (tuning off, stream capture, serving): the
// fewest waves per workgroup that keep the system's rows in register tiles
// (split over the workgroup for large PD cells), else the default.  At 32
// users the split holds one wave per SIMD and loses to streaming the rows
// (512 antennas, 3300 subcarriers: 0.52 ms against 0.32 ms), so there the
// fewest waves that stream are taken instead.
int default_shape(const Prob &p) {
    const bool up32 = pick_up(p.U) == 32;
    for (int nw : kNWs) {
        int mt;
        bool sp;
        pick_tiles(p, nw, false, &mt, &sp);
        if (mt > 0 && !(sp && up32) && nw_feasible(p, nw)) return nw;
    }
    if (up32)
        for (int nw : kNWs)
            if (nw_feasible(p, nw)) return nw | kStreamBit;
    if (nw_feasible(p, kDefaultNW)) return kDefaultNW;
    for (int nw : kNWs)
        if (nw_feasible(p, nw)) return nw;
    return 0;
}

// Chooses the launch shape for this call; may run the call several times on
// `st` to time the candidates (outputs are rewritten by the real launch that
// follows).
int choose_shape(const Prob &p, int prec, int mode, int K, const float2 *H, const float2 *s, float2 *x,
                 cx<float> *ainv, float *scale_out, int *status, hipStream_t st) {
    const int dflt = default_shape(p);
    const int forced = env_int("PRECODE_FUSED_WAVES", 0);
    if (forced && nw_feasible(p, forced)) return forced;
    if (!env_int("PRECODE_AUTOTUNE", 1)) return dflt;
    const std::string tk = tune_key(p, prec, mode, K);
    const std::string path = cache_path();
    std::string dk;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        dk = device_key();
        auto it = g_tuned.find(dk + " " + tk);
        if (it == g_tuned.end()) {
            load_cache(path);
            it = g_tuned.find(dk + " " + tk);
        }
        if (it != g_tuned.end() && shape_ok(p, it->second)) return it->second;
    }
    if (!t_autotune) return dflt;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return dflt;
    // candidates: every feasible waves count with its register tiles, and
    // with its rows streamed when the channel exceeds the cache.  The timing
    // repeats the call on the same inputs, which then sit in the cache and
    // hide a streamed shape's second HBM pass; a larger channel is re-read
    // from HBM on every call, so there the timing is fair to every shape
    // (with 32 users, 512 antennas and 3300 subcarriers the streamed shapes
    // take 0.33 ms and the register-tile split 0.54 ms).  A shape whose
    // register tiles do not fit streams anyway and is a candidate as such.
    int cands[6], nc = 0;
    const bool cache_hot = size_t(p.n_sc) * size_t(p.B) * size_t(p.U) * sizeof(float2) <= kCacheBytes;
    bool any_tiles = false;
    for (int nw : kNWs) {
        int mt;
        bool sp;
        pick_tiles(p, nw, false, &mt, &sp);
        if (nw_feasible(p, nw) && mt > 0) any_tiles = true;
    }
    for (int nw : kNWs) {
        if (!nw_feasible(p, nw)) continue;
        int mt;
        bool sp;
        pick_tiles(p, nw, false, &mt, &sp);
        if (mt > 0) cands[nc++] = nw;
        if ((mt == 0 && !any_tiles) || (mt > 0 && !cache_hot)) cands[nc++] = nw | kStreamBit;
    }
    int best = nc > 0 ? cands[0] : dflt;
    if (nc > 1) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return dflt;
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return dflt;
        }
        // every candidate once untimed (a kernel's first launch also loads
        // it), then kRounds rounds over the candidates in turn, each timing
        // kCalls back-to-back calls (so that the dispatch gaps between calls,
        // larger under a tracing profiler, do not decide the shape); a
        // candidate's time is its best round, so a one-off stall in one round
        // does not decide the shape either
        constexpr int kRounds = 3, kCalls = 8;
        float best_of[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        bool ok = true;
        for (int i = 0; i < nc && ok; ++i)
            ok = run_once(cands[i], p, prec, mode, K, H, s, x, ainv, scale_out, status, st) == hipSuccess;
        for (int round = 0; round < kRounds && ok; ++round)
            for (int i = 0; i < nc && ok; ++i) {
                ok = hipEventRecord(e0, st) == hipSuccess;
                for (int r = 0; r < kCalls && ok; ++r)
                    ok = run_once(cands[i], p, prec, mode, K, H, s, x, ainv, scale_out, status, st) == hipSuccess;
                float ms = 0.f;
                ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (ok && (round == 0 || ms < best_of[i])) best_of[i] = ms;
            }
        if (ok) {
            best = cands[0];
            float bm = best_of[0];
            for (int i = 1; i < nc; ++i)
                if (best_of[i] < bm) {
                    bm = best_of[i];
                    best = cands[i];
                }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (!ok) {
            (void)hipGetLastError();
            return dflt;
        }
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[dk + " " + tk] = best;
    save_entry(path, dk, tk, best);
    return best;
}

hipError_t run_mode(const Prob &p, int precision, int mode, int K, const float2 *H, const float2 *s, float2 *x,
                    cx<float> *ainv, float *scale_out, int *status, hipStream_t st, int *nw_used) {
    const int prec = prec_of(precision);
    const int shape = choose_shape(p, prec, mode, K, H, s, x, ainv, scale_out, status, st);
    if (shape == 0) return hipErrorNotSupported;
    if (nw_used) *nw_used = shape & ~kStreamBit;
    return run_once(shape, p, prec, mode, K, H, s, x, ainv, scale_out, status, st);
}

}  // namespace

bool fused_supported(const Prob &p, int precision) {
    if (prec_of(precision) < 0) return false;
    // the batch launches use the default shape; every entry point needs it
    if (!nw_feasible(p, kDefaultNW)) return false;
    if (p.arch == kPD) return p.pd_fp64 == 0;
    for (int c = 0; c < p.C; ++c) {
        if (p.fp64[c]) return false;
        if (p.off[c + 1] - p.off[c] < p.U) return false;
    }
    return true;
}

int fused_default_waves() { return kDefaultNW; }

void fused_set_autotune(bool on) { t_autotune = on; }

void fused_autotune_reset() {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned.clear();
    g_loaded.clear();
}

hipError_t fused_run(const Prob &p, int precision, const float2 *H, const float2 *s, float2 *x, float *scale_out,
                     int *status, hipStream_t st, int *nw_used) {
    if (!fused_supported(p, precision)) return hipErrorNotSupported;
    if (p.n_sc == 0) return hipSuccess;
    // full path: factors are written by the first slice only (ainv unused)
    return run_mode(p, precision, kFull, p.K, H, s, x, nullptr, scale_out, status, st, nw_used);
}

hipError_t fused_prepare(const Prob &p, int precision, const float2 *H, float2 *ainv, float *scale_out, int *status,
                         hipStream_t st) {
    if (!fused_supported(p, precision)) return hipErrorNotSupported;
    if (p.n_sc == 0) return hipSuccess;
    return run_mode(p, precision, kPrepare, 0, H, nullptr, nullptr, (cx<float> *)ainv, scale_out, status, st,
                    nullptr);
}

hipError_t fused_symbols(const Prob &p, int precision, int nk, const float2 *H, const float2 *ainv,
                         const int *status, const float2 *s, float2 *x, hipStream_t st) {
    if (!fused_supported(p, precision)) return hipErrorNotSupported;
    if (p.n_sc == 0 || nk == 0) return hipSuccess;
    // status is only read in this mode
    return run_mode(p, precision, kSymbols, nk, H, s, x, (cx<float> *)ainv, nullptr, (int *)status, st, nullptr);
}

}  // namespace pc
