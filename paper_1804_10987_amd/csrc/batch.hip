// batch.hip -- heterogeneous batches of fused PD / FD problems (cells of
// different B, cluster sizes, U and subcarrier counts) in as few launches as
// the kernel's shape classes allow.
//
// Every problem is cut into slices of at most kMaxKFused symbols (each slice
// recomputes its factors, as the single-problem path does).  Slices are
// grouped by shape class -- tile width UP (16 / 32), PD or FD, channel tiles
// per wave MAXT -- and each class is one launch whose grid is the sum of its
// slices' workgroups.  The slice table sits in device memory; a workgroup
// finds its slice by binary search over the slices' first block index and
// then runs the same body as the single-problem kernel.
#include <string.h>

#include <algorithm>
#include <vector>

#include "fused_kernel.h"

namespace pc {
namespace {

constexpr int NW = 4;  // waves per workgroup of the batch launches
constexpr int kThreads = 64 * NW;

struct Entry {
    Prob p;
    const float2 *H, *s;
    float2 *x;
    float *scale_out;
    int *status;
    int K;       // symbols of this slice
    int block0;  // first block of this slice within its class launch
};

struct Class {
    int up, arch, maxt;
    bool operator==(const Class &o) const { return up == o.up && arch == o.arch && maxt == o.maxt; }
    bool operator<(const Class &o) const {
        return up != o.up ? up < o.up : (arch != o.arch ? arch < o.arch : maxt < o.maxt);
    }
};

Class class_of(const Prob &p) {
    const int up = pick_up(p.U);
    return Class{up, p.arch, pick_maxt(p, up, NW)};
}

int blocks_of(const Prob &p) { return p.n_sc * (p.arch == kPD ? 1 : (p.C + NW - 1) / NW); }

// Slices of every problem, in launch order (by class, then problem order).
struct Plan {
    std::vector<Entry> e;
    std::vector<Class> cls;    // class of each run
    std::vector<int> first;    // first entry of each run, plus the end
    std::vector<int> blocks;   // grid of each run
    std::vector<int> kmax;     // most symbols of a slice in each run
};

Plan make_plan(const BatchProblem *bp, int n) {
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return class_of(bp[a].p) < class_of(bp[b].p); });
    Plan pl;
    for (int oi = 0; oi < n; ++oi) {
        const BatchProblem &q = bp[order[oi]];
        const Class c = class_of(q.p);
        if (pl.cls.empty() || !(pl.cls.back() == c)) {
            pl.cls.push_back(c);
            pl.first.push_back((int)pl.e.size());
            pl.blocks.push_back(0);
            pl.kmax.push_back(0);
        }
        if (q.p.n_sc == 0) continue;
        for (int k0 = 0; k0 < q.p.K; k0 += kMaxKFused) {
            const int kk = std::min(kMaxKFused, q.p.K - k0);
            Entry en;
            en.p = q.p;
            en.p.K = kk;
            en.H = q.H;
            en.s = q.s + (size_t)k0 * q.p.n_sc * q.p.U;
            en.x = q.x + (size_t)k0 * q.p.n_sc * q.p.B;
            // factors are identical for every slice; the first writes them
            en.scale_out = k0 == 0 ? q.scale_out : nullptr;
            en.status = k0 == 0 ? q.status : nullptr;
            en.K = kk;
            en.block0 = pl.blocks.back();
            pl.blocks.back() += blocks_of(q.p);
            pl.kmax.back() = std::max(pl.kmax.back(), kk);
            pl.e.push_back(en);
        }
    }
    pl.first.push_back((int)pl.e.size());
    return pl;
}

template <int UP, int ARCH, int PREC, int MAXT>
__global__ void __launch_bounds__(kThreads, (min_waves<UP, MAXT>()))
    fused_batch_k(const Entry *__restrict__ tab, int n) {
    const int b = blockIdx.x;
    int lo = 0, hi = n - 1;  // last slice with block0 <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const Entry &E = tab[lo];
    fused_body<UP, ARCH, PREC, MAXT, NW>(E.p, E.p.off, b - E.block0, E.K, kFull, E.H, E.s, E.x, nullptr, E.scale_out,
                                     E.status);
}

template <int UP, int ARCH, int PREC, int MAXT>
hipError_t launch(const Entry *tab, int n, int blocks, int kmax, hipStream_t st) {
    const void *fn = (const void *)fused_batch_k<UP, ARCH, PREC, MAXT>;
    const size_t lds = Lds<UP>::bytes(kmax, NW);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((fused_batch_k<UP, ARCH, PREC, MAXT>), dim3(blocks), dim3(kThreads), lds, st, tab, n);
    return hipGetLastError();
}

template <int UP, int ARCH, int PREC>
hipError_t launch_t(int maxt, const Entry *tab, int n, int blocks, int kmax, hipStream_t st) {
    switch (maxt) {
        case 1: return launch<UP, ARCH, PREC, 1>(tab, n, blocks, kmax, st);
        case 2: return launch<UP, ARCH, PREC, 2>(tab, n, blocks, kmax, st);
        case 4: return launch<UP, ARCH, PREC, 4>(tab, n, blocks, kmax, st);
        default:
            if constexpr (UP == 16) return launch<UP, ARCH, PREC, 8>(tab, n, blocks, kmax, st);
            return hipErrorNotSupported;
    }
}

template <int UP, int ARCH>
hipError_t launch_prec(int prec, int maxt, const Entry *tab, int n, int blocks, int kmax, hipStream_t st) {
    switch (prec) {
        case kF32: return launch_t<UP, ARCH, kF32>(maxt, tab, n, blocks, kmax, st);
        case kF16: return launch_t<UP, ARCH, kF16>(maxt, tab, n, blocks, kmax, st);
        default: return launch_t<UP, ARCH, kBF16>(maxt, tab, n, blocks, kmax, st);
    }
}

}  // namespace

size_t fused_batch_table_bytes(const BatchProblem *bp, int n) {
    size_t slices = 0;
    for (int i = 0; i < n; ++i)
        if (bp[i].p.n_sc > 0) slices += (size_t)(bp[i].p.K + kMaxKFused - 1) / kMaxKFused;
    return slices * sizeof(Entry);
}

void fused_batch_fill(const BatchProblem *bp, int n, void *host) {
    const Plan pl = make_plan(bp, n);
    if (!pl.e.empty()) memcpy(host, pl.e.data(), pl.e.size() * sizeof(Entry));
}

hipError_t fused_batch_launch(const BatchProblem *bp, int n, int precision, const void *dev, hipStream_t st,
                              int *launches) {
    const Plan pl = make_plan(bp, n);
    const int prec = prec_of(precision);
    const Entry *tab = (const Entry *)dev;
    int nl = 0;
    for (size_t r = 0; r < pl.cls.size(); ++r) {
        const int f = pl.first[r], cnt = pl.first[r + 1] - f;
        if (cnt == 0) continue;
        const Class c = pl.cls[r];
        hipError_t e;
        if (c.up == 16)
            e = c.arch == kPD ? launch_prec<16, kPD>(prec, c.maxt, tab + f, cnt, pl.blocks[r], pl.kmax[r], st)
                              : launch_prec<16, kFD>(prec, c.maxt, tab + f, cnt, pl.blocks[r], pl.kmax[r], st);
        else
            e = c.arch == kPD ? launch_prec<32, kPD>(prec, c.maxt, tab + f, cnt, pl.blocks[r], pl.kmax[r], st)
                              : launch_prec<32, kFD>(prec, c.maxt, tab + f, cnt, pl.blocks[r], pl.kmax[r], st);
        if (e != hipSuccess) return e;
        ++nl;
    }
    if (launches) *launches = nl;
    return hipSuccess;
}

}  // namespace pc
