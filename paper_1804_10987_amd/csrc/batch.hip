// batch.hip -- heterogeneous batches of fused PD / FD problems (cells of
// different B, cluster sizes, U and subcarrier counts) in as few launches as
// the kernel's shape classes allow.
//
// Problems are grouped by tile width UP (16 for U <= 16, 32 for U <= 32);
// each group -- PD and FD problems alike -- is one launch whose grid is the
// sum of its problems' workgroups (one wave per local system, NW systems per
// workgroup).  The problem table sits in device memory; a workgroup finds its
// problem by binary search over the problems' first block index and then runs
// the same body as the single-problem kernel.
#include <string.h>

#include <algorithm>
#include <vector>

#include "fused_kernel.h"

namespace pc {
namespace {

constexpr int NW = 4;  // waves per workgroup of the batch launches

struct Entry {
    Prob p;
    const float2 *H, *s;
    float2 *x;
    float *scale_out;
    int *status;
    int K;       // symbols
    int block0;  // first block of this problem within its class launch
};

// Launch class of a problem: its tile width.
int class_of(const Prob &p) { return pick_up(p.U); }

// Problems in launch order (by class, then problem order).
struct Plan {
    std::vector<Entry> e;
    std::vector<int> cls;     // class (tile width) of each run
    std::vector<int> first;   // first entry of each run, plus the end
    std::vector<int> blocks;  // grid of each run
    std::vector<int> rows;    // largest system of each run (rows, multiple of 32)
};

Plan make_plan(const BatchProblem *bp, int n) {
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return class_of(bp[a].p) < class_of(bp[b].p); });
    Plan pl;
    for (int oi = 0; oi < n; ++oi) {
        const BatchProblem &q = bp[order[oi]];
        const int c = class_of(q.p);
        if (pl.cls.empty() || pl.cls.back() != c) {
            pl.cls.push_back(c);
            pl.first.push_back((int)pl.e.size());
            pl.blocks.push_back(0);
            pl.rows.push_back(0);
        }
        if (q.p.n_sc == 0) continue;
        Entry en;
        en.p = q.p;
        en.H = q.H;
        en.s = q.s;
        en.x = q.x;
        en.scale_out = q.scale_out;
        en.status = q.status;
        en.K = q.p.K;
        en.block0 = pl.blocks.back();
        pl.blocks.back() += blocks_for(q.p, NW);
        pl.rows.back() = std::max(pl.rows.back(), system_rows(q.p));
        pl.e.push_back(en);
    }
    pl.first.push_back((int)pl.e.size());
    return pl;
}

template <int UP, int PREC, bool STAGE>
__global__ void __launch_bounds__(64 * NW, (min_waves<UP, STAGE>()))
    fused_batch_k(const Entry *__restrict__ tab, int n, int stage_rows) {
    const int b = blockIdx.x;
    int lo = 0, hi = n - 1;  // last problem with block0 <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const Entry &E = tab[lo];
    fused_body<UP, PREC, NW, STAGE>(E.p, E.p.off, b - E.block0, E.K, kFull, stage_rows, E.H, E.s, E.x, nullptr,
                             E.scale_out, E.status);
}

template <int UP, int PREC, bool STAGE>
hipError_t launch1(const Entry *tab, int n, int blocks, int stage, hipStream_t st) {
    const void *fn = (const void *)fused_batch_k<UP, PREC, STAGE>;
    const size_t lds = Lds<UP>::bytes(NW, stage);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((fused_batch_k<UP, PREC, STAGE>), dim3(blocks), dim3(64 * NW), lds, st, tab, n, stage);
    return hipGetLastError();
}

template <int UP, int PREC>
hipError_t launch(const Entry *tab, int n, int blocks, int rows, hipStream_t st) {
    const int stage = stage_rows_for(UP, rows, NW);
    return stage > 0 ? launch1<UP, PREC, true>(tab, n, blocks, stage, st)
                     : launch1<UP, PREC, false>(tab, n, blocks, 0, st);
}

template <int UP>
hipError_t launch_prec(int prec, const Entry *tab, int n, int blocks, int rows, hipStream_t st) {
    switch (prec) {
        case kF32: return launch<UP, kF32>(tab, n, blocks, rows, st);
        case kF16: return launch<UP, kF16>(tab, n, blocks, rows, st);
        default: return launch<UP, kBF16>(tab, n, blocks, rows, st);
    }
}

}  // namespace

size_t fused_batch_table_bytes(const BatchProblem *bp, int n) {
    size_t cnt = 0;
    for (int i = 0; i < n; ++i)
        if (bp[i].p.n_sc > 0) ++cnt;
    return cnt * sizeof(Entry);
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
        const hipError_t e = pl.cls[r] == 16 ? launch_prec<16>(prec, tab + f, cnt, pl.blocks[r], pl.rows[r], st)
                                             : launch_prec<32>(prec, tab + f, cnt, pl.blocks[r], pl.rows[r], st);
        if (e != hipSuccess) return e;
        ++nl;
    }
    if (launches) *launches = nl;
    return hipSuccess;
}

}  // namespace pc
