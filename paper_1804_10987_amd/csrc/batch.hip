// batch.hip -- heterogeneous batches of fused PD / FD problems (cells of
// different B, cluster sizes, U and subcarrier counts) in as few launches as
// the kernels' shape classes allow.
//
// Register-tile problems are grouped by tile width UP (16 for U <= 16, 32
// for U <= 32), channel tiles per wave held in registers (1, 2, 4 or
// streamed) and load width (U == UP with an aligned channel, or not); wide
// problems (wide.hip: U <= 64, B_c < U, FP64 route) by system order (16, 32,
// 48 or 64; an FD problem's clusters each in their own class).  Each group -- PD and FD problems alike -- is one launch whose grid is
// the sum of its problems' workgroups.  The problem table sits in device
// memory; a workgroup finds its problem by binary search over the problems'
// first block index and then runs the same body as the single-problem kernel.
// Problems of the one-wave FP64 kernel launch one by one.
#include <string.h>

#include <algorithm>
#include <vector>

#include "fused_kernel.h"

namespace pc {
namespace {

constexpr int NW = 4;  // waves per workgroup of the batch launches

using Entry = BatchEntry;

// Launch class of a problem: wide or not, tile width (system order for
// wide problems), register tiles per wave and load width.
struct Class {
    int wide, up, maxt, vec;
    bool operator==(const Class &o) const { return wide == o.wide && up == o.up && maxt == o.maxt && vec == o.vec; }
    bool operator<(const Class &o) const {
        if (wide != o.wide) return wide < o.wide;
        return up != o.up ? up < o.up : (maxt != o.maxt ? maxt < o.maxt : vec < o.vec);
    }
};

Class class_of(const BatchProblem &q) {
    if (q.kind == kBatchWide) return Class{1, wide_order(q.p), 0, 0};
    return Class{0, pick_up(q.p.U), pick_maxt(q.p), pick_vec(q.p, q.H) ? 1 : 0};
}

bool in_table(const BatchProblem &q) { return q.kind != kBatchF64; }

// Table entries in launch order (by class, then problem order).  A wide FD
// problem whose clusters fall into different order classes gets one entry
// per cluster (cl >= 0), each in its own cluster's class.
struct Plan {
    std::vector<Entry> e;
    std::vector<Class> cls;   // class of each run
    std::vector<int> first;   // first entry of each run, plus the end
    std::vector<int> blocks;  // grid of each run
};

struct Unit {
    int prob, cl;
    Class c;
};

Plan make_plan(const BatchProblem *bp, int n) {
    std::vector<Unit> units;
    for (int i = 0; i < n; ++i) {
        const BatchProblem &q = bp[i];
        if (!in_table(q) || q.p.n_sc == 0) continue;
        const Class c = class_of(q);
        bool split = false;
        if (q.kind == kBatchWide && q.p.arch == kFD)
            for (int cl = 0; cl < q.p.C; ++cl) split = split || wide_cluster_order(q.p, cl) != c.up;
        if (!split) {
            units.push_back(Unit{i, -1, c});
        } else {
            for (int cl = 0; cl < q.p.C; ++cl) units.push_back(Unit{i, cl, Class{1, wide_cluster_order(q.p, cl), 0, 0}});
        }
    }
    std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) { return a.c < b.c; });
    Plan pl;
    for (const Unit &u : units) {
        const BatchProblem &q = bp[u.prob];
        if (pl.cls.empty() || !(pl.cls.back() == u.c)) {
            pl.cls.push_back(u.c);
            pl.first.push_back((int)pl.e.size());
            pl.blocks.push_back(0);
        }
        Entry en;
        en.p = q.p;
        en.H = q.H;
        en.s = q.s;
        en.x = q.x;
        en.scale_out = q.scale_out;
        en.status = q.status;
        en.K = q.p.K;
        en.block0 = pl.blocks.back();
        en.cl = u.cl;
        pl.blocks.back() += u.cl >= 0 ? q.p.n_sc : (u.c.wide ? n_inst(q.p) : blocks_for(q.p, NW));
        pl.e.push_back(en);
    }
    pl.first.push_back((int)pl.e.size());
    return pl;
}

template <int UP, int PREC, int MAXT, bool VEC>
__global__ void __launch_bounds__(64 * NW, (min_waves<UP, MAXT, PREC>()))
    fused_batch_k(const Entry *__restrict__ tab, int n) {
    const int b = blockIdx.x;
    int lo = 0, hi = n - 1;  // last problem with block0 <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    const Entry &E = tab[lo];
    fused_body<UP, PREC, NW, MAXT, VEC, false>(E.p, &E.p, b - E.block0, E.K, kFull, E.H, E.s, E.x, nullptr, E.scale_out,
                                   E.status);
}

template <int UP, int PREC, int MAXT, bool VEC>
hipError_t launch(const Entry *tab, int n, int blocks, hipStream_t st) {
    const void *fn = (const void *)fused_batch_k<UP, PREC, MAXT, VEC>;
    const size_t lds = Lds<UP>::bytes(NW);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((fused_batch_k<UP, PREC, MAXT, VEC>), dim3(blocks), dim3(64 * NW), lds, st, tab, n);
    return hipGetLastError();
}

template <int UP, int PREC, bool VEC>
hipError_t launch_v(int maxt, const Entry *tab, int n, int blocks, hipStream_t st) {
    switch (maxt) {
        case 0: return launch<UP, PREC, 0, VEC>(tab, n, blocks, st);
        case 1: return launch<UP, PREC, 1, VEC>(tab, n, blocks, st);
        case 2: return launch<UP, PREC, 2, VEC>(tab, n, blocks, st);
        case 4: return launch<UP, PREC, 4, VEC>(tab, n, blocks, st);
        default: return hipErrorNotSupported;
    }
}

template <int UP>
hipError_t launch_prec(int prec, int maxt, int vec, const Entry *tab, int n, int blocks, hipStream_t st) {
    switch (prec) {
        case kF32: return vec ? launch_v<UP, kF32, true>(maxt, tab, n, blocks, st)
                              : launch_v<UP, kF32, false>(maxt, tab, n, blocks, st);
        case kF16: return vec ? launch_v<UP, kF16, true>(maxt, tab, n, blocks, st)
                              : launch_v<UP, kF16, false>(maxt, tab, n, blocks, st);
        default: return vec ? launch_v<UP, kBF16, true>(maxt, tab, n, blocks, st)
                            : launch_v<UP, kBF16, false>(maxt, tab, n, blocks, st);
    }
}

}  // namespace

size_t fused_batch_table_bytes(const BatchProblem *bp, int n) {
    return make_plan(bp, n).e.size() * sizeof(Entry);
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
        if (c.wide) e = wide_batch_launch(c.up, tab + f, cnt, pl.blocks[r], st);
        else if (c.up == 16) e = launch_prec<16>(prec, c.maxt, c.vec, tab + f, cnt, pl.blocks[r], st);
        else e = launch_prec<32>(prec, c.maxt, c.vec, tab + f, cnt, pl.blocks[r], st);
        if (e != hipSuccess) return e;
        ++nl;
    }
    for (int i = 0; i < n; ++i) {
        const BatchProblem &q = bp[i];
        if (q.kind != kBatchF64 || q.p.n_sc == 0) continue;
        const hipError_t e = fused_f64_run(q.p, q.H, q.s, q.x, q.scale_out, q.status, st);
        if (e != hipSuccess) return e;
        ++nl;
    }
    if (launches) *launches = nl;
    return hipSuccess;
}

}  // namespace pc
