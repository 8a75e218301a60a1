#!/usr/bin/env python3
"""Benchmark: PD-WF precoding throughput on one MI355X.

Workload: B = 256 antennas as 8 clusters of 32, U = 16 users, 1200
subcarriers x 14 OFDM symbols per frame, i.i.d. Rayleigh complex64 channel,
16-QAM symbols, SNR 10 dB (kappa = U / SNR).  A step precodes one frame:
Gram -> cluster sum -> regularize -> invert -> beta -> solve -> precode for
every subcarrier and symbol, in one fused launch.  The headline runs the
split-precision form: Gram and precode products as hi + lo FP16 MFMA (three
products, FP32 accumulation), inversion and solve in FP32; its error against
the FP64 oracle is reported with it (and the exact-FP32-product form's).  Frames rotate over enough distinct input/output
buffers that the working set exceeds the 256 MB last-level cache, so every
step streams its channel from HBM.

Prints one JSON line.  value = subcarrier-symbols precoded per second.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "precoded subcarriers/s (B=256,U=16) + p99 symbol latency vs plain, rel err ≤1e-3"
HBM_PEAK_GBS = 8000.0
HEAD_PREC = "split_fp16"
LLC_BYTES = 256 << 20


PROFILE = os.path.join(ROOT, "profiles", "fused_pd_b256_u16_n1200.md")
KERNEL_SOURCES = ["fused_kernel.h", "fused_nw.inc", "fused_launch.h", "common.h"]


def kernel_digest():
    """First 16 hex digits of the sha256 of the fused kernel's sources."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1804_10987_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed
    rocprofv3 counter summary, or None when the kernel's sources changed
    since those counters were taken (or there is no summary)."""
    try:
        fields = dict(l.split(": ", 1) for l in open(PROFILE).read().splitlines() if ": " in l and
                      l.split(": ", 1)[0] in ("traffic_bytes_per_launch", "kernel_source_digest", "traffic_kernel"))
    except OSError:
        return None, None
    if fields.get("kernel_source_digest", "").strip() != kernel_digest():
        return None, None
    return int(fields["traffic_bytes_per_launch"]), fields.get("traffic_kernel", "").strip()


def variant_params(pc, name):
    """Call parameters of a precision variant name: "<precision>" or
    "<precision>+refine1" (one fused FP64-residual refinement step)."""
    prec, _, ref = name.partition("+refine")
    return pc.params(precision=prec, impl="fused", refine_steps=int(ref) if ref else 0)


def algorithmic_bytes(B, U, K, n_sc):
    """HBM bytes the method must move per frame: the channel once, the symbols
    and the precoded vectors once (complex64)."""
    return 8 * n_sc * (B * U + K * U + K * B)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="headline launches only (for profiling)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the heterogeneous batch leg")
    ap.add_argument("--only-batch", action="store_true", help="run only the heterogeneous batch leg (for profiling)")
    ap.add_argument("--cell", type=int, default=2, choices=(2, 3),
                    help="2: the headline cell (B=256 as 8x32, U=16, 1200 subcarriers); 3: B=512 as 16x32, U=32, "
                         "3300 subcarriers, correlated channel (for profiling; the headline line is cell 2)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB float32 copy kernel 10 times (HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(clusters are batch entries on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1804_10987_amd as pc
    import synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        # elementwise kernel reading 1 GiB and writing 1 GiB per launch: the
        # reference for scaling the FETCH_SIZE / WRITE_SIZE counters
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(10):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_kernel": "torch.mul(a, 1.0, out=b), float32", "read_bytes": a.numel() * 4,
                          "write_bytes": b.numel() * 4, "launches": 10}), flush=True)
        return
    if args.only_batch:
        print(json.dumps({"batch_mix": batch_mix_leg(pc.Context(0), pc, dev, args)}), flush=True)
        return
    cell = synth.config(args.cell)
    B, U, K, n_sc, sizes = cell.B, cell.U, cell.K, cell.n_sc, list(cell.sizes)
    frame_bytes = algorithmic_bytes(B, U, K, n_sc)
    n_frames = max(2, math.ceil(2 * LLC_BYTES / frame_bytes))

    H0, s0 = synth.make_cell(cell, seed=0, frame=0)
    Hs, Ss, Xs = [], [], []
    for f in range(n_frames):
        H, s = (H0, s0) if f == 0 else synth.make_cell(cell, seed=0, frame=f)
        Hs.append(torch.from_numpy(H).to(dev))
        Ss.append(torch.from_numpy(s).to(dev))
        Xs.append(torch.empty((K, n_sc, B), dtype=torch.complex64, device=dev))
    betas = [torch.empty(n_sc, dtype=torch.float32, device=dev) for _ in range(n_frames)]
    stats = [torch.empty(n_sc, dtype=torch.int32, device=dev) for _ in range(n_frames)]
    torch.cuda.synchronize()

    ctx = pc.Context(0)
    stream = torch.cuda.current_stream()

    def time_path(fn, steps, warmup):
        """Eager: runs fn(frame) warmup + steps times, one host call per frame;
        returns (ms/step, per-launch ms list).  The per-launch times include
        any wait for the host to enqueue the next call."""
        for i in range(warmup):
            fn(i % n_frames)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for i in range(steps):
            ev[i][0].record(stream)
            fn(i % n_frames)
            ev[i][1].record(stream)
        t1.record(stream)
        torch.cuda.synchronize()
        total = t0.elapsed_time(t1)
        per = [a.elapsed_time(b) for a, b in ev]
        return total / steps, per

    def time_graph(fn, steps, warmup, n_streams=1):
        """The timed region as one HIP graph replay of exactly `steps` frames:
        fn(frame) for frames 0, 1, ... rotating over the frame buffers,
        recorded once into a graph (after `warmup` eager calls, which also
        settle the launch-shape autotuner), replayed once untimed, then once
        timed; returns (ms per frame, frames timed).  No host call sits
        between launches.  With n_streams > 1 the frames go round-robin to
        that many streams forked from and joined back into the graph's stream,
        so one frame's launch may overlap the next one's (each frame has its
        own buffers)."""
        for i in range(warmup):
            fn(i % n_frames)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        side = [torch.cuda.Stream() for _ in range(n_streams)] if n_streams > 1 else []
        with torch.cuda.graph(g, stream=cs):
            fork = torch.cuda.Event()
            fork.record(cs)
            for s_ in side:
                s_.wait_event(fork)
            for i in range(steps):
                f = i % n_frames
                if side:
                    with torch.cuda.stream(side[i % n_streams]):
                        fn(f)
                else:
                    fn(f)
            for s_ in side:
                join = torch.cuda.Event()
                join.record(s_)
                cs.wait_event(join)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        g.replay()
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps, steps

    def pd_fused(f, prec=HEAD_PREC):
        ctx.pd(Hs[f], Ss[f], cell.kappa, sizes, "wf", variant_params(pc, prec),
               x=Xs[f], beta=betas[f], status=stats[f], stream=torch.cuda.current_stream())

    def pd_plain(f):
        ctx.pd(Hs[f], Ss[f], cell.kappa, sizes, "wf", pc.params(impl="plain"),
               x=Xs[f], beta=betas[f], status=stats[f], stream=torch.cuda.current_stream())

    fd_w = [torch.empty((n_sc * len(sizes),), dtype=torch.float32, device=dev) for _ in range(n_frames)]
    fd_st = [torch.empty((n_sc * len(sizes),), dtype=torch.int32, device=dev) for _ in range(n_frames)]

    def fd_run(f, ratio=0.5, impl="auto"):
        ctx.fd(Hs[f], Ss[f], cell.kappa, sizes, "wf", pc.params(fp64_ratio=ratio, impl=impl),
               x=Xs[f], weights=fd_w[f], status=fd_st[f], stream=torch.cuda.current_stream())

    # ---- headline: PD-WF, fused, split FP16 ------------------------------
    # throughput and the kernel's average duration from graph replays (one
    # launch per frame, nothing else in the timed region)
    ms, steps_timed = time_graph(pd_fused, args.steps, args.warmup)
    value = n_sc * K / (ms * 1e-3)
    launch_ms = ms
    achieved = frame_bytes / (launch_ms * 1e-3) / 1e9
    traffic, traffic_kernel = measured_traffic() if args.cell == 2 else (None, None)
    traffic_src = ("rocprofv3 FETCH_SIZE + WRITE_SIZE of %s, scaled by a copy kernel's counts; %s"
                   % (traffic_kernel, os.path.relpath(PROFILE, ROOT))) if traffic else \
        "no counters for the current kernel sources"
    # per-frame latency of eager calls (host enqueue included)
    _, per = time_path(pd_fused, max(20, args.steps // 4), 2)
    per = np.array(per)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "subcarrier-symbols/s",
        "n_gpus": 1,
        "steps": steps_timed,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16 hi+lo split MFMA (3 products), fp32 accumulate; fp32 inversion and solve",
        "data": "synthetic",
        "config": {
            "workload": "PD-WF, B=%d as %d clusters x %d, U=%d, %d subcarriers x %d symbols, %s complex64, "
                        "%d-QAM, SNR %g dB" % (B, len(sizes), sizes[0], U, n_sc, K,
                                               "i.i.d. Rayleigh" if cell.channel == "rayleigh" else
                                               "Kronecker-correlated (r = %g)" % cell.r, cell.qam, cell.snr_db),
            "arch": "PD", "mode": "WF", "B": B, "C": len(sizes), "U": U, "n_sc": n_sc, "K": K,
            "impl": ctx.last_impl, "precision": HEAD_PREC, "frames_rotated": n_frames,
            "waves_per_workgroup": ctx.last_waves,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "fused_k (split FP16, one PD subcarrier per workgroup of %d waves)" % ctx.last_waves
                      if ctx.last_waves > 1 else "fused_k (split FP16, one PD subcarrier per wave)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "algorithmic_bytes_per_launch": frame_bytes,
            "launch_ms": launch_ms,
            "traffic": traffic,
            "traffic_source": traffic_src,
        },
        "latency": {"eager_frame_p50_ms": float(np.percentile(per, 50)),
                    "eager_frame_p99_ms": float(np.percentile(per, 99)),
                    "note": "one host call per frame; includes host enqueue time"},
    }
    variants = {}
    for prec in (() if args.quick else ("fp32", "split_bf16", "split_fp16+refine1", "split_bf16+refine1")):
        ms_v, _ = time_graph(lambda f, prec=prec: pd_fused(f, prec), args.steps, args.warmup)
        variants[prec] = {"ms_per_step": ms_v, "value": n_sc * K / (ms_v * 1e-3),
                          "achieved_gbs": frame_bytes / (ms_v * 1e-3) / 1e9, "waves_per_workgroup": ctx.last_waves}
    out["pd_precision_variants"] = variants
    if not args.quick:
        # consecutive frames on two streams: the next frame's loads overlap the
        # previous frame's inversion and tail (not the headline: each launch's
        # own duration grows under the overlap, so it stays out of the
        # profiling runs that time the headline kernel)
        ms_2s, _ = time_graph(pd_fused, args.steps, 3, n_streams=2)
        out["pd_two_streams"] = {"ms_per_frame": ms_2s, "value": n_sc * K / (ms_2s * 1e-3),
                                 "achieved_gbs": frame_bytes / (ms_2s * 1e-3) / 1e9,
                                 "note": "frames round-robin on 2 streams inside one graph, one launch per frame; "
                                         "throughput over the timed region"}
    # every launch shape the autotuner chooses from, forced
    shapes = {}
    for nw in (() if args.quick else (1, 2, 4)):
        os.environ["PRECODE_FUSED_WAVES"] = str(nw)
        ms_s, _ = time_graph(pd_fused, max(16, args.steps // 4), 3)
        shapes[str(nw)] = {"ms_per_step": ms_s, "used": ctx.last_waves}
    os.environ.pop("PRECODE_FUSED_WAVES", None)
    out["pd_launch_shapes"] = shapes
    if not args.quick:
        steps2 = max(10, args.steps // 4)
        ms_plain, _ = time_graph(pd_plain, steps2, 3)
        out["vs_plain"] = {"plain_ms_per_step": ms_plain, "speedup": ms_plain / ms,
                           "plain_value": n_sc * K / (ms_plain * 1e-3)}
        ms_fd32, _ = time_graph(lambda f: fd_run(f, ratio=2.0, impl="fused"), steps2, 3)
        ms_fd, _ = time_graph(lambda f: fd_run(f), steps2, 3)
        fd_impl = ctx.last_impl
        ms_fd_plain, _ = time_graph(lambda f: fd_run(f, ratio=2.0, impl="plain"), max(8, steps2 // 2), 2)
        ms_fd_plain64, _ = time_graph(lambda f: fd_run(f, impl="plain"), max(8, steps2 // 2), 2)
        out["fd"] = {
            "fused_fp32_ms_per_step": ms_fd32, "fused_fp32_value": n_sc * K / (ms_fd32 * 1e-3),
            "fused_fp32_achieved_gbs": frame_bytes / (ms_fd32 * 1e-3) / 1e9,
            "plain_fp32_ms_per_step": ms_fd_plain, "speedup_vs_plain": ms_fd_plain / ms_fd32,
            "note": "clusters of %d with U = %d meet U / B_c >= 0.5: the default routing takes the FP64 route"
                    % (sizes[0], U),
            "default_route_ms_per_step": ms_fd, "default_route_impl": fd_impl,
            "default_route_value": n_sc * K / (ms_fd * 1e-3),
            "plain_fp64_route_ms_per_step": ms_fd_plain64, "fp64_route_speedup_vs_plain": ms_fd_plain64 / ms_fd,
        }
    if not args.quick:
        out["comparison"] = comparison_leg(ctx, pc, Hs, Ss, Xs, cell, dev, time_graph, args)
    if not args.quick and not args.no_batch:
        out["batch_mix"] = batch_mix_leg(ctx, pc, dev, args)
    if not args.quick and not args.no_serving:
        out["serving"] = serving_leg(ctx, pc, Hs, Ss, cell, dev, args)
    if not args.no_cpu:
        out["cpu_baseline"], out["rel_err"] = cpu_baseline(cell, Hs[0], Ss[0], Xs[0], betas[0], ctx, pc, stream,
                                                           (HEAD_PREC, "fp32", "split_bf16", "split_fp16+refine1",
                                                            "split_bf16+refine1"))
    print(json.dumps(out), flush=True)


FP32_VECTOR_PEAK_TFLOPS = 157.3


def central_flops(B, U, K):
    """Real flops per subcarrier of centralized WF in the B x B form: the
    lower triangle of M = H H^H (4 B^2 U), its Cholesky (4 B^3 / 3), the
    forward and back substitution with U right-hand sides (8 B^2 U) and the
    precode Q s (8 K B U); one complex multiply-add counts 8."""
    return 4 * B * B * U + 4 * B ** 3 / 3 + 8 * B * B * U + 8 * K * B * U


def comparison_leg(ctx, pc, Hs, Ss, Xs, cell, dev, time_graph, args):
    """The comparison precoders and the UE side of the BER link at the
    headline shape, each on graph replay over the rotating frames."""
    import torch

    import synth
    from paper_1804_10987_amd import ber

    n_sc, B, U, K, sizes = cell.n_sc, cell.B, cell.U, cell.K, list(cell.sizes)
    nf = len(Hs)
    steps = max(8, args.steps // 8)
    beta = torch.empty(n_sc, dtype=torch.float32, device=dev)
    st = torch.empty(n_sc, dtype=torch.int32, device=dev)
    w = torch.empty(n_sc * len(sizes), dtype=torch.float32, device=dev)
    wst = torch.empty(n_sc * len(sizes), dtype=torch.int32, device=dev)
    cur = torch.cuda.current_stream

    def central(f):
        ctx.central(Hs[f], Ss[f], cell.kappa, x=Xs[f], beta=beta, status=st, stream=cur())

    def mrt(f):
        ctx.mrt(Hs[f], Ss[f], sizes, x=Xs[f], weights=w, status=wst, stream=cur())

    noise = torch.zeros((K, n_sc, U), dtype=torch.complex64, device=dev)
    y = torch.empty((K, n_sc, U), dtype=torch.complex64, device=dev)

    def receive(f):
        pc.ue_receive(Hs[f], Xs[f], noise, 0.1, beta, s_hat=y, stream=cur())

    out = {}
    ms_c, _ = time_graph(central, max(4, steps // 4), 2)
    fl = central_flops(B, U, K) * n_sc
    out["central_wf_bxb"] = {
        "ms_per_frame": ms_c, "value": n_sc * K / (ms_c * 1e-3),
        "roofline": {"bound": "alu", "achieved": fl / (ms_c * 1e-3) / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": fl / (ms_c * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                     "flops_per_frame": fl},
        "note": "Theorem 1's B x B form: FP32 tiled Cholesky of M = H H^H + kappa I_B per subcarrier"}
    ms_m, _ = time_graph(mrt, steps, 3)
    by = algorithmic_bytes(B, U, K, n_sc)
    out["mrt"] = {"ms_per_frame": ms_m, "value": n_sc * K / (ms_m * 1e-3),
                  "roofline": {"bound": "hbm", "achieved": by / (ms_m * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": by / (ms_m * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    ms_r, _ = time_graph(receive, steps, 3)
    by_r = 8 * n_sc * (B * U + K * B + 2 * K * U)
    out["ue_receive"] = {"ms_per_frame": ms_r,
                         "roofline": {"bound": "hbm", "achieved": by_r / (ms_r * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": by_r / (ms_r * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                      "bytes_per_frame": by_r}}
    # one whole PD link frame (QAM map, precode, receive, decisions, count), eager
    lcell = cell.with_(qam=64, snr_db=0.0)
    H, lab, wn = synth.device_link_frame(lcell, dev, seed=7, frame=0)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(2):
        ber.frame_errors(ctx, "pd", H, lab, wn, lcell.snr_db, lcell.qam, sizes, count=count)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        ber.frame_errors(ctx, "pd", H, lab, wn, lcell.snr_db, lcell.qam, sizes, count=count)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    out["ber_link_pd"] = {"ms_per_frame": dt * 1e3, "bits_per_s": n_sc * K * U * 6 / dt,
                          "note": "64-QAM, eager host calls (map, precode, receive, count) per frame"}
    return out


SYMBOL_PERIOD_S = 1e-3 / 14  # LTE: 14 OFDM symbols per 1 ms subframe


def serving_leg(ctx, pc, Hs, Ss, cell, dev, args):
    """Continuous-batching serving (precode_serve): per-frame jobs arrive as a
    Poisson process, each frame's 14 symbols are released one symbol period
    apart and precoded from the resident factors.  Reports per-symbol latency
    (completion - release) p50/p99 and throughput for the fused kernels and
    for the plain kernels in the same loop, at swept arrival rates; then the
    same for a heterogeneous cell mix."""
    import numpy as np
    import torch

    import synth

    def run(jobs, arr, impl, period=SYMBOL_PERIOD_S, max_active=16, slab_gib=4):
        _, lat, st = ctx.serve(jobs, arr, symbol_period_s=period, max_active=max_active, n_streams=4,
                               impl=impl, slab_bytes=slab_gib << 30)
        torch.cuda.synchronize()
        return {"p50_us": st["lat_p50_s"] * 1e6, "p99_us": st["lat_p99_s"] * 1e6,
                "max_us": st["lat_max_s"] * 1e6, "wait_p99_us": st["wait_p99_s"] * 1e6,
                "throughput": st["throughput"], "peak_active": st["peak_active"],
                "peak_slab_mb": st["peak_bytes"] / 2**20}

    n_jobs = 96
    xs = [torch.empty((cell.K, cell.n_sc, cell.B), dtype=torch.complex64, device=dev) for _ in range(n_jobs)]
    jobs = [dict(arch="pd", mode="wf", H=Hs[i % len(Hs)], s=Ss[i % len(Ss)], x=xs[i], rho=cell.kappa,
                 sizes=cell.sizes) for i in range(n_jobs)]
    res = {"workload": "PD-WF frames of the headline cell (B=256 8x32, U=16, 1200 subcarriers), 14 symbols "
                       "each released every %.1f us, Poisson frame arrivals" % (SYMBOL_PERIOD_S * 1e6),
           "jobs": n_jobs, "max_active": 16, "streams": 4, "rates": {}}
    run(jobs[:8], [0.0] * 8, "auto")  # warm the loop and kernels
    run(jobs[:8], [0.0] * 8, "plain")
    for rate in (1000.0, 4000.0, 16000.0):
        arr = synth.poisson_arrivals(rate, n_jobs, seed=7).tolist()
        f = run(jobs, arr, "auto")
        p = run(jobs, arr, "plain")
        res["rates"]["%g/s" % rate] = {"fused": f, "plain": p, "p99_plain_over_fused": p["p99_us"] / f["p99_us"]}
    # saturation: every frame at t=0 with all symbols released at once
    f = run(jobs, [0.0] * n_jobs, "auto", period=0.0)
    p = run(jobs, [0.0] * n_jobs, "plain", period=0.0)
    res["saturated"] = {"fused": f, "plain": p, "throughput_fused_over_plain": f["throughput"] / p["throughput"]}
    del xs, jobs
    # heterogeneous mix (B in 64..512, cluster sizes 16/32/64, U 4..64, 300/1200/3300 subcarriers)
    cells = synth.mix(48, seed=11)
    mjobs = []
    for i, c in enumerate(cells):
        H, s = synth.device_cell(c, dev, seed=11, cell_id=i)
        mjobs.append(dict(arch="pd" if i % 2 == 0 else "fd", mode="wf", H=H, s=s, rho=c.kappa, sizes=c.sizes))
    arr = synth.poisson_arrivals(2000.0, len(mjobs), seed=11).tolist()
    # plain-kernel jobs of the mix keep up to ~2.6 GiB each resident (FP64-width workspace); 16 slots
    f = run(mjobs, arr, "auto", slab_gib=64)
    p = run(mjobs, arr, "plain", slab_gib=64)
    res["mix"] = {"cells": len(cells), "rate": "2000/s", "slab_gib": 64, "pd_fd": "alternating", "fused": f, "plain": p,
                  "p99_plain_over_fused": p["p99_us"] / f["p99_us"]}
    return res


def batch_mix_leg(ctx, pc, dev, args):
    """The heterogeneous batch: 64 cells of the mix (B in 64..512, clusters of
    16/32/64 antennas or uneven, U in 4..64, 300/1200/3300 subcarriers, 14
    symbols, PD and FD alternating), channels and symbols drawn on the device,
    as one batch plan (a HIP graph: register-tile classes, one-wave FP64 and
    wide FP64 launches) replayed, against the plain kernels (one call per
    cell, recorded into one graph)."""
    import torch

    import synth

    res = {}
    for uneven in (False, True):
        cells = synth.mix(64, seed=0, uneven=uneven)
        jobs = []
        for i, c in enumerate(cells):
            H, s = synth.device_cell(c, dev, seed=21, cell_id=i)
            jobs.append(dict(arch="pd" if i % 2 == 0 else "fd", mode="wf", H=H, s=s, rho=c.kappa, sizes=c.sizes))
        units = sum(c.n_sc * c.K for c in cells)
        plan = ctx.batch_plan(jobs)
        plan.launch()
        torch.cuda.synchronize()
        reps = 5
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            plan.launch()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        fused_jobs, launches = plan.fused_jobs, plan.launches
        xs = [o[0] for o in plan.outputs]

        def plain_call(i):
            j = jobs[i]
            fn = ctx.pd if j["arch"] == "pd" else ctx.fd
            fn(j["H"], j["s"], j["rho"], j["sizes"], "wf", pc.params(impl="plain"), x=xs[i])

        for i in range(len(jobs)):  # grows the plain workspace outside the capture
            plain_call(i)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        with torch.cuda.graph(g, stream=cs):
            for i in range(len(jobs)):
                plain_call(i)
        g.replay()
        torch.cuda.synchronize()
        t0.record()
        g.replay()
        t1.record()
        torch.cuda.synchronize()
        ms_plain = t0.elapsed_time(t1)
        res["uneven" if uneven else "even"] = {
            "cells": len(cells), "subcarrier_symbols": units, "fused_jobs": fused_jobs, "launches": launches,
            "ms_per_batch": ms, "value": units / (ms * 1e-3),
            "plain_ms_per_batch": ms_plain, "speedup_vs_plain": ms_plain / ms,
            "hbm_gb": sum(8 * c.n_sc * (c.B * c.U + c.K * (c.U + c.B)) for c in cells) / 1e9}
        plan.destroy()
        del plan, jobs, xs, g
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    res["precision"] = "fp32 (register tiles); FP64 on the one-wave and wide FP64 kernels"
    return res


def cpu_model():
    """The host CPU's model name (lscpu's "Model name", from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_oracle(cell, H, s, threads, min_s):
    """Subcarrier-symbols per second of the FP64 oracle on `threads` host
    threads over the given frame (H, s), repeated until min_s of wall time."""
    import oracle

    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.pd(H, s, cell.kappa, cell.sizes, threads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_s:
            break
    return reps * H.shape[0] * s.shape[0] / el, reps, el


def cpu_baseline(cell, Hd, sd, xd, bd, ctx, pc, stream, precs):
    """The FP64 oracle on the host cores over the same frame (repeated until
    about 2 s of wall time), on one core, and on bounded samples of the tiny
    and the precision workloads; and the GPU's error against it on that
    frame for each precision in precs."""
    import numpy as np
    import torch

    import oracle
    import synth

    H, s = synth.make_cell(cell, seed=0, frame=0)
    gpu = {}
    for prec in precs:
        ctx.pd(Hd, sd, cell.kappa, list(cell.sizes), "wf", variant_params(pc, prec), x=xd, beta=bd, stream=stream)
        torch.cuda.synchronize()
        gpu[prec] = (xd.cpu().numpy(), bd.cpu().numpy())
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = min(threads, int(os.environ.get("OMP_NUM_THREADS", threads)))
    oracle.build(force=False)
    xo, bo, st = oracle.pd(H, s, cell.kappa, cell.sizes, threads=threads)
    value, reps, el = time_oracle(cell, H, s, threads, 2.0)
    one, reps1, el1 = time_oracle(cell, H[:300], s[:, :300], 1, 2.0)
    others = {}
    for i, frac in ((1, 1), (3, 8)):
        c = synth.config(i)
        Hc, sc_ = synth.make_cell(c, seed=0, frame=0)
        n = max(1, c.n_sc // frac)
        v, r, e_ = time_oracle(c, Hc[:n], sc_[:, :n], threads, 1.0)
        others[str(i)] = {"value": v, "cores": threads,
                          "sample": "%d x %d subcarriers x %d symbols (B=%d, U=%d), %.2f s wall"
                                    % (r, n, c.K, c.B, c.U, e_)}
    rel = {"vs": "FP64 oracle, full frame 0; per (subcarrier, symbol) ||x - x_oracle|| / ||x_oracle||"}
    for prec, (xg, bg) in gpu.items():
        e = np.linalg.norm(xg - xo, axis=-1) / np.linalg.norm(xo, axis=-1)
        rel[prec] = {"max": float(e.max()), "p99": float(np.percentile(e, 99)), "p50": float(np.percentile(e, 50)),
                     "beta_max": float(np.max(np.abs(bg - bo) / bo))}
    return ({"value": value, "unit": "subcarrier-symbols/s", "cores": threads, "kind": "oracle",
             "sample": "%d full frame(s) (1200 subcarriers x 14 symbols), %.2f s wall" % (reps, el),
             "cpu_model": cpu_model(),
             "one_core": {"value": one, "cores": 1,
                          "sample": "%d x 300 subcarriers x 14 symbols, %.2f s wall" % (reps1, el1)},
             "workloads": others}, rel)


if __name__ == "__main__":
    main()
