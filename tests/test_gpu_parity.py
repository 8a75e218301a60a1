"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Error metric: e = ||x_gpu - x_oracle||_2 / ||x_oracle||_2 per (subcarrier,
symbol) B-vector; the FP32 paths must reach max e <= 1e-5, and beta / FD
weights relative error <= 1e-5.  Status flags must agree exactly.
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def pc(torch):
    import paper_1804_10987_amd as m

    return m


@pytest.fixture(scope="module")
def ctx(pc):
    return pc.Context(0)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _vec_err(xg, xo):
    num = np.linalg.norm(xg - xo, axis=-1)
    den = np.linalg.norm(xo, axis=-1)
    return num / np.where(den > 0, den, 1.0)


def _run(torch, ctx, pc, arch, H, s, kappa, sizes, mode, **prm):
    Hd, sd = _dev(torch, H), _dev(torch, s)
    fn = ctx.pd if arch == "pd" else ctx.fd
    x, sc, st = fn(Hd, sd, kappa, sizes, mode, pc.params(**prm))
    torch.cuda.synchronize()
    return x.cpu().numpy(), sc.cpu().numpy(), st.cpu().numpy()


def _oracle(arch, H, s, kappa, sizes, mode, tau=0.125, power=1.0, Es=1.0):
    if arch == "pd":
        return oracle.pd(H, s, kappa, sizes, zf=(mode == "zf"), power=power, Es=Es)
    return oracle.fd(H, s, kappa, sizes, zf=(mode == "zf"), tau=tau, power=power, Es=Es)


def _check(xg, scg, stg, xo, sco, sto, tol=TOL):
    assert (stg & 1 == sto).all(), (stg, sto)
    ok = sto == 0
    e = _vec_err(xg, xo)
    assert np.isfinite(xg).all()
    assert e.max() <= tol, "max rel err %.3e" % e.max()
    rel = np.abs(scg - sco) / np.where(sco > 0, sco, 1.0)
    assert rel[ok].max(initial=0) <= tol, "scale rel err %.3e" % rel.max()
    return e.max()


CASES = [
    # name, cell, mode
    ("cfg1", synth.config(1), "wf"),
    ("cfg1_zf", synth.config(1), "zf"),
    ("ragged", synth.Cell(B=100, sizes=(37, 63), U=13, n_sc=37, K=19, snr_db=5.0, qam=16), "wf"),
    ("ragged_zf", synth.Cell(B=100, sizes=(37, 63), U=13, n_sc=37, K=19, snr_db=5.0, qam=16), "zf"),
    ("u32", synth.Cell(B=128, sizes=(64, 64), U=32, n_sc=20, K=14, snr_db=10.0), "wf"),
    ("u1", synth.Cell(B=16, sizes=(16,), U=1, n_sc=9, K=3, snr_db=0.0), "wf"),
    ("k1", synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=5, K=1), "wf"),
    ("k70", synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=6, K=70), "wf"),
    ("many_clusters", synth.Cell(B=96, sizes=(12,) * 8, U=6, n_sc=11, K=14, qam=64), "wf"),
    ("u20_kron", synth.Cell(B=160, sizes=(40, 40, 80), U=20, n_sc=13, K=17, channel="kron", r=0.5), "wf"),
    # PD rows past one wave's registers: split over the waves of a workgroup
    ("b256", synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=20, K=14), "wf"),
    ("b300_ragged", synth.Cell(B=300, sizes=(100, 200), U=12, n_sc=9, K=19, snr_db=5.0), "wf"),
]


# (impl, precision, tolerance): FP32 paths 1e-5; split 16-bit MFMA (hi + lo,
# three products, FP32 accumulation) FP16 1e-5, BF16 1e-3 (the reduced-precision
# bound; its hi + lo keeps ~16 mantissa bits per operand)
PATHS = [("fused", "fp32", 1e-5), ("plain", "fp32", 1e-5), ("fused", "split_fp16", 1e-5),
         ("fused", "split_bf16", 1e-3)]


@pytest.mark.parametrize("impl,prec,tol", PATHS, ids=["%s-%s" % (a, b) for a, b, _ in PATHS])
@pytest.mark.parametrize("arch", ["pd", "fd"])
@pytest.mark.parametrize("name,cell,mode", CASES, ids=[c[0] for c in CASES])
def test_parity(torch, ctx, pc, name, cell, mode, arch, impl, prec, tol):
    H, s = synth.make_cell(cell, seed=11)
    print("case", name, arch, mode, impl, prec, flush=True)
    # keep every instance on the FP32 path here (the FP64 route has its own test)
    xg, scg, stg = _run(torch, ctx, pc, arch, H, s, cell.kappa, cell.sizes, mode, impl=impl, fp64_ratio=2.0,
                        precision=prec)
    assert ctx.last_impl == impl
    xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, mode)
    e = _check(xg, scg, stg, xo, sco, sto, tol=tol)
    print("max rel err %.3e" % e, flush=True)


@pytest.mark.parametrize("arch", ["pd", "fd"])
def test_power_and_params(torch, ctx, pc, arch):
    cell = synth.Cell(B=64, sizes=(16, 48), U=8, n_sc=7, K=5)
    H, s = synth.make_cell(cell, seed=3)
    for impl in ("fused", "plain"):
        xg, scg, stg = _run(torch, ctx, pc, arch, H, s, 0.4, cell.sizes, "wf", impl=impl, power=2.5, Es=0.7,
                            tau=0.3, fp64_ratio=2.0)
        xo, sco, sto = _oracle(arch, H, s, 0.4, cell.sizes, "wf", tau=0.3, power=2.5, Es=0.7)
        _check(xg, scg, stg, xo, sco, sto)


@pytest.mark.parametrize("impl", ["auto", "plain"])
def test_fd_small_clusters_auto(torch, ctx, pc, impl):
    """FD with clusters smaller than U (B_c x B_c branch) and square clusters
    (FP64 route by the default ratio 0.5): on the plain kernels each cluster
    takes its own route; by default the whole cell runs on the wide FP64
    kernel (every cluster flagged FP64)."""
    cell = synth.Cell(B=44, sizes=(4, 12, 8, 20), U=8, n_sc=9, K=6)
    H, s = synth.make_cell(cell, seed=5)
    for mode in ("wf", "zf"):
        xg, scg, stg = _run(torch, ctx, pc, "fd", H, s, cell.kappa, cell.sizes, mode, impl=impl)
        assert ctx.last_impl == ("plain" if impl == "plain" else "fused")
        xo, sco, sto = _oracle("fd", H, s, cell.kappa, cell.sizes, mode)
        _check(xg, scg, stg, xo, sco, sto)
        if impl == "plain":
            # clusters with U / B_c >= 0.5 ran on the FP64 route
            assert ((stg[:, [0, 1, 2]] & 2) == 2).all() and ((stg[:, 3] & 2) == 0).all()
        else:
            assert ((stg & 2) == 2).all()


def test_fp64_route_square(torch, ctx, pc):
    """B_c = U: ill-conditioned local systems go to the FP64 route and meet 1e-5."""
    cell = synth.Cell(B=64, sizes=(16,) * 4, U=16, n_sc=40, K=14, snr_db=20.0)
    H, s = synth.make_cell(cell, seed=7)
    xg, scg, stg = _run(torch, ctx, pc, "fd", H, s, cell.kappa, cell.sizes, "wf")
    xo, sco, sto = _oracle("fd", H, s, cell.kappa, cell.sizes, "wf")
    assert (stg == 2).all()
    _check(xg, scg, stg, xo, sco, sto)
    # PD with precision=fp64
    xg, scg, stg = _run(torch, ctx, pc, "pd", H, s, cell.kappa, cell.sizes, "wf", precision="fp64")
    xo, sco, sto = _oracle("pd", H, s, cell.kappa, cell.sizes, "wf")
    _check(xg, scg, stg, xo, sco, sto, tol=1e-6)


@pytest.mark.parametrize("cell", [
    synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=37, K=14, snr_db=10.0),         # U / B_c = 0.5
    synth.Cell(B=64, sizes=(16,) * 4, U=16, n_sc=23, K=19, snr_db=20.0),          # B_c = U
    synth.Cell(B=47, sizes=(11, 14, 22), U=11, n_sc=15, K=5, snr_db=5.0, qam=16),  # ragged, U < 16
    synth.Cell(B=5, sizes=(1, 2, 2), U=1, n_sc=7, K=3, snr_db=0.0),                 # U = 1, tiny clusters
    synth.Cell(B=128, sizes=(32,) * 4, U=32, n_sc=11, K=14, snr_db=10.0, channel="kron"),  # B_c = U = 32
    synth.Cell(B=88, sizes=(40, 48), U=24, n_sc=9, K=17, snr_db=5.0),            # two row tiles, U in 17..32
    synth.Cell(B=64, sizes=(64,), U=20, n_sc=6, K=3, snr_db=15.0),               # B_c = 64 (ratio 0.3)
], ids=["b256_bc32_u16", "bc16_u16", "ragged_u11", "u1_tiny", "bc32_u32", "bc40_48_u24", "bc64_u20"])
@pytest.mark.parametrize("mode", ["wf", "zf"])
def test_fd_fp64_route_fused(torch, ctx, pc, cell, mode):
    """FD whose every cluster takes the FP64 route (U / B_c >= the ratio) with
    U <= 32 and U <= B_c <= 64 runs in one fused launch (Gram, inversion and
    solve in FP64, precode on FP32 MFMA): against the oracle and against the
    plain FP64 kernels; every instance flagged FP64."""
    H, s = synth.make_cell(cell, seed=21)
    ratio = min(cell.U / b for b in cell.sizes)
    xg, scg, stg = _run(torch, ctx, pc, "fd", H, s, cell.kappa, cell.sizes, mode, fp64_ratio=min(0.5, ratio))
    assert ctx.last_impl == "fused" and ctx.last_waves == 4
    assert ((stg & 2) == 2).all()
    xo, sco, sto = _oracle("fd", H, s, cell.kappa, cell.sizes, mode)
    _check(xg, scg, stg, xo, sco, sto)
    xp, scp, stp = _run(torch, ctx, pc, "fd", H, s, cell.kappa, cell.sizes, mode, impl="plain",
                        fp64_ratio=min(0.5, ratio))
    assert ctx.last_impl == "plain" and (stp == stg).all()
    assert _vec_err(xg, xp).max() <= TOL


@pytest.mark.parametrize("cell", [
    synth.Cell(B=24, sizes=(12, 12), U=12, n_sc=19, K=17, snr_db=15.0),
    synth.Cell(B=64, sizes=(32, 32), U=32, n_sc=7, K=17, snr_db=15.0),
], ids=["b24_u12", "b64_u32"])
@pytest.mark.parametrize("mode", ["wf", "zf"])
def test_pd_fp64_route_fused(torch, ctx, pc, cell, mode):
    """PD with U / B = 0.5 and B <= 64 (every subcarrier on the FP64 route)
    runs on the fused FP64 kernel, 17 symbols (two chunks): against the oracle
    and the plain FP64 kernels; precision FP64 (precode in FP64 as well) runs
    on the wide FP64 kernel."""
    H, s = synth.make_cell(cell, seed=13)
    xg, scg, stg = _run(torch, ctx, pc, "pd", H, s, cell.kappa, cell.sizes, mode)
    assert ctx.last_impl == "fused" and (stg == 2).all()
    xo, sco, sto = _oracle("pd", H, s, cell.kappa, cell.sizes, mode)
    _check(xg, scg, stg, xo, sco, sto)
    xp, scp, stp = _run(torch, ctx, pc, "pd", H, s, cell.kappa, cell.sizes, mode, impl="plain")
    assert (stp == stg).all() and _vec_err(xg, xp).max() <= TOL
    xw, scw, stw = _run(torch, ctx, pc, "pd", H, s, cell.kappa, cell.sizes, mode, precision="fp64")
    assert ctx.last_impl == "fused" and (stw == 2).all()
    _check(xw, scw, stw, xo, sco, sto, tol=1e-6)


def test_fd_fp64_route_fused_singular(torch, ctx, pc):
    """ZF on the fused FP64 route with a silent user in one cluster: that
    cluster's system is singular, flagged FAIL | FP64 with zero output; the
    others match the oracle."""
    cell = synth.Cell(B=64, sizes=(32, 32), U=16, n_sc=5, K=3)
    H, s = synth.make_cell(cell, seed=4)
    H[3, 32:, 5] = 0.0
    xg, scg, stg = _run(torch, ctx, pc, "fd", H, s, 0.0, cell.sizes, "zf")
    assert ctx.last_impl == "fused"
    assert stg[3, 1] == 3 and scg[3, 1] == 0.0 and not np.any(xg[:, 3, 32:])
    xo, sco, sto = _oracle("fd", H, s, 0.0, cell.sizes, "zf")
    assert sto[3, 1] == 1
    keep = [n for n in range(cell.n_sc) if n != 3]
    assert _vec_err(xg[:, keep], xo[:, keep]).max() <= TOL


@pytest.mark.parametrize("impl", ["fused", "plain"])
@pytest.mark.parametrize("defect", ["duplicate", "zero"])
def test_singular_zf_sets_status(torch, ctx, pc, impl, defect):
    """ZF with a duplicated (collinear) or silent user: the Gram matrix is
    singular, the instance is flagged and its output is zero."""
    cell = synth.Cell(B=32, sizes=(16, 16), U=4, n_sc=6, K=3)
    H, s = synth.make_cell(cell, seed=9)
    H[2, :, 3] = H[2, :, 1] if defect == "duplicate" else 0.0
    xg, scg, stg = _run(torch, ctx, pc, "pd", H, s, 0.0, cell.sizes, "zf", impl=impl, fp64_ratio=2.0)
    assert stg[2] & 1 == 1 and scg[2] == 0.0 and not np.any(xg[:, 2])
    xo, sco, sto = _oracle("pd", H, s, 0.0, cell.sizes, "zf")
    assert sto[2] == 1
    keep = [n for n in range(6) if n != 2]
    assert _vec_err(xg[:, keep], xo[:, keep]).max() <= TOL


def test_empty_inputs(torch, ctx, pc):
    H = torch.zeros((0, 64, 8), dtype=torch.complex64, device="cuda")
    s = torch.zeros((14, 0, 8), dtype=torch.complex64, device="cuda")
    x, b, st = ctx.pd(H, s, 0.5, [32, 32])
    assert x.shape == (14, 0, 64)
    cell = synth.config(1)
    Hn, sn = synth.make_cell(cell)
    Hd = _dev(torch, Hn)
    s0 = torch.zeros((0, cell.n_sc, cell.U), dtype=torch.complex64, device="cuda")
    x, b, st = ctx.pd(Hd, s0, cell.kappa, cell.sizes)
    torch.cuda.synchronize()
    _, bo, _ = oracle.pd(Hn, sn[:1], cell.kappa, cell.sizes)
    assert np.allclose(b.cpu().numpy(), bo, rtol=TOL, atol=0)


def test_deterministic(torch, ctx, pc):
    cell = synth.config(1)
    H, s = synth.make_cell(cell, seed=1)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    for arch in ("pd", "fd"):
        fn = ctx.pd if arch == "pd" else ctx.fd
        a = fn(Hd, sd, cell.kappa, cell.sizes)[0].clone()
        b = fn(Hd, sd, cell.kappa, cell.sizes)[0]
        assert torch.equal(a, b)


@pytest.mark.parametrize("impl,prec,tol", [("fused", "fp32", 1e-5), ("plain", "fp32", 1e-5),
                                            ("fused", "split_fp16", 1e-5)])
@pytest.mark.parametrize("arch", ["pd", "fd"])
def test_frame_symbols_match_one_shot(torch, ctx, pc, arch, impl, prec, tol):
    """Per-frame factors kept resident, symbols precoded one (and several) at a
    time, equal the oracle's one-shot frame."""
    cell = synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=16, K=14)
    H, s = synth.make_cell(cell, seed=2)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    f = ctx.frame(arch, Hd, cell.kappa, cell.sizes, "wf", pc.params(fp64_ratio=2.0, impl=impl, precision=prec))
    assert ctx.last_impl == impl
    xs = [f.symbols(sd[k:k + 1]) for k in range(4)] + [f.symbols(sd[4:])]
    sc, st = f.factors()
    torch.cuda.synchronize()
    xg = torch.cat(xs).cpu().numpy()
    xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, "wf")
    _check(xg, sc.cpu().numpy(), st.cpu().numpy(), xo, sco, sto, tol=tol)
    f.release()


def test_batch_matches_individual(torch, ctx, pc):
    cells = [synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=10, K=14),
             synth.Cell(B=128, sizes=(64, 64), U=16, n_sc=7, K=9, snr_db=3.0),
             synth.Cell(B=96, sizes=(40, 56), U=12, n_sc=5, K=20)]
    jobs, refs = [], []
    for i, c in enumerate(cells):
        H, s = synth.make_cell(c, seed=20 + i)
        arch = "pd" if i % 2 == 0 else "fd"
        jobs.append(dict(arch=arch, mode="wf", H=_dev(torch, H), s=_dev(torch, s), rho=c.kappa, sizes=c.sizes))
        refs.append(_oracle(arch, H, s, c.kappa, c.sizes, "wf"))
    outs = ctx.batch(jobs)
    torch.cuda.synchronize()
    for (x, sc, st), (xo, sco, sto), j in zip(outs, refs, jobs):
        scg = sc.cpu().numpy().reshape(sco.shape)
        stg = st.cpu().numpy().reshape(sto.shape)
        _check(x.cpu().numpy(), scg, stg, xo, sco, sto)


def _rescaled_err(arch, cell, xg, scg, xo, sco):
    """Error of the precoded vectors after replacing the GPU's beta / w_c by
    the oracle's: isolates the solve (z = A^-1 s) from the Lemma-1 factor."""
    xr = np.array(xg, dtype=np.complex128)
    if arch == "pd":
        xr *= (scg / sco)[None, :, None]  # x = H z / beta
    else:
        off = np.concatenate([[0], np.cumsum(cell.sizes)])
        for c in range(len(cell.sizes)):
            xr[:, :, off[c]:off[c + 1]] *= (sco[:, c] / scg[:, c])[None, :, None]  # x_c = w_c H_c u_c
    return _vec_err(xr, xo).max()


@pytest.mark.parametrize("arch,cell,ratio,envelope", [
    ("pd", synth.config(1), 2.0, True),
    ("fd", synth.Cell(B=64, sizes=(16, 16, 32), U=16, n_sc=24, K=14, snr_db=20.0), 0.5, True),   # FP64 route, B_c = U
    ("fd", synth.Cell(B=64, sizes=(16, 16, 32), U=16, n_sc=24, K=14, snr_db=20.0), 2.0, False),  # forced FP32, B_c = U
    ("pd", synth.Cell(B=24, sizes=(24,), U=16, n_sc=12, K=6, snr_db=20.0), 2.0, False),           # forced FP32, U/B = 0.67
])
@pytest.mark.parametrize("impl", ["auto", "plain"])
def test_refinement_fp64_residual(torch, ctx, pc, arch, cell, ratio, envelope, impl):
    """One refinement step with the residual in FP64 from the complex64
    channel, fused (factorization, then the refine-and-precode kernel) where
    the fused kernel takes the shape, else on the plain kernels.  It refines
    the solve, not the Lemma-1 factor: with the factor replaced by the
    oracle's the error never grows and meets the FP32 bound; inside the
    routing envelope (FP64 for U / B_eff >= 0.5) the full result meets it
    too."""
    H, s = synth.make_cell(cell, seed=5)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    fn = ctx.pd if arch == "pd" else ctx.fd
    # the unrefined result of the same kernels
    x0, sc0, _ = fn(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params(fp64_ratio=ratio, impl=impl))
    impl0 = ctx.last_impl
    x1, sc1, st1 = fn(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params(fp64_ratio=ratio, refine_steps=1, impl=impl))
    torch.cuda.synchronize()
    # fused unless forced plain (the FP64 route, ratio 0.5 here, runs its
    # fused FP64 solve)
    assert ctx.last_impl == ("plain" if impl == "plain" else "fused") and impl0 == ctx.last_impl
    xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, "wf")
    assert (st1.cpu().numpy().reshape(sto.shape) & 1 == sto).all()
    scg0, scg1 = (v.cpu().numpy().reshape(sco.shape).astype(np.float64) for v in (sc0, sc1))
    d0 = _rescaled_err(arch, cell, x0.cpu().numpy(), scg0, xo, sco)
    d1 = _rescaled_err(arch, cell, x1.cpu().numpy(), scg1, xo, sco)
    e0 = _vec_err(x0.cpu().numpy(), xo).max()
    e1 = _vec_err(x1.cpu().numpy(), xo).max()
    print("refinement (%s): solve err %.3e -> %.3e, full err %.3e -> %.3e" % (ctx.last_impl, d0, d1, e0, e1),
          flush=True)
    assert d1 <= max(d0, 2e-7) and d1 <= TOL
    if envelope:
        _check(x1.cpu().numpy(), scg1, st1.cpu().numpy().reshape(sto.shape), xo, sco, sto)


@pytest.mark.parametrize("nw", [1, 2, 4])
@pytest.mark.parametrize("name", ["cfg1", "ragged", "u32", "u20_kron", "many_clusters", "k70", "b256",
                                  "b300_ragged"])
def test_launch_shapes(torch, ctx, pc, monkeypatch, nw, name):
    """Every launch shape the autotuner may pick, forced: one system per wave
    in workgroups of 1, 2 or 4 waves, and (PD rows past one wave's registers)
    a subcarrier split over the 2 or 4 waves of a workgroup; plus the
    streamed rows."""
    _, cell, mode = next(c for c in CASES if c[0] == name)
    monkeypatch.setenv("PRECODE_FUSED_WAVES", str(nw))
    H, s = synth.make_cell(cell, seed=11)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    for stream in ("0", "1"):
        monkeypatch.setenv("PRECODE_FUSED_STREAM", stream)
        for arch in ("pd", "fd"):
            fn = ctx.pd if arch == "pd" else ctx.fd
            x, sc, st = fn(Hd, sd, cell.kappa, cell.sizes, mode, pc.params(fp64_ratio=2.0))
            torch.cuda.synchronize()
            if ctx.last_impl != "fused":
                continue
            print("%s %s nw=%d stream=%s used=%d" % (name, arch, nw, stream, ctx.last_waves), flush=True)
            xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, mode)
            _check(x.cpu().numpy(), sc.cpu().numpy().reshape(sco.shape), st.cpu().numpy().reshape(sto.shape),
                   xo, sco, sto)


def test_autotuned_shape_is_cached_and_deterministic(torch, ctx, pc, monkeypatch):
    monkeypatch.delenv("PRECODE_FUSED_WAVES", raising=False)
    monkeypatch.setenv("PRECODE_AUTOTUNE", "1")
    cell = synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=300, K=14)
    H, s = synth.make_cell(cell, seed=12)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    x1, _, _ = ctx.pd(Hd, sd, cell.kappa, cell.sizes)
    w1 = ctx.last_waves
    x2, _, _ = ctx.pd(Hd, sd, cell.kappa, cell.sizes)
    torch.cuda.synchronize()
    # 256 rows of 16 users are 8 tiles: one wave per subcarrier would stream
    # them twice, so only the split shapes (2 or 4 waves) are candidates
    assert w1 in (2, 4) and ctx.last_waves == w1
    assert torch.equal(x1, x2)


def test_tune_cache_file(torch, ctx, pc, monkeypatch, tmp_path):
    """A tuned launch shape is appended to the cache file, keyed by device and
    HIP runtime; after a reset the process takes the shape from the file
    without timing again (here an entry edited to another feasible shape)."""
    path = tmp_path / "tune.txt"
    monkeypatch.delenv("PRECODE_FUSED_WAVES", raising=False)
    monkeypatch.setenv("PRECODE_AUTOTUNE", "1")
    monkeypatch.setenv("PRECODE_TUNE_CACHE", str(path))
    pc.autotune_reset()
    try:
        cell = synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=301, K=14)
        H, s = synth.make_cell(cell, seed=14)
        Hd, sd = _dev(torch, H), _dev(torch, s)
        ctx.pd(Hd, sd, cell.kappa, cell.sizes)
        torch.cuda.synchronize()
        w1 = ctx.last_waves
        lines = [ln for ln in path.read_text().split("\n") if ln]
        assert len(lines) == 1
        dev, key, nw, stream = lines[0].split()
        assert int(nw) == w1 and stream == "0" and dev.startswith("gfx950") and "|hip" in dev
        other = 4 if w1 == 2 else 2
        path.write_text("%s %s %d 0\n" % (dev, key, other))
        pc.autotune_reset()
        x2, sc2, st2 = ctx.pd(Hd, sd, cell.kappa, cell.sizes)
        torch.cuda.synchronize()
        assert ctx.last_waves == other
        assert len([ln for ln in path.read_text().split("\n") if ln]) == 1  # read, not tuned again
        xo, sco, sto = _oracle("pd", H, s, cell.kappa, cell.sizes, "wf")
        _check(x2.cpu().numpy(), sc2.cpu().numpy(), st2.cpu().numpy(), xo, sco, sto)
    finally:
        pc.autotune_reset()


@pytest.mark.parametrize("u,expect", [(16, 2), (32, 1)])
def test_untuned_default_shape(torch, ctx, pc, monkeypatch, u, expect):
    """With tuning off (as under stream capture and in serving) PD takes the
    fewest waves per workgroup that keep the rows in register tiles at 16
    users, and the fewest that stream them at 32 users."""
    monkeypatch.delenv("PRECODE_FUSED_WAVES", raising=False)
    monkeypatch.setenv("PRECODE_AUTOTUNE", "0")
    cell = synth.Cell(B=256, sizes=(32,) * 8, U=u, n_sc=23, K=14)
    H, s = synth.make_cell(cell, seed=13)
    xg, scg, stg = _run(torch, ctx, pc, "pd", H, s, cell.kappa, cell.sizes, "wf")
    assert ctx.last_impl == "fused" and ctx.last_waves == expect
    xo, sco, sto = _oracle("pd", H, s, cell.kappa, cell.sizes, "wf")
    _check(xg, scg, stg, xo, sco, sto)


# Mixed batch spanning every launch class: tile widths 16 / 32, PD / FD,
# 1..8 channel tiles per wave, symbol slicing (K > 64), FD clusters smaller
# than U and U > 32 (wide FP64 kernel), FP64-route clusters (one-wave FP64
# kernel), an empty job.
MIX = [
    ("pd", synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=10, K=14)),
    ("fd", synth.Cell(B=128, sizes=(64, 64), U=16, n_sc=7, K=9, snr_db=3.0)),
    ("pd", synth.Cell(B=96, sizes=(40, 56), U=12, n_sc=5, K=20)),
    ("pd", synth.Cell(B=512, sizes=(64,) * 8, U=16, n_sc=6, K=14)),
    ("pd", synth.Cell(B=160, sizes=(80, 80), U=24, n_sc=4, K=70, channel="kron")),
    ("fd", synth.Cell(B=192, sizes=(48, 64, 80), U=20, n_sc=5, K=14, snr_db=15.0)),
    ("pd", synth.Cell(B=1024, sizes=(128,) * 8, U=16, n_sc=3, K=5)),
    ("fd", synth.Cell(B=40, sizes=(8, 32), U=12, n_sc=6, K=14)),
    ("pd", synth.Cell(B=128, sizes=(128,), U=40, n_sc=3, K=14)),
    ("fd", synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=0, K=14)),
    ("fd", synth.Cell(B=384, sizes=(32,) * 12, U=16, n_sc=9, K=14)),
]


def _mix_jobs(torch, cells, seed=40):
    jobs, host = [], []
    for i, (arch, c) in enumerate(cells):
        H, s = synth.make_cell(c, seed=seed + i)
        jobs.append(dict(arch=arch, mode="wf", H=_dev(torch, H), s=_dev(torch, s), rho=c.kappa, sizes=c.sizes))
        host.append((arch, c, H, s))
    return jobs, host


def test_batch_mixed_classes(torch, ctx, pc, monkeypatch):
    # the batch launches run one system per wave: compare with single calls
    # in that mode (one wave per workgroup never splits a subcarrier)
    monkeypatch.setenv("PRECODE_FUSED_WAVES", "1")
    jobs, host = _mix_jobs(torch, MIX)
    outs = ctx.batch(jobs)
    torch.cuda.synchronize()
    for (x, sc, st), (arch, c, H, s), j in zip(outs, host, jobs):
        print("batch job %s B=%d U=%d n_sc=%d K=%d" % (arch, c.B, c.U, c.n_sc, c.K), flush=True)
        if c.n_sc == 0:
            continue
        fn = ctx.pd if arch == "pd" else ctx.fd
        xi, sci, sti = fn(j["H"], j["s"], c.kappa, c.sizes, "wf")
        torch.cuda.synchronize()
        # same kernel body, same arithmetic as the single-problem call
        e = (x - xi).abs().max().item() / max(xi.abs().max().item(), 1e-30)
        assert e <= 1e-6, e
        assert torch.equal(st.flatten(), sti.flatten())
        xo, sco, sto = _oracle(arch, H, s, c.kappa, c.sizes, "wf")
        _check(x.cpu().numpy(), sc.cpu().numpy().reshape(sco.shape), st.cpu().numpy().reshape(sto.shape),
               xo, sco, sto)


@pytest.mark.parametrize("prec,tol", [("split_fp16", 1e-5), ("split_bf16", 1e-3)])
def test_batch_split_precision(torch, ctx, pc, prec, tol):
    # every job with symbols runs on a fused kernel: the register tiles at the
    # split precision, the FP64 kernels (FP64 route, U > 32, B_c < U) in FP64
    cells = [mc for mc in MIX if mc[1].n_sc > 0]
    jobs, host = _mix_jobs(torch, cells, seed=60)
    outs = ctx.batch(jobs, precision=prec)
    torch.cuda.synchronize()
    for (x, sc, st), (arch, c, H, s) in zip(outs, host):
        xo, sco, sto = _oracle(arch, H, s, c.kappa, c.sizes, "wf")
        stg = st.cpu().numpy().reshape(sto.shape)
        _check(x.cpu().numpy(), sc.cpu().numpy().reshape(sco.shape), stg, xo, sco, sto,
               tol=1e-5 if (stg & 2).all() else tol)
    # a job without symbols (factors only) needs the plain kernels
    arch, c = MIX[0]
    H, s = synth.make_cell(c, seed=61)
    j0 = dict(arch=arch, mode="wf", H=_dev(torch, H), s=_dev(torch, s[:0]), rho=c.kappa, sizes=c.sizes)
    with pytest.raises(pc.PrecodeError):
        ctx.batch([j0], precision=prec)


def test_batch_plan_graph_replays(torch, ctx, pc):
    """The recorded graph, replayed three times with eager work and cleared
    outputs in between, reproduces the eager batch every time."""
    jobs, host = _mix_jobs(torch, MIX, seed=80)
    ref = [tuple(t.clone() for t in o) for o in ctx.batch(jobs)]
    torch.cuda.synchronize()
    plan = ctx.batch_plan(jobs)
    assert plan.launches >= 1
    for rep in range(3):
        for x, sc, st in plan.outputs:
            x.zero_()
            sc.zero_()
            st.fill_(7)
        _ = (torch.ones(1 << 20, device="cuda") * 2).sum()  # unrelated eager work
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for (x, sc, st), (xr, scr, str_), (arch, c, H, s) in zip(plan.outputs, ref, host):
            if c.n_sc == 0:
                continue
            assert torch.equal(x, xr), "replay %d differs" % rep
            assert torch.equal(sc, scr) and torch.equal(st, str_)
    plan.destroy()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("split_fp16", 1e-5), ("split_bf16", 1e-3)])
@pytest.mark.parametrize("arch", ["pd", "fd"])
def test_full_size(torch, ctx, pc, arch, prec, tol):
    """B=256 as 8 x 32, U=16, 1200 subcarriers x 14 symbols in the launch
    configuration the benchmark times; every subcarrier and symbol against
    the oracle (a few tens of ms of host time)."""
    cell = synth.config(2)
    H, s = synth.make_cell(cell, seed=0)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    prm = pc.params(fp64_ratio=2.0, precision=prec)
    fn = ctx.pd if arch == "pd" else ctx.fd
    x, sc, st = fn(Hd, sd, cell.kappa, cell.sizes, "wf", prm)
    torch.cuda.synchronize()
    assert ctx.last_impl == "fused"
    xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, "wf")
    e = _check(x.cpu().numpy(), sc.cpu().numpy().reshape(sco.shape), st.cpu().numpy().reshape(sto.shape),
               xo, sco, sto, tol=tol)
    print("max rel err %.3e" % e, flush=True)


@pytest.fixture(scope="module")
def cell_u32(torch):
    """B=512 as 16 x 32, U=32, 3300 subcarriers x 14 symbols, channel with
    exponential antenna correlation r = 0.5; 16 sampled subcarriers for the
    oracle."""
    cell = synth.config(3)
    H, s = synth.make_cell(cell, seed=0)
    idx = np.sort(np.random.default_rng(3).choice(cell.n_sc, size=16, replace=False))
    return cell, H[idx].copy(), s[:, idx].copy(), _dev(torch, H), _dev(torch, s), idx


@pytest.mark.parametrize("impl,prec,ratio,tol", [
    ("fused", "fp32", 2.0, 1e-5), ("fused", "split_fp16", 2.0, 1e-5), ("fused", "split_bf16", 2.0, 1e-3),
    ("auto", "fp32", 0.5, 1e-5)], ids=["fused-fp32", "fused-split_fp16", "fused-split_bf16", "default_route"])
@pytest.mark.parametrize("arch", ["pd", "fd"])
def test_full_size_sampled_u32(torch, ctx, pc, cell_u32, arch, impl, prec, ratio, tol):
    """The 32-user workload at full size; the oracle checks the sampled
    subcarriers.  With the default ratio 0.5, FD's square local systems
    (B_c = U = 32) take the FP64 route."""
    cell, Hs, ss, Hd, sd, idx = cell_u32
    print("u32 full size: arch %s impl %s prec %s ratio %g" % (arch, impl, prec, ratio), flush=True)
    fn = ctx.pd if arch == "pd" else ctx.fd
    x, sc, st = fn(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params(fp64_ratio=ratio, precision=prec, impl=impl))
    torch.cuda.synchronize()
    if impl == "fused":
        assert ctx.last_impl == "fused"
    xo, sco, sto = _oracle(arch, Hs, ss, cell.kappa, cell.sizes, "wf")
    stg = st.cpu().numpy().reshape((cell.n_sc,) + sto.shape[1:])[idx]
    if arch == "fd":
        assert ((stg & 2) == (2 if ratio <= 1.0 else 0)).all()
    e = _check(x.cpu().numpy()[:, idx], sc.cpu().numpy().reshape((cell.n_sc,) + sco.shape[1:])[idx], stg,
               xo, sco, sto, tol=tol)
    print("max rel err %.3e" % e, flush=True)


@pytest.mark.parametrize("waves", [1, 2, 4])
@pytest.mark.parametrize("prec", ["split_fp16", "fp32"])
def test_silent_cluster_small_channel(torch, ctx, pc, monkeypatch, waves, prec):
    """One switched-off cluster (32 zero antenna rows) and a channel scaled by
    1e-5 (kappa by 1e-10: the same problem): an all-zero register tile must
    not fix the FP16 scaling exponent of the Gram, or the other tiles' low
    parts fall into FP16 subnormals."""
    monkeypatch.setenv("PRECODE_FUSED_WAVES", str(waves))
    cell = synth.config(2).with_(n_sc=64)
    H, s = synth.make_cell(cell, seed=4)
    H[:, :32, :] = 0
    H = (H * np.float32(1e-5)).astype(np.complex64)
    kappa = cell.kappa * 1e-10
    x, sc, st = _run(torch, ctx, pc, "pd", H, s, kappa, cell.sizes, "wf", precision=prec, impl="fused")
    xo, sco, sto = _oracle("pd", H, s, kappa, cell.sizes, "wf")
    e = _check(x, sc, st, xo, sco, sto, tol=1e-5)
    print("waves %d %s max rel err %.3e" % (waves, prec, e), flush=True)


@pytest.mark.parametrize("scale", [1e-3, 400.0, 3e4])
@pytest.mark.parametrize("prec", ["fp32", "split_fp16", "split_bf16"])
@pytest.mark.parametrize("arch,U", [("pd", 4), ("pd", 16), ("pd", 24), ("fd", 8), ("fd", 16)])
def test_channel_scale(torch, ctx, pc, arch, U, prec, scale):
    """x does not depend on the channel's scale (kappa scaled with G): the
    inversion must keep full precision whatever the magnitude of A."""
    cell = synth.Cell(B=128, sizes=(32,) * 4, U=U, n_sc=40, K=5, snr_db=10.0, qam=16)
    H, s = synth.make_cell(cell, seed=9)
    H = (H * np.float32(scale)).astype(np.complex64)
    kappa = cell.kappa * scale * scale
    tol = 1e-3 if prec == "split_bf16" else 1e-5
    x, sc, st = _run(torch, ctx, pc, arch, H, s, kappa, cell.sizes, "wf", precision=prec, impl="fused",
                     fp64_ratio=2.0)
    xo, sco, sto = _oracle(arch, H, s, kappa, cell.sizes, "wf")
    e = _check(x, sc.reshape(sco.shape), st.reshape(sto.shape), xo, sco, sto, tol=tol)
    print("%s U=%d %s scale %g max rel err %.3e" % (arch, U, prec, scale, e), flush=True)


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16", "fp32"])
@pytest.mark.parametrize("arch", ["pd", "fd"])
def test_refinement_fused_full_frame(torch, ctx, pc, arch, prec):
    """The fused refinement at 256 antennas (8 x 32), 16 users, 1200
    subcarriers x 14 symbols: runs fused, never increases the solve error,
    and the full result meets the FP32 bound at every precision."""
    cell = synth.config(2)
    H, s = synth.make_cell(cell, seed=6)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    fn = ctx.pd if arch == "pd" else ctx.fd
    x0, sc0, _ = fn(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params(fp64_ratio=2.0, precision=prec))
    x1, sc1, st1 = fn(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params(fp64_ratio=2.0, precision=prec, refine_steps=1))
    torch.cuda.synchronize()
    assert ctx.last_impl == "fused"
    xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, "wf")
    scg0, scg1 = (v.cpu().numpy().reshape(sco.shape).astype(np.float64) for v in (sc0, sc1))
    # the factor is not refined (the prepare pass may sum the clusters in
    # another launch shape's order)
    assert np.abs(scg1 - scg0).max() <= 1e-6 * np.abs(scg0).max()
    d0 = _rescaled_err(arch, cell, x0.cpu().numpy(), scg0, xo, sco)
    d1 = _rescaled_err(arch, cell, x1.cpu().numpy(), scg1, xo, sco)
    e1 = _check(x1.cpu().numpy(), scg1, st1.cpu().numpy().reshape(sto.shape), xo, sco, sto)
    print("%s %s refinement: solve err %.3e -> %.3e, full %.3e" % (arch, prec, d0, d1, e1), flush=True)
    assert d1 <= max(d0, 2e-7)


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16", "fp32"])
def test_refinement_fused_u32_sampled(torch, ctx, pc, cell_u32, prec):
    """The fused refinement at the 32-user workload (512 antennas as 16 x 32,
    3300 subcarriers, correlated channel), PD: the sampled subcarriers meet
    the FP32 bound against the oracle at every precision."""
    cell, Hs, ss, Hd, sd, idx = cell_u32
    x, sc, st = ctx.pd(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params(precision=prec, refine_steps=1))
    torch.cuda.synchronize()
    assert ctx.last_impl == "fused"
    xo, sco, sto = _oracle("pd", Hs, ss, cell.kappa, cell.sizes, "wf")
    e = _check(x.cpu().numpy()[:, idx], sc.cpu().numpy()[idx], st.cpu().numpy()[idx], xo, sco, sto)
    print("u32 %s refined max rel err %.3e" % (prec, e), flush=True)
