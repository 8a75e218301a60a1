"""GPU: the wide FP64 kernel (one workgroup per local system of order <= 64,
in classes of order 32, 48 and 64) through the C ABI against the FP64
oracle: PD and FD with U in 33..64, FD
clusters smaller than U (the B_c x B_c form of Sec. III-C's case split),
mixed forms and routes in one cell, ragged row counts past one 64-row chunk,
several symbol chunks, ZF and its singular cases; and the heterogeneous
batch of the cell mix (B in 64..512, B_c in 16/32/64 or uneven, U in 4..64)
on the fused kernels only, cell by cell against the oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

# every step in FP64, the result rounded to complex64
TOL = 1e-6


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


def _oracle(arch, H, s, kappa, sizes, mode):
    if arch == "pd":
        return oracle.pd(H, s, kappa, sizes, zf=(mode == "zf"))
    return oracle.fd(H, s, kappa, sizes, zf=(mode == "zf"))


def _check(x, sc, st, xo, sco, sto, tol=TOL):
    x, sc, st = x.cpu().numpy(), sc.cpu().numpy().reshape(sco.shape), st.cpu().numpy().reshape(sto.shape)
    assert (st & 1 == sto).all()
    assert np.isfinite(x).all()
    e = _vec_err(x, xo).max()
    assert e <= tol, "max rel err %.3e" % e
    ok = sto == 0
    rel = np.abs(sc - sco) / np.where(sco > 0, sco, 1.0)
    assert rel[ok].max(initial=0) <= tol, "scale rel err %.3e" % rel[ok].max(initial=0)
    return st


# (name, arch, cell): every system of these cells is outside the register-tile
# and one-wave FP64 kernels
CELLS = [
    ("pd_u40", "pd", synth.Cell(B=128, sizes=(64, 64), U=40, n_sc=7, K=14, snr_db=10.0)),
    ("pd_u64_b200", "pd", synth.Cell(B=200, sizes=(72, 128), U=64, n_sc=5, K=17, snr_db=15.0)),  # 4 row chunks, ragged
    ("pd_u33_b64", "pd", synth.Cell(B=64, sizes=(64,), U=33, n_sc=6, K=5, snr_db=5.0)),          # U / B > 0.5
    ("pd_u48_kron", "pd", synth.Cell(B=96, sizes=(96,), U=48, n_sc=4, K=40, snr_db=20.0, channel="kron")),
    ("fd_bform_u40", "fd", synth.Cell(B=96, sizes=(16, 32, 48), U=40, n_sc=6, K=14, snr_db=10.0)),  # B_c < U and B_c >= U
    ("fd_bform_small", "fd", synth.Cell(B=44, sizes=(4, 12, 8, 20), U=24, n_sc=5, K=9, snr_db=5.0)),
    ("fd_bform_u64", "fd", synth.Cell(B=128, sizes=(1, 31, 33, 63), U=64, n_sc=3, K=17, snr_db=20.0)),
    ("fd_uform_u40", "fd", synth.Cell(B=210, sizes=(80, 130), U=40, n_sc=4, K=3, snr_db=10.0)),
    ("fd_bform_u56", "fd", synth.Cell(B=80, sizes=(40, 40), U=56, n_sc=5, K=14, snr_db=15.0)),  # order 40 < U
    ("fd_mixed_u12", "fd", synth.Cell(B=40, sizes=(8, 32), U=12, n_sc=8, K=14, snr_db=10.0)),  # one B_c < U, one FP32 route
    ("fd_u2_bc1", "fd", synth.Cell(B=7, sizes=(1, 6), U=2, n_sc=5, K=1, snr_db=0.0)),  # a 1-antenna cluster
]


@pytest.mark.parametrize("mode", ["wf", "zf"])
@pytest.mark.parametrize("name,arch,cell", CELLS, ids=[c[0] for c in CELLS])
def test_wide_parity(torch, ctx, pc, name, arch, cell, mode):
    H, s = synth.make_cell(cell, seed=71)
    print("wide", name, mode, flush=True)
    fn = ctx.pd if arch == "pd" else ctx.fd
    x, sc, st = fn(_dev(torch, H), _dev(torch, s), cell.kappa, cell.sizes, mode, pc.params(impl="fused"))
    torch.cuda.synchronize()
    assert ctx.last_impl == "fused"
    xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, mode)
    stg = _check(x, sc, st, xo, sco, sto)
    assert ((stg & 2) == 2).all()


def test_wide_deterministic_and_precisions(torch, ctx, pc):
    """Bitwise repeatable; precision FP64 and the split precisions take the
    same FP64 kernel for these systems (the same bits)."""
    cell = synth.Cell(B=128, sizes=(32, 96), U=40, n_sc=6, K=14, snr_db=10.0)
    H, s = synth.make_cell(cell, seed=72)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    ref = ctx.pd(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params())
    for prec in ("fp32", "fp64", "split_fp16", "split_bf16"):
        out = ctx.pd(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params(precision=prec))
        torch.cuda.synchronize()
        assert ctx.last_impl == "fused"
        for a, b in zip(ref, out):
            assert torch.equal(a, b), prec


def test_wide_precision_fp64_small_systems(torch, ctx, pc):
    """precision FP64 with U <= 32 (the one-wave FP64 kernel leaves it to the
    plain kernels' FP64 precode): the wide kernel, against the oracle."""
    cell = synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=9, K=14, snr_db=10.0)
    H, s = synth.make_cell(cell, seed=73)
    for arch in ("pd", "fd"):
        fn = ctx.pd if arch == "pd" else ctx.fd
        x, sc, st = fn(_dev(torch, H), _dev(torch, s), cell.kappa, cell.sizes, "wf", pc.params(precision="fp64"))
        torch.cuda.synchronize()
        assert ctx.last_impl == "fused"
        xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, "wf")
        _check(x, sc, st, xo, sco, sto)


@pytest.mark.parametrize("arch,cell,defect", [
    ("pd", synth.Cell(B=96, sizes=(96,), U=40, n_sc=5, K=3), "zero"),
    ("pd", synth.Cell(B=96, sizes=(96,), U=40, n_sc=5, K=3), "duplicate"),
    ("fd", synth.Cell(B=48, sizes=(16, 32), U=40, n_sc=5, K=3), "zero_row"),
])
def test_wide_singular_zf(torch, ctx, pc, arch, cell, defect):
    """ZF with a silent or duplicated user (U x U form) or a silent antenna
    (B_c x B_c form): that system is singular, flagged FAIL | FP64 with a zero
    output and scale; the others match the oracle."""
    H, s = synth.make_cell(cell, seed=74)
    if defect == "zero":
        H[2, :, 7] = 0.0
    elif defect == "duplicate":
        H[2, :, 9] = H[2, :, 3]
    else:
        H[2, 5, :] = 0.0  # cluster 0 (16 x 40) loses an antenna row: M_0 singular
    fn = ctx.pd if arch == "pd" else ctx.fd
    x, sc, st = fn(_dev(torch, H), _dev(torch, s), 0.0, cell.sizes, "zf", pc.params())
    torch.cuda.synchronize()
    x, sc, st = x.cpu().numpy(), sc.cpu().numpy(), st.cpu().numpy()
    xo, sco, sto = _oracle(arch, H, s, 0.0, cell.sizes, "zf")
    sc, st = sc.reshape(sco.shape), st.reshape(sto.shape)
    if arch == "pd":
        assert st[2] == 3 and sc[2] == 0.0 and not np.any(x[:, 2]) and sto[2] == 1
        keep = [n for n in range(cell.n_sc) if n != 2]
        assert _vec_err(x[:, keep], xo[:, keep]).max() <= 1e-5
    else:
        assert st[2, 0] == 3 and sc[2, 0] == 0.0 and not np.any(x[:, 2, :16]) and sto[2, 0] == 1
        assert (st & 1 == sto).all()
        good = sto == 0
        assert np.abs(sc - sco)[good].max() <= 1e-5 * sco[good].max()
        mask = np.ones(x.shape[1:], dtype=bool)
        mask[2, :16] = False
        err = np.abs(x - xo)[:, mask].max() / np.abs(xo).max()
        assert err <= 1e-5


def test_wide_larger_frame(torch, ctx, pc):
    """512 antennas, 64 users: PD over 8 row chunks per subcarrier, FD with
    16-antenna clusters (B_c x B_c form), every subcarrier against the oracle."""
    cell = synth.Cell(B=512, sizes=(16,) * 32, U=64, n_sc=12, K=14, snr_db=10.0)
    H, s = synth.make_cell(cell, seed=75)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    for arch in ("pd", "fd"):
        print("wide larger frame", arch, flush=True)
        fn = ctx.pd if arch == "pd" else ctx.fd
        x, sc, st = fn(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params())
        torch.cuda.synchronize()
        assert ctx.last_impl == "fused"
        xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, "wf")
        _check(x, sc, st, xo, sco, sto)


def _mix(uneven, n_sc=2):
    # the cell mix with its shapes and SNRs, few subcarriers each so that the
    # oracle checks every cell
    return [c.with_(n_sc=n_sc) for c in synth.mix(64, seed=0, uneven=uneven)]


@pytest.mark.parametrize("uneven", [False, True], ids=["even", "uneven"])
def test_batch_cell_mix_fused(torch, ctx, pc, uneven):
    """The 64-cell mix (B in 64..512, clusters of 16/32/64 antennas or
    uneven, U in 4..64, PD and FD alternating) as one batch plan: every job
    runs on the fused kernels (register tiles, one-wave FP64, wide FP64) and
    every cell matches the oracle."""
    cells = _mix(uneven)
    jobs, host = [], []
    for i, c in enumerate(cells):
        H, s = synth.make_cell(c, seed=300 + i)
        arch = "pd" if i % 2 == 0 else "fd"
        jobs.append(dict(arch=arch, mode="wf", H=_dev(torch, H), s=_dev(torch, s), rho=c.kappa, sizes=c.sizes))
        host.append((arch, c, H, s))
    plan = ctx.batch_plan(jobs)
    print("cell mix: %d jobs, %d fused, %d launches" % (len(jobs), plan.fused_jobs, plan.launches), flush=True)
    assert plan.fused_jobs == len(jobs)
    plan.launch()
    torch.cuda.synchronize()
    for (x, sc, st), (arch, c, H, s) in zip(plan.outputs, host):
        xo, sco, sto = _oracle(arch, H, s, c.kappa, c.sizes, "wf")
        # FP32 tiles on the FP32 route: 1e-5; the FP64 kernels: tighter
        _check(x, sc, st, xo, sco, sto, tol=1e-5)
    plan.destroy()


FRAME_CELLS = [
    ("pd_u40", "pd", synth.Cell(B=128, sizes=(64, 64), U=40, n_sc=7, K=17, snr_db=10.0)),
    ("fd_bform_u40", "fd", synth.Cell(B=96, sizes=(16, 32, 48), U=40, n_sc=6, K=17, snr_db=10.0)),
    ("fd_small_u24", "fd", synth.Cell(B=44, sizes=(4, 12, 8, 20), U=24, n_sc=5, K=17, snr_db=5.0)),
]


@pytest.mark.parametrize("name,arch,cell", FRAME_CELLS, ids=[c[0] for c in FRAME_CELLS])
def test_wide_frame_api(torch, ctx, pc, name, arch, cell):
    """The frame split on the wide FP64 kernel: prepare stores scale A^-1 in
    FP64, symbols are precoded from it in two passes (across a 16-symbol
    chunk boundary); the same result as the one-launch call to within FP64
    rounding, and the oracle's."""
    H, s = synth.make_cell(cell, seed=76)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    fr = ctx.frame(arch, Hd, cell.kappa, cell.sizes, "wf", pc.params())
    assert ctx.last_impl == "fused"
    xs = [fr.symbols(sd[0:5].contiguous()), fr.symbols(sd[5:17].contiguous())]
    w, st = fr.factors()
    torch.cuda.synchronize()
    x = torch.cat(xs, 0)
    fr.release()
    fn = ctx.pd if arch == "pd" else ctx.fd
    x1, w1, st1 = fn(Hd, sd, cell.kappa, cell.sizes, "wf", pc.params())
    torch.cuda.synchronize()
    assert torch.equal(st.flatten(), st1.flatten()) and torch.equal(w.flatten(), w1.flatten())
    assert _vec_err(x.cpu().numpy(), x1.cpu().numpy()).max() <= 1e-7
    xo, sco, sto = _oracle(arch, H, s, cell.kappa, cell.sizes, "wf")
    _check(x, w, st, xo, sco, sto)


@pytest.mark.parametrize("period", [5e-5, 0.0], ids=["released", "all_at_arrival"])
def test_wide_serving(torch, ctx, pc, period):
    """Serving jobs the register-tile kernels do not take (U = 64, clusters
    smaller than U, FP64-route cells) on the wide kernel: prepare and symbol
    passes, or one launch when every symbol is released at arrival; each job
    bitwise the same alone and in the mix, and the oracle's."""
    cells = [("pd", synth.Cell(B=128, sizes=(128,), U=64, n_sc=6, K=14, snr_db=10.0)),
             ("fd", synth.Cell(B=96, sizes=(16, 32, 48), U=40, n_sc=5, K=14, snr_db=10.0)),
             ("fd", synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=9, K=14, snr_db=10.0)),
             ("pd", synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=10, K=14))]
    jobs, host = [], []
    for i, (arch, c) in enumerate(cells):
        H, s = synth.make_cell(c, seed=77, cell_id=i)
        jobs.append(dict(arch=arch, mode="wf", H=_dev(torch, H), s=_dev(torch, s), rho=c.kappa, sizes=c.sizes))
        host.append((arch, c, H, s))
    outs, lat, stt = ctx.serve(jobs, [0.0, 0.0001, 0.0002, 0.0002], symbol_period_s=period, max_active=3,
                               n_streams=2)
    torch.cuda.synchronize()
    assert stt["jobs_done"] == len(jobs) and stt["symbols_done"] == 14 * len(jobs)
    for i, ((arch, c, H, s), (x, sc, st)) in enumerate(zip(host, outs)):
        print("wide serving job %d %s U=%d" % (i, arch, c.U), flush=True)
        (xa, sca, sta), = ctx.serve([jobs[i]], [0.0], symbol_period_s=period, max_active=1, n_streams=1)[0]
        torch.cuda.synchronize()
        assert torch.equal(x, xa) and torch.equal(sc, sca)
        xo, sco, sto = _oracle(arch, H, s, c.kappa, c.sizes, "wf")
        _check(x, sc, st, xo, sco, sto, tol=1e-5)
