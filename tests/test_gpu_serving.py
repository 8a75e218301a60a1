"""GPU: continuous-batching serving loop (precode_serve).

Jobs from a heterogeneous cell mix arrive over time, are admitted against an
HBM budget and overlap on the device; every job's result must be bitwise the
same as when it is served alone, and match the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t

    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def ctx():
    import paper_1804_10987_amd as pc

    return pc.Context(0)


def _cells():
    return [
        ("pd", synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=24, K=14, snr_db=10.0)),
        ("fd", synth.Cell(B=128, sizes=(32,) * 4, U=12, n_sc=17, K=14, snr_db=5.0)),
        ("pd", synth.Cell(B=96, sizes=(40, 56), U=20, n_sc=11, K=14, snr_db=15.0)),
        ("fd", synth.Cell(B=48, sizes=(4, 20, 24), U=6, n_sc=9, K=14, snr_db=0.0)),  # B_c < U: plain kernels
        ("pd", synth.Cell(B=64, sizes=(64,), U=40, n_sc=5, K=14, snr_db=20.0)),      # U > 32: plain kernels
        ("fd", synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=30, K=14, snr_db=10.0)),
    ]


def _jobs(torch, cells, seed=0):
    jobs, host = [], []
    for i, (arch, c) in enumerate(cells):
        H, s = synth.make_cell(c, seed=seed, cell_id=i)
        jobs.append(dict(arch=arch, mode="wf", H=torch.from_numpy(H).cuda(), s=torch.from_numpy(s).cuda(),
                         rho=c.kappa, sizes=c.sizes))
        host.append((arch, c, H, s))
    return jobs, host


def _check_oracle(i, arch, c, H, s, x, sc, stt):
    if arch == "pd":
        xo, sco, sto = oracle.pd(H, s, c.kappa, c.sizes)
    else:
        xo, sco, sto = oracle.fd(H, s, c.kappa, c.sizes)
    xg = x.cpu().numpy().reshape(xo.shape)
    e = np.linalg.norm(xg - xo, axis=-1) / np.maximum(np.linalg.norm(xo, axis=-1), 1e-30)
    print("job %d %s B=%d U=%d max rel err %.2e" % (i, arch, c.B, c.U, e.max()), flush=True)
    assert e.max() <= 1e-5
    sco, sto = np.asarray(sco).ravel(), np.asarray(sto).ravel()
    assert ((stt.cpu().numpy().ravel() & 1) == sto).all()
    scg = sc.cpu().numpy().ravel()
    assert (np.abs(scg - sco) <= 1e-5 * np.abs(sco)).all()


def test_serving_mix_equals_alone_and_oracle(torch, ctx):
    cells = _cells()
    jobs, host = _jobs(torch, cells)
    arrivals = [0.0, 0.0002, 0.0004, 0.0005, 0.0009, 0.0010]
    print("serving mix of %d jobs" % len(jobs), flush=True)
    outs, lat, st = ctx.serve(jobs, arrivals, symbol_period_s=5e-5, max_active=4, n_streams=3)
    torch.cuda.synchronize()
    assert st["jobs_done"] == len(jobs)
    assert st["symbols_done"] == 14 * len(jobs)
    assert all((l >= 0).all() for l in lat)
    for i, ((arch, c, H, s), (x, sc, stt)) in enumerate(zip(host, outs)):
        # alone: the same job through the same loop with nothing else in flight
        (xa, sca, sta), = ctx.serve([jobs[i]], [0.0], symbol_period_s=5e-5, max_active=1, n_streams=1)[0]
        torch.cuda.synchronize()
        assert torch.equal(x, xa), "job %d differs alone vs in the mix" % i
        assert torch.equal(sc, sca)
        _check_oracle(i, arch, c, H, s, x, sc, stt)


def test_serving_zero_period_one_launch(torch, ctx):
    """Every symbol released at arrival: the jobs on the fused kernels take
    one launch from Gram to precode.  Each result is bitwise the same alone
    and in the mix, and matches the oracle."""
    cells = _cells()
    jobs, host = _jobs(torch, cells, seed=5)
    arrivals = [0.0, 0.0001, 0.0001, 0.0003, 0.0004, 0.0004]
    print("serving mix of %d jobs, zero symbol period" % len(jobs), flush=True)
    outs, lat, st = ctx.serve(jobs, arrivals, symbol_period_s=0.0, max_active=4, n_streams=3)
    torch.cuda.synchronize()
    assert st["jobs_done"] == len(jobs)
    assert st["symbols_done"] == 14 * len(jobs)
    assert all((l >= 0).all() for l in lat)
    for i, ((arch, c, H, s), (x, sc, stt)) in enumerate(zip(host, outs)):
        (xa, sca, sta), = ctx.serve([jobs[i]], [0.0], symbol_period_s=0.0, max_active=1, n_streams=1)[0]
        torch.cuda.synchronize()
        assert torch.equal(x, xa), "job %d differs alone vs in the mix" % i
        assert torch.equal(sc, sca)
        _check_oracle(i, arch, c, H, s, x, sc, stt)


def test_serving_admission_by_budget(torch, ctx):
    """A slab that fits about one job at a time still serves every job, in
    arrival order, with admission waits."""
    cells = [("pd", synth.Cell(B=64, sizes=(32, 32), U=16, n_sc=64, K=14)) for _ in range(5)]
    jobs, host = _jobs(torch, cells, seed=3)
    per_job = 64 * 16 * 16 * 8 + 64 * 8 + 1024
    outs, lat, st = ctx.serve(jobs, [0.0] * 5, symbol_period_s=2e-5, max_active=8, n_streams=2,
                              slab_bytes=int(per_job * 1.5))
    torch.cuda.synchronize()
    assert st["jobs_done"] == 5 and st["peak_active"] == 1
    assert st["wait_p99_s"] > 0
    ref = ctx.serve([jobs[0]], [0.0], symbol_period_s=2e-5, max_active=1, n_streams=1)[0][0][0]
    assert torch.equal(outs[0][0], ref)


def test_serving_rejects_oversize_job(torch, ctx):
    import paper_1804_10987_amd as pc

    jobs, _ = _jobs(torch, [("pd", synth.Cell(B=64, sizes=(64,), U=16, n_sc=64, K=14))])
    with pytest.raises(pc.PrecodeError):
        ctx.serve(jobs, [0.0], slab_bytes=1024)


def test_serving_zero_symbol_job_retires_after_its_factors(torch, ctx):
    """A job with K = 0 (factors only) retires, and hands its slab region
    back, only after its factors and their copies are done: jobs admitted
    after it into the same region (one-job slab) keep their results, and
    the K = 0 job's beta and status match the oracle."""
    c0 = synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=48, K=14, snr_db=10.0)
    H, s = synth.make_cell(c0, seed=21)
    H2, s2 = synth.make_cell(c0, seed=22)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    jobs = [dict(arch="pd", mode="wf", H=dev(H), s=dev(s[:0]), rho=c0.kappa, sizes=c0.sizes),
            dict(arch="pd", mode="wf", H=dev(H2), s=dev(s2), rho=c0.kappa, sizes=c0.sizes)]
    per_job = 48 * 8 * 8 * 8 + 48 * 8 + 1024
    outs, lat, st = ctx.serve(jobs, [0.0, 0.0], symbol_period_s=0.0, max_active=4, n_streams=2,
                              slab_bytes=int(per_job * 1.2))
    torch.cuda.synchronize()
    assert st["jobs_done"] == 2
    _, bo, so = oracle.pd(H, s[:1], c0.kappa, c0.sizes)
    assert (outs[0][2].cpu().numpy() == so).all()
    assert np.abs(outs[0][1].cpu().numpy() - bo).max() <= 1e-5 * bo.max()
    _check_oracle(1, "pd", c0, H2, s2, *outs[1])
