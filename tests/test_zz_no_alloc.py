"""GPU: precode_pd_noalloc (no device allocation by the call) against
precode_pd on the same inputs, through the C ABI: the fused refinement
(its factors in the library's fixed array), the plain kernels (their
workspace in that array) and the fused kernels without workspace, two calls in a row with the second smaller
(the array keeps the first call's contents), and a call too large for the
array rejected before anything runs."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _vec_err(xg, xo):
    num = np.linalg.norm(xg - xo, axis=-1)
    den = np.linalg.norm(xo, axis=-1)
    return num / np.where(den > 0, den, 1.0)


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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [
    # (cell, params): fused refinement, plain kernels (forced, U > 32), fused
    # without workspace (register tiles; the wide FP64 kernel at U > 32)
    (synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=300, K=14, snr_db=10.0), dict(precision="split_fp16", refine_steps=1)),
    (synth.Cell(B=128, sizes=(64, 64), U=40, n_sc=50, K=9, snr_db=15.0), dict(impl="plain")),
    (synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=64, K=14, snr_db=10.0), dict()),
    (synth.Cell(B=128, sizes=(64, 64), U=40, n_sc=50, K=9, snr_db=15.0), dict()),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_matches_precode_pd(torch, pc, case):
    cell, prm = CASES[case]
    ctx = pc.Context(0)
    for n_sc in (cell.n_sc, cell.n_sc // 3):  # the second call smaller
        c = cell.with_(n_sc=n_sc)
        H, s = synth.make_cell(c, seed=40 + n_sc)
        Hd, sd = _dev(torch, H), _dev(torch, s)
        print("noalloc case %d n_sc %d %s" % (case, n_sc, prm), flush=True)
        x0, b0, st0 = ctx.pd(Hd, sd, c.kappa, c.sizes, "wf", pc.params(**prm))
        impl0 = ctx.last_impl
        x1, b1, st1 = ctx.pd_noalloc(Hd, sd, c.kappa, c.sizes, "wf", pc.params(**prm))
        torch.cuda.synchronize()
        assert ctx.last_impl == impl0
        assert torch.equal(st0, st1)
        # the same kernels; the fused launch shape may differ (precode_pd
        # times the shapes once, the fixed-workspace call takes the default)
        xa, xb = x0.cpu().numpy(), x1.cpu().numpy()
        assert _vec_err(xb, xa).max() <= TOL
        ba, bb = b0.cpu().numpy(), b1.cpu().numpy()
        assert (np.abs(bb - ba) <= TOL * np.abs(ba)).all()
        xo, bo, so = oracle.pd(H, s, c.kappa, c.sizes)
        assert ((st1.cpu().numpy() & 1) == so).all()
        assert _vec_err(xb, xo).max() <= TOL
        assert (np.abs(bb - bo) <= TOL * bo).all()
    ctx.close()


def test_noalloc_rejects_oversize(torch, pc):
    """The plain kernels' workspace of 3300 subcarriers with 40 users (the
    plain kernels forced: by default this shape runs on the wide FP64 kernel,
    which needs none) is larger than the fixed array: PRECODE_ENOMEM, nothing
    written."""
    ctx = pc.Context(0)
    c = synth.Cell(B=128, sizes=(64, 64), U=40, n_sc=3300, K=2, snr_db=10.0)
    H = torch.zeros((c.n_sc, c.B, c.U), dtype=torch.complex64, device="cuda")
    s = torch.zeros((c.K, c.n_sc, c.U), dtype=torch.complex64, device="cuda")
    x = torch.full((c.K, c.n_sc, c.B), 7.0, dtype=torch.complex64, device="cuda")
    with pytest.raises(pc.PrecodeError) as ei:
        ctx.pd_noalloc(H, s, c.kappa, c.sizes, "wf", pc.params(impl="plain"), x=x)
    assert ei.value.code == -3
    torch.cuda.synchronize()
    assert bool((x == 7.0).all())
    ctx.close()
