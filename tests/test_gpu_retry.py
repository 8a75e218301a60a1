"""GPU: the FP64 route for instances whose FP32 factorization fails.

Theorem 1 (Sec. II-B) needs A invertible, not well conditioned.  An FP32
factorization marks a pivot not above 2^-20 of its original diagonal entry
as failed; such an instance must be solved again on the FP64 route (status
PRECODE_ST_FP64) and match the FP64 oracle, whose pivot test is 2^-40.  Only
an instance the FP64 route cannot factor either is FAIL | FP64 with x = 0.

The nearly collinear user pair: user 1 equals user 0 except for one antenna
entry offset by 1/8.  With integer channel entries the FP32 Gram is exact
up to its last rounding, the exact Schur complement of user 1 is about 1/64
(relative 1e-8 of its diagonal entry, between the two thresholds), and the
FP32 elimination leaves only rounding noise of a few units in the last place
of the diagonal (relative 2e-7 < 2^-20): the FP32 pivot test fails for sure
and the FP64 one passes.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5
ST_OK, ST_FAIL, ST_FP64 = 0, 1, 2


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


def collinear_cell(B, U, n_sc, K, bad, amp, seed=0, singular=()):
    """Integer channel entries in [-amp, amp] (complex64-exact) with user 1 a
    near copy of user 0 on the subcarriers in `bad` and an exact copy on
    those in `singular`; QPSK symbols."""
    rng = np.random.default_rng(seed)
    H = (rng.integers(-amp, amp + 1, (n_sc, B, U)) + 1j * rng.integers(-amp, amp + 1, (n_sc, B, U)))
    for n in bad:
        H[n, :, 1] = H[n, :, 0]
        H[n, 0, 1] += 0.125
    for n in singular:
        H[n, :, 1] = H[n, :, 0]
    H = H.astype(np.complex64)
    s = ((rng.integers(0, 2, (K, n_sc, U)) * 2 - 1) + 1j * (rng.integers(0, 2, (K, n_sc, U)) * 2 - 1))
    s = (s / np.sqrt(2)).astype(np.complex64)
    return H, s


def _check(xg, scg, stg, xo, sco, sto, expect_status):
    assert (stg == expect_status).all(), (stg, expect_status)
    assert ((sto & ST_FAIL) == (expect_status & ST_FAIL)).all()
    e = _vec_err(xg, xo)
    assert np.isfinite(xg).all()
    assert e.max() <= TOL, "max rel err %.3e" % e.max()
    ok = (expect_status & ST_FAIL) == 0
    rel = np.abs(scg - sco) / np.where(sco > 0, sco, 1.0)
    assert rel[ok].max(initial=0) <= TOL, "scale rel err %.3e" % rel[ok].max()
    assert (scg[~ok] == 0).all()


# (B, sizes, U, amp): B = 32 keeps one register tile per wave; B = 256 takes
# the split workgroup (2 or 4 waves) or the streamed rows (1 wave).
PD_SHAPES = [(32, (32,), 4, 400), (256, (32,) * 8, 4, 120)]


@pytest.mark.parametrize("shape", PD_SHAPES, ids=["b32", "b256"])
@pytest.mark.parametrize("waves", [1, 2, 4])
@pytest.mark.parametrize("impl", ["fused", "plain"])
def test_pd_near_collinear_retried_in_fp64(torch, pc, ctx, monkeypatch, shape, waves, impl):
    B, sizes, U, amp = shape
    if impl == "plain" and waves != 1:
        pytest.skip("launch shape applies to the fused kernel")
    monkeypatch.setenv("PRECODE_FUSED_WAVES", str(waves))
    n_sc, K, bad = 8, 5, (3, 6)
    H, s = collinear_cell(B, U, n_sc, K, bad, amp)
    x, sc, st = ctx.pd(_dev(torch, H), _dev(torch, s), 0.0, sizes, "zf", pc.params(impl=impl))
    torch.cuda.synchronize()
    assert ctx.last_impl == impl
    xo, bo, so = oracle.pd(H, s, 0.0, sizes, zf=True)
    expect = np.zeros(n_sc, np.int32)
    expect[list(bad)] = ST_FP64
    _check(x.cpu().numpy(), sc.cpu().numpy(), st.cpu().numpy(), xo, bo, so, expect)


@pytest.mark.parametrize("impl", ["fused", "plain"])
def test_pd_exactly_singular_fails_on_fp64_route(torch, pc, ctx, impl):
    n_sc, K = 6, 3
    H, s = collinear_cell(64, 4, n_sc, K, bad=(1,), amp=300, singular=(4,))
    sizes = (32, 32)
    x, sc, st = ctx.pd(_dev(torch, H), _dev(torch, s), 0.0, sizes, "zf", pc.params(impl=impl))
    torch.cuda.synchronize()
    xo, bo, so = oracle.pd(H, s, 0.0, sizes, zf=True)
    assert so[4] == ST_FAIL and so[1] == ST_OK
    expect = np.zeros(n_sc, np.int32)
    expect[1] = ST_FP64
    expect[4] = ST_FP64 | ST_FAIL
    xg = x.cpu().numpy()
    assert (xg[:, 4] == 0).all()
    _check(xg, sc.cpu().numpy(), st.cpu().numpy(), xo, bo, so, expect)


@pytest.mark.parametrize("impl", ["fused", "plain"])
def test_fd_near_collinear_retried_in_fp64(torch, pc, ctx, impl):
    # FD-ZF, clusters of 32 antennas with 4 users (U / B_c < 0.5: the FP32
    # route); every cluster of the bad subcarriers holds the collinear pair
    n_sc, K, B, U = 6, 4, 64, 4
    sizes = (32, 32)
    rng = np.random.default_rng(5)
    H = (rng.integers(-400, 401, (n_sc, B, U)) + 1j * rng.integers(-400, 401, (n_sc, B, U)))
    for n in (2, 5):
        H[n, :, 1] = H[n, :, 0]
        H[n, 0, 1] += 0.125   # cluster 0
        H[n, 40, 1] += 0.125  # cluster 1
    H = H.astype(np.complex64)
    s = ((rng.integers(0, 2, (K, n_sc, U)) * 2 - 1) + 0j).astype(np.complex64)
    x, w, st = ctx.fd(_dev(torch, H), _dev(torch, s), 0.0, sizes, "zf", pc.params(impl=impl))
    torch.cuda.synchronize()
    xo, wo, so = oracle.fd(H, s, 0.0, sizes, zf=True)
    expect = np.zeros((n_sc, 2), np.int32)
    expect[[2, 5]] = ST_FP64
    _check(x.cpu().numpy(), w.cpu().numpy(), st.cpu().numpy(), xo, wo, so, expect)


@pytest.mark.parametrize("impl", ["fused", "plain"])
def test_frame_api_keeps_fp64_route_across_symbol_passes(torch, pc, ctx, impl):
    n_sc, K, B, U = 8, 6, 256, 4
    sizes = (32,) * 8
    H, s = collinear_cell(B, U, n_sc, K, bad=(0, 5), amp=120, seed=3)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    fr = ctx.frame("pd", Hd, 0.0, sizes, "zf", pc.params(impl=impl))
    xs = [fr.symbols(sd[k0:k0 + 2].contiguous()) for k0 in range(0, K, 2)]
    sc, st = fr.factors()
    torch.cuda.synchronize()
    x = torch.cat(xs, 0).cpu().numpy()
    fr.release()
    xo, bo, so = oracle.pd(H, s, 0.0, sizes, zf=True)
    expect = np.zeros(n_sc, np.int32)
    expect[[0, 5]] = ST_FP64
    _check(x, sc.cpu().numpy(), st.cpu().numpy(), xo, bo, so, expect)


def test_batch_retries_fused_jobs(torch, pc, ctx):
    H1, s1 = collinear_cell(32, 4, 5, 3, bad=(2,), amp=400, seed=7)
    H2, s2 = collinear_cell(256, 4, 4, 2, bad=(1,), amp=120, seed=8)
    jobs = [
        dict(arch="pd", mode="zf", H=_dev(torch, H1), s=_dev(torch, s1), sizes=(32,), rho=0.0),
        dict(arch="pd", mode="zf", H=_dev(torch, H2), s=_dev(torch, s2), sizes=(32,) * 8, rho=0.0),
    ]
    outs = ctx.batch(jobs)
    torch.cuda.synchronize()
    for (H, s, sizes, bad), (x, sc, st) in zip([(H1, s1, (32,), 2), (H2, s2, (32,) * 8, 1)], outs):
        xo, bo, so = oracle.pd(H, s, 0.0, sizes, zf=True)
        expect = np.zeros(H.shape[0], np.int32)
        expect[bad] = ST_FP64
        _check(x.cpu().numpy(), sc.cpu().numpy(), st.cpu().numpy(), xo, bo, so, expect)


@pytest.mark.parametrize("B,sizes", [(256, (32,) * 8), (64, (32, 32))], ids=["b256_split", "b64_one_wave"])
def test_refinement_retry(torch, ctx, pc, B, sizes):
    """One refinement step over a frame with nearly collinear (FP32 fails, FP64
    solves) and exactly singular subcarriers, 40 symbols (three chunks): the
    refinement kernel hands the FP64-route instances to the FP64 solve (at 256
    antennas the split workgroup's master wave), the others are refined; all
    against the oracle."""
    bad, singular = (3, 10), (7,)
    H, s = collinear_cell(B, 4, 12, 40, bad, 120 if B > 64 else 400, seed=31, singular=singular)
    x, sc, st = ctx.pd(_dev(torch, H), _dev(torch, s), 0.0, sizes, "zf",
                       pc.params(precision="split_fp16", refine_steps=1, fp64_ratio=2.0))
    torch.cuda.synchronize()
    assert ctx.last_impl == "fused"
    xo, sco, sto = oracle.pd(H, s, 0.0, sizes, zf=True)
    expect = np.zeros(12, dtype=np.int32)
    expect[list(bad)] = ST_FP64
    expect[list(singular)] = ST_FAIL | ST_FP64
    _check(x.cpu().numpy(), sc.cpu().numpy(), st.cpu().numpy(), xo, sco, sto, expect)
