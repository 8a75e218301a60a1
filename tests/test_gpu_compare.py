"""GPU: the comparison precoders and the uncoded-BER link (Sec. III-D)
through the C ABI, against the FP64 oracle.

* precode_central (B x B form of Theorem 1) and precode_mrt against
  oracle.central / oracle.mrt, per (subcarrier, symbol) B-vector
* the UE kernels against oracle/ber.py on seeded inputs
* the whole link (precoder, UE factor, receive, decisions, bit errors) of
  PD, FD, centralized WF and MRT against the oracle's link
* PD and centralized WF give the same decisions on the same noise (Sec.
  III-D), and FD's loss against PD shrinks as the clusters grow

Decisions are integers decided by floating point: the GPU decides in FP32,
the oracle in FP64.  A symbol whose oracle estimate lies within DELTA of a
decision boundary may go either way; every other decision must agree, and
bit-error counts may differ by at most the bits of the ambiguous symbols.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.ber as ober
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
U32 = 2.0 ** -24
DELTA = 1e-4


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


def _cond_bxb(H, kappa):
    """cond(H H^H + kappa I_B) per subcarrier from the U x U Gram's spectrum."""
    n_sc, B, U = H.shape
    H = H.astype(np.complex128)
    ev = np.linalg.eigvalsh(np.conj(np.transpose(H, (0, 2, 1))) @ H)
    lo = ev[:, 0] + kappa if B <= U else np.full(n_sc, kappa)
    return (ev[:, -1] + kappa) / lo


# ---------------------------------------------------------------------------
# centralized WF, B x B form
# ---------------------------------------------------------------------------
CENTRAL = [
    ("b64u8", synth.Cell(B=64, sizes=(64,), U=8, n_sc=16, K=14, snr_db=10.0)),
    ("b100u13_ragged", synth.Cell(B=100, sizes=(100,), U=13, n_sc=9, K=5, snr_db=5.0)),
    ("b256u16", synth.Cell(B=256, sizes=(256,), U=16, n_sc=24, K=14, snr_db=10.0)),
    ("b40u24", synth.Cell(B=40, sizes=(40,), U=24, n_sc=8, K=3, snr_db=15.0)),
    ("b33u33", synth.Cell(B=33, sizes=(33,), U=33, n_sc=4, K=2, snr_db=20.0)),
    ("b16u4", synth.Cell(B=16, sizes=(16,), U=4, n_sc=5, K=1, snr_db=0.0)),
    ("b512u16", synth.Cell(B=512, sizes=(512,), U=16, n_sc=6, K=14, snr_db=10.0)),
    ("b256u16_kron", synth.Cell(B=256, sizes=(256,), U=16, n_sc=10, K=4, snr_db=20.0, channel="kron", r=0.5)),
]


def central_tol(H, kappa):
    """Forward error of an FP32 Cholesky solve: a modest multiple of
    cond(M) u per instance; never looser than the 1e-3 bar of the headline
    metric, never tighter than the FP32 paths' 1e-5."""
    B = H.shape[1]
    return np.clip(4.0 * math.sqrt(B) * _cond_bxb(H, kappa) * U32, TOL, 1e-3)


@pytest.mark.parametrize("name,cell", CENTRAL, ids=[c[0] for c in CENTRAL])
def test_central_parity(torch, ctx, pc, name, cell):
    H, s = synth.make_cell(cell, seed=31)
    print("central", name, flush=True)
    x, beta, st = ctx.central(_dev(torch, H), _dev(torch, s), cell.kappa)
    torch.cuda.synchronize()
    xo, bo, so = oracle.central(H, s, cell.kappa)
    assert (st.cpu().numpy() == so).all() and (so == 0).all()
    tol = central_tol(H, cell.kappa)
    e = _vec_err(x.cpu().numpy(), xo)
    print("max err %.3e, max err / tol %.3f" % (e.max(), (e / tol[None, :]).max()), flush=True)
    assert (e <= tol[None, :]).all()
    rb = np.abs(beta.cpu().numpy() - bo) / bo
    assert (rb <= tol).all()


def test_central_equals_pd_on_gpu(torch, ctx, pc):
    """Theorem 1 both ways on the GPU: the fused PD kernel and the B x B
    kernel give the same precoded vectors."""
    cell = synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=40, K=14, snr_db=10.0)
    H, s = synth.make_cell(cell, seed=32)
    Hd, sd = _dev(torch, H), _dev(torch, s)
    xp, bp, _ = ctx.pd(Hd, sd, cell.kappa, cell.sizes)
    xc, bc, _ = ctx.central(Hd, sd, cell.kappa)
    torch.cuda.synchronize()
    tol = central_tol(H, cell.kappa) + TOL
    assert (_vec_err(xc.cpu().numpy(), xp.cpu().numpy().astype(np.complex128)) <= tol[None, :]).all()


def test_central_rejects(torch, ctx, pc):
    H = torch.zeros((2, 64, 8), dtype=torch.complex64, device="cuda")
    s = torch.zeros((1, 2, 8), dtype=torch.complex64, device="cuda")
    with pytest.raises(pc.PrecodeError) as ei:
        ctx.central(H, s, 0.0)  # ZF has no B x B form
    assert ei.value.code == -2
    H = torch.zeros((1, 1024, 64), dtype=torch.complex64, device="cuda")
    s = torch.zeros((1, 1, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(pc.PrecodeError) as ei:
        ctx.central(H, s, 1.0)  # factor tiles and Q beyond the LDS
    assert ei.value.code == -2
    H = torch.zeros((1, 64, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(pc.PrecodeError):
        ctx.central(H, s, 1.0, pc.params(precision="split_fp16"))


def test_central_full_size_sampled(torch, ctx, pc):
    """The headline shape (256 antennas, 16 users, 1200 subcarriers) in one
    call; the oracle checks 60 subcarriers spread over the frame."""
    cell = synth.config(2)
    H, s = synth.make_cell(cell, seed=33)
    x, beta, st = ctx.central(_dev(torch, H), _dev(torch, s), cell.kappa)
    torch.cuda.synchronize()
    idx = np.linspace(0, cell.n_sc - 1, 60).astype(int)
    xo, bo, so = oracle.central(H[idx], s[:, idx], cell.kappa)
    tol = central_tol(H[idx], cell.kappa)
    assert (st.cpu().numpy() == 0).all()
    assert (_vec_err(x.cpu().numpy()[:, idx], xo) <= tol[None, :]).all()
    assert (np.abs(beta.cpu().numpy()[idx] - bo) / bo <= tol).all()


# ---------------------------------------------------------------------------
# MRT
# ---------------------------------------------------------------------------
MRT = [
    ("two", synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=12, K=14)),
    ("ragged", synth.Cell(B=100, sizes=(37, 63), U=13, n_sc=9, K=19)),
    ("eight", synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=20, K=14)),
    ("central", synth.Cell(B=256, sizes=(256,), U=16, n_sc=7, K=3)),
    ("u64", synth.Cell(B=128, sizes=(64, 64), U=64, n_sc=5, K=2)),
    ("b300u40_chunks", synth.Cell(B=300, sizes=(100, 200), U=40, n_sc=4, K=3)),  # 3 row chunks, ragged tail
    # the matrix-core kernel (U = 16 or 32, B <= 512), each launch shape:
    # 4 waves x 1 tile, ragged last tile, clusters across tiles, 2 symbol chunks
    ("mfma_b100u16", synth.Cell(B=100, sizes=(37, 63), U=16, n_sc=9, K=19)),
    ("mfma_b20u32_k1", synth.Cell(B=20, sizes=(20,), U=32, n_sc=3, K=1)),
    ("mfma_b256u32", synth.Cell(B=256, sizes=(64,) * 4, U=32, n_sc=6, K=17)),  # 8 waves x 1 tile
    ("mfma_b480u16", synth.Cell(B=480, sizes=(96,) * 5, U=16, n_sc=5, K=3)),  # 8 x 2, waves with 1 tile
    ("mfma_b512u32", synth.Cell(B=512, sizes=(32,) * 16, U=32, n_sc=5, K=14)),  # 8 x 2
    ("generic_b544u16", synth.Cell(B=544, sizes=(272, 272), U=16, n_sc=3, K=2)),  # past 512 rows
]


@pytest.mark.parametrize("name,cell", MRT, ids=[c[0] for c in MRT])
def test_mrt_parity(torch, ctx, pc, name, cell):
    H, s = synth.make_cell(cell, seed=34)
    print("mrt", name, flush=True)
    x, w, st = ctx.mrt(_dev(torch, H), _dev(torch, s), cell.sizes, pc.params(power=1.3))
    torch.cuda.synchronize()
    xo, wo, so = oracle.mrt(H, s, cell.sizes, power=1.3)
    assert (st.cpu().numpy() == so).all()
    assert _vec_err(x.cpu().numpy(), xo).max() <= TOL
    assert (np.abs(w.cpu().numpy() - wo) <= TOL * wo).all()


def test_mrt_zero_cluster(torch, ctx, pc):
    cell = synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=4, K=3)
    H, s = synth.make_cell(cell, seed=35)
    H[2, 32:] = 0
    x, w, st = ctx.mrt(_dev(torch, H), _dev(torch, s), cell.sizes)
    torch.cuda.synchronize()
    xo, wo, so = oracle.mrt(H, s, cell.sizes)
    assert (st.cpu().numpy() == so).all() and so[2, 1] == 1
    xg = x.cpu().numpy()
    assert (xg[:, 2, 32:] == 0).all()
    assert _vec_err(xg, xo).max() <= TOL


def test_mrt_zero_cluster_mfma(torch, ctx, pc):
    # a silent cluster on the matrix-core kernel: weight 0, status FAIL, x 0
    cell = synth.Cell(B=96, sizes=(40, 56), U=16, n_sc=4, K=5)
    H, s = synth.make_cell(cell, seed=36)
    H[1, :40] = 0
    x, w, st = ctx.mrt(_dev(torch, H), _dev(torch, s), cell.sizes)
    torch.cuda.synchronize()
    xo, wo, so = oracle.mrt(H, s, cell.sizes)
    assert (st.cpu().numpy() == so).all() and so[1, 0] == 1
    xg = x.cpu().numpy()
    assert (xg[:, 1, :40] == 0).all()
    assert _vec_err(xg, xo).max() <= TOL
    assert (np.abs(w.cpu().numpy() - wo) <= TOL * wo).all()


@pytest.mark.parametrize("U", [16, 13])  # the matrix-core kernel and the general one
def test_mrt_no_symbols(torch, ctx, pc, U):
    # K = 0: weights and status only
    cell = synth.Cell(B=96, sizes=(40, 56), U=U, n_sc=5, K=1)
    H, s = synth.make_cell(cell, seed=39)
    s0 = np.zeros((0, cell.n_sc, U), np.complex64)
    x, w, st = ctx.mrt(_dev(torch, H), _dev(torch, s0), cell.sizes)
    torch.cuda.synchronize()
    assert tuple(x.shape) == (0, cell.n_sc, cell.B)
    _, wo, so = oracle.mrt(H, s, cell.sizes)
    assert (st.cpu().numpy() == so).all()
    assert (np.abs(w.cpu().numpy() - wo) <= TOL * wo).all()


def test_mrt_misaligned_channel(torch, ctx, pc):
    # a channel that is not 16-byte aligned takes the general kernel
    cell = synth.Cell(B=64, sizes=(32, 32), U=16, n_sc=3, K=4)
    H, s = synth.make_cell(cell, seed=37)
    flat = torch.empty(H.size + 1, dtype=torch.complex64, device="cuda")
    Hd = flat[1:].view(H.shape)
    Hd.copy_(_dev(torch, H))
    assert Hd.data_ptr() % 16 == 8
    x, w, st = ctx.mrt(Hd, _dev(torch, s), cell.sizes)
    torch.cuda.synchronize()
    xo, wo, so = oracle.mrt(H, s, cell.sizes)
    assert (st.cpu().numpy() == so).all()
    assert _vec_err(x.cpu().numpy(), xo).max() <= TOL


def test_mrt_full_frame(torch, ctx, pc):
    # every subcarrier of the 256-antenna / 16-user frame (8 clusters of 32)
    cell = synth.config(2)
    H, s = synth.make_cell(cell, seed=38)
    x, w, st = ctx.mrt(_dev(torch, H), _dev(torch, s), cell.sizes)
    torch.cuda.synchronize()
    xo, wo, so = oracle.mrt(H, s, cell.sizes)
    assert (st.cpu().numpy() == so).all()
    assert _vec_err(x.cpu().numpy(), xo).max() <= TOL
    assert (np.abs(w.cpu().numpy() - wo) <= TOL * wo).all()


# ---------------------------------------------------------------------------
# the UE kernels on seeded inputs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [4, 16, 64, 256])
def test_qam_map(torch, pc, order):
    lab = np.arange(order * 3, dtype=np.int32) % order
    s = pc.qam_map(_dev(torch, lab), order)
    torch.cuda.synchronize()
    assert np.abs(s.cpu().numpy() - ober.qam_map(lab, order)).max() <= 1e-6


UE_SHAPES = [
    (7, 100, 13, 70),  # K beyond one launch's 64 symbols
    (5, 256, 16, 14),  # two row chunks, 16 row groups of 4 x 4 blocks
    (3, 300, 64, 64),  # 256 blocks, one row group, rows in chunks of 32
    (4, 1, 1, 1),
    (3, 37, 5, 3),
]


@pytest.mark.parametrize("n_sc,B,U,K", UE_SHAPES)
def test_ue_receive(torch, pc, n_sc, B, U, K):
    rng = np.random.default_rng(36)
    H = synth.cn_noise((n_sc, B, U), rng)
    x = synth.cn_noise((K, n_sc, B), rng)
    w = synth.cn_noise((K, n_sc, U), rng)
    scale = rng.uniform(0.5, 2.0, n_sc).astype(np.float32)
    y = pc.ue_receive(_dev(torch, H), _dev(torch, x), _dev(torch, w), 0.3, _dev(torch, scale))
    y0 = pc.ue_receive(_dev(torch, H), _dev(torch, x))
    torch.cuda.synchronize()
    yo = ober.receive(H, x, w, 0.3, scale)
    assert _vec_err(y.cpu().numpy(), yo).max() <= TOL
    assert _vec_err(y0.cpu().numpy(), ober.receive(H, x, None, 0.0, None)).max() <= TOL


def test_ue_gain(torch, pc):
    rng = np.random.default_rng(37)
    n_sc, U = 300, 16
    E = np.eye(U)[None] * 0.9 + 0.05 * synth.cn_noise((n_sc, U, U), rng)
    yp = np.ascontiguousarray(np.transpose(E, (2, 0, 1))).astype(np.complex64)  # [v][n][u] = E[n][u][v]
    b = pc.ue_gain(_dev(torch, yp), 0.05, 1.0)
    torch.cuda.synchronize()
    bo = ober.joint_beta(E.astype(np.complex64).astype(np.complex128), 0.05)
    assert (np.abs(b.cpu().numpy() - bo) <= TOL * np.abs(bo)).all()


def _boundary_distance(s_hat, order):
    """Distance of each estimate's nearest axis coordinate to a decision
    boundary (boundaries at (2 i + 2 - m) d, i = 0..m-2)."""
    m = int(round(math.sqrt(order)))
    d = ober.pam_spacing(order)
    bnd = (2 * np.arange(m - 1) + 2 - m) * d
    dr = np.min(np.abs(np.real(s_hat)[..., None] - bnd), axis=-1)
    di = np.min(np.abs(np.imag(s_hat)[..., None] - bnd), axis=-1)
    return np.minimum(dr, di)


@pytest.mark.parametrize("order", [4, 16, 64])
def test_qam_errors(torch, pc, order):
    rng = np.random.default_rng(38 + order)
    lab = synth.labels((5, 40, 16), order, rng)
    # noise of 0.6 level half-spacings: a few percent of the decisions wrong
    noise = 0.6 * ober.pam_spacing(order) * synth.cn_noise(lab.shape, rng)
    s_hat = (ober.qam_map(lab, order) + noise).astype(np.complex64)
    out = torch.empty(lab.shape, dtype=torch.int32, device="cuda")
    cnt, _ = pc.qam_errors(_dev(torch, s_hat), _dev(torch, lab), order, labels_out=out)
    torch.cuda.synchronize()
    s64 = s_hat.astype(np.complex128)
    lo = ober.demap(s64, order)
    amb = _boundary_distance(s64, order) <= DELTA
    g = out.cpu().numpy()
    assert (g[~amb] == lo[~amb]).all()
    ref = ober.bit_errors(lab, lo)
    assert abs(int(cnt.item()) - ref) <= int(amb.sum()) * ober.bits_per_symbol(order)
    assert ref > 0


# ---------------------------------------------------------------------------
# the whole link
# ---------------------------------------------------------------------------
def oracle_link(scheme, H, lab, w, snr_db, order, sizes, tau=0.125, joint=False):
    n_sc, B, U = H.shape
    N0 = 10.0 ** (-snr_db / 10.0)
    kappa = U * N0

    def prec(sym):
        if scheme == "pd":
            return oracle.pd(H, sym, kappa, sizes)[:2]
        if scheme == "fd":
            return oracle.fd(H, sym, kappa, sizes, tau=tau)[0], None
        if scheme == "central":
            return oracle.central(H, sym, kappa)[:2]
        return oracle.mrt(H, sym, sizes)[0], None

    x, scale = prec(ober.qam_map(lab, order))
    if scale is None or joint:
        xp, _ = prec(ober.pilots(n_sc, U))
        scale = ober.joint_beta(ober.effective_channel(H, xp), N0)
    s_hat = ober.receive(H, x, w, N0, scale)
    return s_hat, ober.demap(s_hat, order), scale


LINK = synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=32, K=14, snr_db=10.0, qam=16)


@pytest.mark.parametrize("joint", [False, True])
@pytest.mark.parametrize("scheme", ["pd", "fd", "central", "mrt"])
def test_link_parity(torch, ctx, pc, scheme, joint):
    from paper_1804_10987_amd import ber

    H, lab, w = synth.link_frame(LINK, seed=40)
    print("link", scheme, joint, flush=True)
    out = torch.empty(lab.shape, dtype=torch.int32, device="cuda")
    cnt, s_hat, scale = ber.frame_errors(ctx, scheme, _dev(torch, H), _dev(torch, lab), _dev(torch, w),
                                         LINK.snr_db, LINK.qam, LINK.sizes, joint=joint, labels_out=out)
    torch.cuda.synchronize()
    so, lo, sco = oracle_link(scheme, H, lab, w, LINK.snr_db, LINK.qam, LINK.sizes, joint=joint)
    tol = central_tol(H, LINK.kappa) if scheme == "central" else np.full(LINK.n_sc, TOL)
    assert (np.abs(scale.cpu().numpy() - sco) <= 2 * tol * sco).all()
    assert (_vec_err(s_hat.cpu().numpy(), so) <= 2 * tol[None, :]).all()
    amb = _boundary_distance(so, LINK.qam) <= DELTA
    g = out.cpu().numpy()
    assert (g[~amb] == lo[~amb]).all()
    ref = ober.bit_errors(lab, lo)
    assert abs(int(cnt.item()) - ref) <= int(amb.sum()) * 4
    assert ref > 0


def test_pd_equals_central_ber(torch, ctx, pc):
    """Sec. III-D: PD-WF achieves the BER of centralized WF.  Same channel,
    symbols and noise: the decisions agree except where both estimates sit
    on a decision boundary."""
    from paper_1804_10987_amd import ber

    cell = synth.Cell(B=256, sizes=(32,) * 8, U=16, n_sc=300, K=14, snr_db=3.0, qam=64)
    H, lab, w = synth.device_link_frame(cell, "cuda", seed=41, frame=0)
    outs = {}
    for scheme in ("pd", "central"):
        o = torch.empty(lab.shape, dtype=torch.int32, device="cuda")
        cnt, s_hat, _ = ber.frame_errors(ctx, scheme, H, lab, w, cell.snr_db, cell.qam, cell.sizes, labels_out=o)
        outs[scheme] = (int(cnt.item()), o.cpu().numpy(), s_hat.cpu().numpy())
    (cp, lp, sp), (cc, lc, sc) = outs["pd"], outs["central"]
    diff = lp != lc
    near = _boundary_distance(sc.astype(np.complex128), cell.qam) <= 1e-3
    assert not (diff & ~near).any()
    assert abs(cp - cc) <= 6 * int(diff.sum())
    assert cp > 1000  # a BER regime where the comparison means something


def test_fd_loss_shrinks_with_cluster_size(torch, ctx, pc):
    """Sec. III-D: FD-WF loses BER against PD-WF (= centralized WF) when the
    clusters are small; with the same 256 antennas, 2 clusters of 128 lose
    less than 8 clusters of 32, and PD is best."""
    from paper_1804_10987_amd import ber

    res = {}
    for name, sizes, scheme in [("pd", (32,) * 8, "pd"), ("fd128", (128, 128), "fd"), ("fd32", (32,) * 8, "fd")]:
        cell = synth.Cell(B=256, sizes=sizes, U=16, n_sc=300, K=14, snr_db=12.0, qam=64)
        res[name] = ber.ber(ctx, scheme, cell, cell.snr_db, frames=2, seed=42)
    print(res, flush=True)
    assert res["pd"] < res["fd128"] < res["fd32"]
