"""Pins for the oracle's comparison precoders, per-cluster FD variants and
uncoded-BER link, against facts the paper and the mathematics fix:

* centralized WF (B x B form of Theorem 1) equals the exact Gaussian-rational
  goldens of that theorem and the PD form (push-through identity of App. B)
* MRT is the large-regularizer limit of WF: centralized MRT of PD-WF with
  kappa -> infinity, per-cluster MRT of FD-WF with tau -> infinity
* per-cluster tau_c / rho_c^2 (eq. regularization, power footnote of
  Sec. III-C) equal default FD on a channel whose clusters are rescaled,
  because a cluster's normalized precoder depends on kappa_c / ||H_c||^2 only
* Gray QAM: unit energy, one bit between neighbours, exact demapping
* the MSE-optimal joint UE factor of the WF precoder is beta_WF (Sec. II-B)
* AWGN closed forms for QPSK and Gray 16-QAM on a single-antenna link
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import oracle.ber as ber
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exact_tiny.json")


def _fr(sv):
    return float(Fraction(sv))


def _cases():
    with open(GOLDEN) as f:
        return [c for c in json.load(f)["cases"] if not c["zf"]]


def _qfunc(v):
    return 0.5 * math.erfc(v / math.sqrt(2.0))


# ---------------------------------------------------------------------------
# centralized WF, B x B form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", _cases(), ids=lambda c: "B%dU%d" % (c["B"], c["U"]))
def test_central_exact(case):
    """beta^2 and beta x of the B x B form equal the exact Theorem-1 values."""
    H = np.array([[complex(*v) for v in row] for row in case["H"]])
    s = np.array([[complex(*v) for v in row] for row in case["s"]])
    x, beta, st = oracle.central(H, s[:, None, :], _fr(case["kappa"]))
    assert st[0] == 0
    b2 = _fr(case["pd_beta2"])
    assert abs(beta[0] ** 2 - b2) <= 1e-13 * b2
    bx = np.array([[complex(_fr(v[0]), _fr(v[1])) for v in xs] for xs in case["pd_beta_x"]])
    assert np.abs(x[:, 0, :] * beta[0] - bx).max() <= 1e-13 * np.abs(bx).max()


@pytest.mark.parametrize("B,U", [(64, 8), (100, 13), (16, 16), (8, 12)])
def test_central_equals_pd(B, U):
    cell = synth.Cell(B=B, sizes=(B,), U=U, n_sc=4, K=5, snr_db=10.0)
    H, s = synth.make_cell(cell, seed=21)
    xp, bp, _ = oracle.pd(H, s, cell.kappa, [B])
    xc, bc, st = oracle.central(H, s, cell.kappa)
    assert (st == 0).all()
    assert np.abs(xc - xp).max() <= 1e-10 * np.abs(xp).max()
    assert np.allclose(bc, bp, rtol=1e-11, atol=0)


def test_central_rejects_zf():
    H = np.ones((1, 4, 2), np.complex128)
    with pytest.raises(ValueError):
        oracle.central(H, np.ones((1, 1, 2)), 0.0)


# ---------------------------------------------------------------------------
# MRT
# ---------------------------------------------------------------------------
def test_mrt_is_wf_limit_central():
    """Centralized MRT = WF with kappa -> infinity.  The B x B form takes
    tr(Q^H Q) directly (Lemma 1's difference of two ~U/kappa terms would
    cancel at this kappa); the gap is O(||H||^2 / kappa)."""
    cell = synth.Cell(B=48, sizes=(48,), U=6, n_sc=3, K=4)
    H, s = synth.make_cell(cell, seed=2)
    xm, wm, sm = oracle.mrt(H, s)
    xc, bc, _ = oracle.central(H, s, 1e12)
    assert (sm == 0).all()
    assert np.abs(xm - xc).max() <= 1e-8 * np.abs(xm).max()


@pytest.mark.parametrize("power_c", [None, (0.5, 0.2, 0.3)])
def test_mrt_is_fd_limit_per_cluster(power_c):
    cell = synth.Cell(B=60, sizes=(12, 32, 16), U=8, n_sc=3, K=4)
    H, s = synth.make_cell(cell, seed=3)
    xm, wm, _ = oracle.mrt(H, s, cell.sizes, power_c=power_c)
    xf, wf, _ = oracle.fd(H, s, cell.kappa, cell.sizes, tau=1e12, power_c=power_c)
    assert np.abs(xm - xf).max() <= 1e-8 * np.abs(xm).max()


def test_mrt_zero_cluster_fails():
    cell = synth.Cell(B=32, sizes=(16, 16), U=4, n_sc=2, K=2)
    H, s = synth.make_cell(cell, seed=4)
    H[1, 16:] = 0
    x, w, st = oracle.mrt(H, s, cell.sizes)
    assert st[1, 1] == 1 and w[1, 1] == 0 and (x[:, 1, 16:] == 0).all()
    assert (st[0] == 0).all() and st[1, 0] == 0


# ---------------------------------------------------------------------------
# per-cluster tau_c and rho_c^2
# ---------------------------------------------------------------------------
def test_fd_uniform_variants_are_default():
    cell = synth.Cell(B=64, sizes=(16, 48), U=8, n_sc=3, K=4)
    H, s = synth.make_cell(cell, seed=5)
    x0, w0, _ = oracle.fd(H, s, cell.kappa, cell.sizes, tau=0.3)
    x1, w1, _ = oracle.fd(H, s, cell.kappa, cell.sizes, tau_c=(0.3, 0.3), power_c=(0.5, 0.5))
    assert np.array_equal(x0, x1) and np.array_equal(w0, w1)


@pytest.mark.parametrize("sizes", [(16, 48), (4, 12, 8, 20)])
def test_fd_per_cluster_by_rescaling(sizes):
    """Scaling H_c by a leaves x_c of FD unchanged if kappa_c scales by a^2
    (Q_c(a H_c, a^2 k) = Q_c(H_c, k) / a and the weight normalizes it), and the
    weight makes E||x_c||^2 = rho_c^2 exactly.  So FD with (tau_c, rho_c^2)
    equals default FD (tau, rho^2 / C) on the channel whose cluster c is scaled
    by a_c = sqrt(tau C rho_c^2 / (tau_c rho^2)), with x_c then scaled by
    sqrt(C rho_c^2 / rho^2).  Covers both Q_c forms (B_c < U and >= U)."""
    C, B, U = len(sizes), sum(sizes), 8
    cell = synth.Cell(B=B, sizes=sizes, U=U, n_sc=3, K=5, snr_db=5.0)
    H, s = synth.make_cell(cell, seed=6)
    rng = np.random.default_rng(7)
    tau_c = rng.uniform(0.05, 2.0, C)
    power, tau = 1.7, 0.125
    share = rng.uniform(0.5, 2.0, C)
    power_c = power * share / share.sum()
    x, w, st = oracle.fd(H, s, cell.kappa, sizes, tau=tau, power=power, tau_c=tau_c, power_c=power_c)
    assert (st == 0).all()
    off = np.concatenate([[0], np.cumsum(sizes)])
    Hs = H.astype(np.complex128)  # the rescaling in FP64, not complex64
    for c in range(C):
        Hs[:, off[c]:off[c + 1]] *= math.sqrt(tau * C * power_c[c] / (tau_c[c] * power))
    xr, _, _ = oracle.fd(Hs, s, cell.kappa, sizes, tau=tau, power=power)
    for c in range(C):
        xr[:, :, off[c]:off[c + 1]] *= math.sqrt(C * power_c[c] / power)
    assert np.abs(x - xr).max() <= 1e-11 * np.abs(x).max()


def test_fd_power_c_must_sum_to_power():
    cell = synth.Cell(B=32, sizes=(16, 16), U=4, n_sc=1, K=1)
    H, s = synth.make_cell(cell, seed=8)
    with pytest.raises(ValueError):
        oracle.fd(H, s, cell.kappa, cell.sizes, power_c=(0.5, 0.6))


# ---------------------------------------------------------------------------
# Gray QAM and the UE side
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [4, 16, 64, 256])
def test_qam_unit_energy_and_gray_neighbours(order):
    lab = np.arange(order)
    pts = ber.qam_map(lab, order)
    assert abs(np.mean(np.abs(pts) ** 2) - 1.0) <= 1e-14
    assert len(set(np.round(pts, 12))) == order
    d = ber.pam_spacing(order)
    nb = 0
    for i in range(order):
        for j in range(order):
            if abs(abs(pts[i] - pts[j]) - 2 * d) <= 1e-12:
                assert bin(i ^ j).count("1") == 1
                nb += 1
    m = int(math.isqrt(order))
    assert nb == 2 * 2 * m * (m - 1)  # ordered neighbour pairs on the grid


@pytest.mark.parametrize("order", [4, 16, 64])
def test_demap_regions(order):
    rng = np.random.default_rng(order)
    lab = rng.integers(0, order, 5000)
    d = ber.pam_spacing(order)
    pert = rng.uniform(-0.999 * d, 0.999 * d, (2, 5000))
    got = ber.demap(ber.qam_map(lab, order) + pert[0] + 1j * pert[1], order)
    assert np.array_equal(got, lab)
    corner = ber.qam_map(np.array([0]), order)
    assert ber.demap(corner * 100.0, order)[0] == 0


def test_bit_errors_counts_bits():
    assert ber.bit_errors(np.array([0, 5, 63]), np.array([0, 6, 0])) == 2 + 6


@pytest.mark.parametrize("sizes", [(32, 32), (8, 24, 32)])
def test_joint_beta_of_wf_is_beta_wf(sizes):
    """beta minimizing the Sec. II-B MSE for P = P_WF is beta_WF (Lemma 1);
    E = H_dl P comes from the receive model on U noise-free pilots, so a
    missing conjugate or transposed operand in receive() fails this too."""
    B, U = sum(sizes), 8
    cell = synth.Cell(B=B, sizes=sizes, U=U, n_sc=5, K=1, snr_db=3.0)
    H, _ = synth.make_cell(cell, seed=9)
    N0 = cell.kappa / U  # kappa = U N0 / rho^2, rho^2 = 1
    xp, beta, _ = oracle.pd(H, ber.pilots(cell.n_sc, U), cell.kappa, sizes)
    E = ber.effective_channel(H, xp)
    assert np.allclose(ber.joint_beta(E, N0), beta, rtol=1e-12, atol=0)
    # the same rule with the central B x B form
    xc, bc, _ = oracle.central(H, ber.pilots(cell.n_sc, U), cell.kappa)
    assert np.allclose(ber.joint_beta(ber.effective_channel(H, xc), N0), bc, rtol=1e-10, atol=0)


def test_zf_noiseless_recovers_symbols():
    cell = synth.Cell(B=64, sizes=(32, 32), U=8, n_sc=4, K=6)
    H, _ = synth.make_cell(cell, seed=10)
    lab = np.random.default_rng(11).integers(0, 64, (6, 4, 8))
    s = ber.qam_map(lab, 64)
    x, beta, _ = oracle.pd(H, s, 0.0, cell.sizes, zf=True)
    s_hat = ber.receive(H, x, None, 0.0, beta)
    assert np.abs(s_hat - s).max() <= 1e-12
    assert ber.bit_errors(lab, ber.demap(s_hat, 64)) == 0


def _single_antenna_ber(order, snr_db, n, zf):
    """B = U = 1, h = 1: x = s (ZF: beta = 1; WF: x = s, beta = 1/(1+kappa)),
    so s_hat = beta (s + n) with N0 = 1/SNR."""
    rng = np.random.default_rng(12)
    snr = 10.0 ** (snr_db / 10.0)
    N0 = 1.0 / snr
    H = np.ones((1, 1, 1), np.complex128)
    lab = rng.integers(0, order, (n, 1, 1))
    w = (rng.standard_normal((n, 1, 1)) + 1j * rng.standard_normal((n, 1, 1))) / math.sqrt(2)
    s = ber.qam_map(lab, order)
    x, beta, _ = oracle.pd(H, s, N0, [1], zf=zf)
    s_hat = ber.receive(H, x, w, N0, beta)
    return ber.bit_errors(lab, ber.demap(s_hat, order)) / (n * ber.bits_per_symbol(order)), N0


def test_awgn_qpsk_closed_form():
    """QPSK on AWGN, per-axis amplitude 1/sqrt(2), per-axis noise N0/2:
    P_b = Q(1/sqrt(N0)); the WF factor only scales, so decisions are ZF's."""
    n = 200000
    p, N0 = _single_antenna_ber(4, 7.0, n, zf=False)
    ref = _qfunc(1.0 / math.sqrt(N0))
    sigma = math.sqrt(ref * (1 - ref) / (2 * n))
    assert abs(p - ref) <= 5 * sigma, (p, ref)


def test_awgn_gray16_closed_form():
    """Gray 16-QAM with ZF on AWGN: per axis, levels -3d..3d with codes
    00, 01, 11, 10; MSB error (Q(d/s) + Q(3d/s)) / 2, LSB error
    Q(d/s) + (Q(3d/s) - Q(5d/s)) / 2, s^2 = N0 / 2, d^2 = 1/10."""
    n = 200000
    p, N0 = _single_antenna_ber(16, 12.0, n, zf=True)
    d, sg = math.sqrt(0.1), math.sqrt(N0 / 2)
    q1, q3, q5 = _qfunc(d / sg), _qfunc(3 * d / sg), _qfunc(5 * d / sg)
    ref = 0.5 * ((q1 + q3) / 2 + q1 + (q3 - q5) / 2)
    sigma = math.sqrt(ref * (1 - ref) / (4 * n))
    assert abs(p - ref) <= 6 * sigma, (p, ref)
