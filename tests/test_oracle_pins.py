"""Pins for the FP64 oracle: checks against what the paper and the mathematics
fix, never against the oracle's own formulas.

* exact Gaussian-rational brute force (Theorem 1 B x B form, Sec. III-C forms)
* PD == centralized WF (Sec. III-B identity, push-through form of App. B)
* invariance of PD to the cluster split, ZF zero interference, power budget
* FD: both Q_c forms (Sec. III-C case split), FD(C=1, tau=1) == centralized
* closed forms (single user, orthogonal columns), metamorphic invariances
* MSE optimality of the WF precoder (problem in Sec. II-B, App. A)
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exact_tiny.json")


def _rng(seed):
    return np.random.default_rng(seed)


def _cn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def _precoder_matrix(fn, H, **kw):
    """P (B x U) of a linear precoder: run it on the unit vectors s = e_u."""
    B, U = H.shape
    S = np.eye(U, dtype=np.complex128)[:, None, :]  # K=U symbols, 1 subcarrier
    out = fn(H[None], S, **kw)
    x = out[0]
    return x[:, 0, :].T, out


# ---------------------------------------------------------------------------
# exact brute force on tiny integer problems
# ---------------------------------------------------------------------------
def _load_golden():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def _fr(sv):
    return float(Fraction(sv))


@pytest.mark.parametrize("case", _load_golden(), ids=lambda c: "B%dU%d%s" % (c["B"], c["U"], "zf" if c["zf"] else "wf"))
def test_exact_pd(case):
    """PD-WF/ZF beta^2 and beta*x equal the exact Theorem-1 values (rel 1e-13)."""
    H = np.array([[complex(*v) for v in row] for row in case["H"]])
    s = np.array([[complex(*v) for v in row] for row in case["s"]])
    kappa = Fraction(case["kappa"])
    x, beta, st = oracle.pd(H, s[:, None, :], float(kappa), case["sizes"], zf=case["zf"])
    assert st[0] == 0
    b2 = _fr(case["pd_beta2"])
    assert abs(beta[0] ** 2 - b2) <= 1e-13 * b2
    bx = np.array([[complex(_fr(v[0]), _fr(v[1])) for v in xs] for xs in case["pd_beta_x"]])
    got = x[:, 0, :] * beta[0]
    assert np.abs(got - bx).max() <= 1e-13 * np.abs(bx).max()


@pytest.mark.parametrize("case", _load_golden(), ids=lambda c: "B%dU%d%s" % (c["B"], c["U"], "zf" if c["zf"] else "wf"))
def test_exact_fd(case):
    """FD weights^2 and x_c / w_c equal the exact Sec. III-C values."""
    H = np.array([[complex(*v) for v in row] for row in case["H"]])
    s = np.array([[complex(*v) for v in row] for row in case["s"]])
    kappa = Fraction(case["kappa"])
    x, w, st = oracle.fd(H, s[:, None, :], float(kappa), case["sizes"], zf=case["zf"],
                         tau=float(Fraction(case["tau"])))
    assert (st == 0).all()
    w2 = np.array([_fr(v) for v in case["fd_w2"]])
    assert np.allclose(w[0] ** 2, w2, rtol=1e-13, atol=0)
    ref = np.array([[complex(_fr(v[0]), _fr(v[1])) for v in xs] for xs in case["fd_x_over_w"]])
    wrow = np.repeat(w[0], case["sizes"])
    got = x[:, 0, :] / wrow[None, :]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# PD == centralized WF (Theorem 1, B x B form) at moderate sizes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B,U,sizes", [(64, 8, (32, 32)), (48, 12, (8, 16, 24)), (20, 20, (10, 10))])
def test_pd_equals_central_bxb(B, U, sizes):
    rng = _rng(1)
    H = _cn(rng, B, U)
    kappa = 0.37
    P, (x, beta, st) = _precoder_matrix(oracle.pd, H, kappa=kappa, sizes=sizes)
    Q = np.linalg.inv(H @ H.conj().T + kappa * np.eye(B)) @ H  # Theorem 1, B x B
    beta_c = math.sqrt(np.trace(Q.conj().T @ Q).real)
    # the B x B system has condition number ~ ||H||^2 / kappa: FP64 bound ~1e-11
    assert abs(beta[0] - beta_c) <= 1e-10 * beta_c
    assert np.abs(P - Q / beta_c).max() <= 1e-10 * np.abs(Q / beta_c).max()


def test_pd_independent_of_cluster_split():
    """Sec. III-B: sum_c H_c x_c = H P_WF s for any split of the array."""
    rng = _rng(2)
    cell = synth.Cell(B=96, sizes=(96,), U=10, n_sc=3, K=4)
    H, s = synth.make_cell(cell, seed=3)
    ref, bref, _ = oracle.pd(H, s, 0.5, [96])
    srng = np.random.default_rng(4)
    for C in (2, 3, 7, 96):
        sizes = synth.uneven_sizes(96, C, srng)
        x, b, _ = oracle.pd(H, s, 0.5, sizes)
        assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.allclose(b, bref, rtol=1e-13, atol=0)


# ---------------------------------------------------------------------------
# ZF: zero multi-user interference
# ---------------------------------------------------------------------------
def test_zf_zero_interference():
    """With kappa = 0 the receive vector H_dl x = H^H x equals s / beta."""
    rng = _rng(5)
    H = _cn(rng, 40, 12)
    s = _cn(rng, 3, 1, 12)
    x, beta, st = oracle.pd(H[None], s, 0.9, [20, 20], zf=True)
    y = np.einsum("bu,kb->ku", H.conj(), x[:, 0, :])
    assert np.abs(y - s[:, 0, :] / beta[0]).max() <= 1e-12


def test_zf_real_channel_transpose():
    """For a real channel H^T x = H^H x = s / beta (the 'H^T x ~ s' statement)."""
    rng = _rng(6)
    H = rng.standard_normal((32, 6)).astype(np.complex128)
    s = _cn(rng, 2, 1, 6)
    x, beta, _ = oracle.pd(H[None], s, 0.0, [32], zf=True)
    y = np.einsum("bu,kb->ku", H, x[:, 0, :])
    assert np.abs(y - s[:, 0, :] / beta[0]).max() <= 1e-12


def test_wf_has_interference_zf_does_not():
    rng = _rng(7)
    H = _cn(rng, 16, 8)
    s = _cn(rng, 1, 1, 8)
    x, beta, _ = oracle.pd(H[None], s, 2.0, [16])
    y = H.conj().T @ x[0, 0]
    assert np.abs(y - s[0, 0] / beta[0]).max() > 1e-3


# ---------------------------------------------------------------------------
# power budget (power constraint, Sec. II-A; tr(P^H P) = rho^2/Es, App. A)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("zf", [False, True])
def test_power_pd(zf):
    rng = _rng(8)
    H = _cn(rng, 64, 8)
    for power, Es in [(1.0, 1.0), (2.5, 0.5)]:
        P, _ = _precoder_matrix(oracle.pd, H, kappa=0.6, sizes=[32, 32], zf=zf, power=power, Es=Es)
        assert abs(np.sum(np.abs(P) ** 2) - power / Es) <= 1e-12 * power / Es


@pytest.mark.parametrize("sizes", [(32, 32), (4, 60), (16, 16, 32)])
def test_power_fd_per_cluster(sizes):
    """FD: every cluster spends rho_c^2 = rho^2 / C (Sec. III-C)."""
    rng = _rng(9)
    H = _cn(rng, 64, 8)
    power, Es = 2.0, 1.0
    P, (x, w, st) = _precoder_matrix(oracle.fd, H, kappa=0.6, sizes=sizes, power=power, Es=Es)
    r0 = 0
    for Bc in sizes:
        pc = np.sum(np.abs(P[r0:r0 + Bc]) ** 2)
        assert abs(pc - power / len(sizes) / Es) <= 1e-12
        r0 += Bc


# ---------------------------------------------------------------------------
# FD: both forms of Q_c and the C = 1 reduction
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("Bc_list", [(12, 4), (8, 8), (7, 9), (3, 13)])
def test_fd_forms_agree(Bc_list):
    """The oracle picks the U x U form for B_c >= U and the B_c x B_c form
    otherwise; check each cluster against the other form (push-through)."""
    U = 8
    rng = _rng(10)
    H = _cn(rng, sum(Bc_list), U)
    kappa, tau = 0.4, 0.125
    P, (x, w, st) = _precoder_matrix(oracle.fd, H, kappa=kappa, sizes=Bc_list, tau=tau)
    C = len(Bc_list)
    kc = tau * C * kappa
    r0 = 0
    for c, Bc in enumerate(Bc_list):
        Hc = H[r0:r0 + Bc]
        if Bc >= U:  # other form: B_c x B_c
            Q = np.linalg.inv(Hc @ Hc.conj().T + kc * np.eye(Bc)) @ Hc
        else:        # other form: U x U
            Q = Hc @ np.linalg.inv(Hc.conj().T @ Hc + kc * np.eye(U))
        wc = math.sqrt((1.0 / C) / np.sum(np.abs(Q) ** 2))
        assert abs(w[0, c] - wc) <= 1e-11 * wc
        assert np.abs(P[r0:r0 + Bc] - wc * Q).max() <= 1e-11 * np.abs(wc * Q).max()
        r0 += Bc


def test_fd_single_cluster_is_centralized():
    """C = 1, tau = 1 gives kappa_c = kappa and rho_c^2 = rho^2: centralized WF."""
    rng = _rng(11)
    H = _cn(rng, 24, 6)
    s = _cn(rng, 3, 1, 6)
    xp, b, _ = oracle.pd(H[None], s, 0.8, [24])
    xf, w, _ = oracle.fd(H[None], s, 0.8, [24], tau=1.0)
    assert np.abs(xp - xf).max() <= 1e-12 * np.abs(xp).max()
    assert abs(w[0, 0] - 1.0 / b[0]) <= 1e-12 / b[0]


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kappa", [0.0, 0.3, 5.0])
def test_single_user_closed_form(kappa):
    """U = 1: x = h s rho / (||h|| sqrt(Es)), beta = sqrt(Es/rho^2) ||h|| / (||h||^2 + kappa)."""
    rng = _rng(12)
    h = _cn(rng, 10, 1)
    s = _cn(rng, 2, 1, 1)
    power, Es = 1.7, 1.3
    x, beta, _ = oracle.pd(h[None], s, kappa, [4, 6], zf=(kappa == 0.0), power=power, Es=Es)
    nh = np.linalg.norm(h)
    for k in range(2):
        ref = h[:, 0] * s[k, 0, 0] * math.sqrt(power) / (nh * math.sqrt(Es))
        assert np.abs(x[k, 0] - ref).max() <= 1e-13 * np.abs(ref).max()
    assert abs(beta[0] - math.sqrt(Es / power) * nh / (nh ** 2 + kappa)) <= 1e-13


def test_orthogonal_columns_closed_form():
    """H with orthogonal columns of squared norms d_u: beta^2 = sum d_u / (d_u + kappa)^2."""
    B, U = 16, 5
    F = np.fft.fft(np.eye(B))[:, :U] / math.sqrt(B)  # orthonormal columns
    d = np.array([0.5, 1.0, 2.0, 4.0, 9.0])
    H = F * np.sqrt(d)[None, :]
    kappa = 0.7
    s = np.ones((1, 1, U), np.complex128)
    x, beta, _ = oracle.pd(H[None], s, kappa, [8, 8])
    assert abs(beta[0] ** 2 - np.sum(d / (d + kappa) ** 2)) <= 1e-13


# ---------------------------------------------------------------------------
# metamorphic invariances (consequences of Theorem 1)
# ---------------------------------------------------------------------------
def test_scale_invariance():
    """(H, kappa) -> (a H, a^2 kappa) leaves x unchanged."""
    rng = _rng(13)
    H = _cn(rng, 1, 32, 6)
    s = _cn(rng, 2, 1, 6)
    x1, _, _ = oracle.pd(H, s, 0.5, [16, 16])
    x2, _, _ = oracle.pd(3.0 * H, s, 0.5 * 9.0, [16, 16])
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x1).max()


def test_user_rotation_invariance():
    """H -> H V, s -> V^H s for a unitary V (U x U) leaves x unchanged."""
    rng = _rng(14)
    H = _cn(rng, 32, 6)
    V, _ = np.linalg.qr(_cn(rng, 6, 6))
    s = _cn(rng, 2, 1, 6)
    x1, _, _ = oracle.pd(H[None], s, 0.5, [16, 16])
    s2 = np.einsum("vu,kv->ku", V.conj(), s[:, 0, :])[:, None, :]
    x2, _, _ = oracle.pd((H @ V)[None], s2, 0.5, [16, 16])
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x1).max()


def test_cluster_rotation_equivariance():
    """H_c -> W_c H_c (W_c unitary B_c x B_c) maps x_c -> W_c x_c (PD)."""
    rng = _rng(15)
    H = _cn(rng, 32, 6)
    s = _cn(rng, 2, 1, 6)
    W, _ = np.linalg.qr(_cn(rng, 12, 12))
    H2 = H.copy()
    H2[4:16] = W @ H[4:16]
    x1, _, _ = oracle.pd(H[None], s, 0.5, [4, 12, 16])
    x2, _, _ = oracle.pd(H2[None], s, 0.5, [4, 12, 16])
    ref = x1.copy()
    ref[:, 0, 4:16] = (W @ x1[:, 0, 4:16].T).T
    assert np.abs(x2 - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# MSE optimality (problem of Sec. II-B; Lagrange condition of App. A)
# ---------------------------------------------------------------------------
def _best_mse(P, H, unoise, Es):
    """min over beta of Es ||I - beta H^H P||_F^2 + beta^2 U N0 (beta real)."""
    M = H.conj().T @ P
    U = M.shape[0]
    a = Es * np.trace(M).real
    c = Es * np.sum(np.abs(M) ** 2) + unoise
    beta = a / c
    return Es * U - a * a / c, beta


def test_wf_minimizes_mse():
    rng = _rng(16)
    B, U = 24, 6
    H = _cn(rng, B, U)
    power, Es, kappa = 1.0, 1.0, 0.45
    unoise = kappa * power  # U N0 = kappa rho^2
    P, (x, beta, _) = _precoder_matrix(oracle.pd, H, kappa=kappa, sizes=[B], power=power, Es=Es)
    f0, b0 = _best_mse(P, H, unoise, Es)
    assert abs(b0 - beta[0]) <= 1e-12 * beta[0]  # the optimal beta is Theorem 1's
    for t in range(50):
        D = _cn(rng, B, U) * (10.0 ** rng.uniform(-4, -0.5))
        P2 = P + D
        P2 *= math.sqrt(power / Es) / np.linalg.norm(P2)  # back onto the power constraint
        f2, _ = _best_mse(P2, H, unoise, Es)
        assert f2 >= f0 - 1e-12


def test_lagrange_condition():
    """beta^2 H_dl^H H_dl P + lambda P = beta H_dl^H holds with lambda = beta^2 kappa
    (the multiplier printed in App. A omits the beta^2 factor)."""
    rng = _rng(17)
    B, U = 20, 5
    H = _cn(rng, B, U)
    kappa = 0.8
    P, (x, beta, _) = _precoder_matrix(oracle.pd, H, kappa=kappa, sizes=[B])
    b = beta[0]
    res = b * b * (H @ H.conj().T) @ P + b * b * kappa * P - b * H
    assert np.abs(res).max() <= 1e-12 * np.abs(b * H).max()
    res_printed = b * b * (H @ H.conj().T) @ P + kappa * P - b * H
    assert np.abs(res_printed).max() > 1e-6


# ---------------------------------------------------------------------------
# degenerate inputs
# ---------------------------------------------------------------------------
def test_zf_rank_deficient_sets_status():
    rng = _rng(18)
    H = _cn(rng, 8, 4)
    H[:, 3] = H[:, 2]  # duplicated user column -> singular Gram under ZF
    s = _cn(rng, 1, 1, 4)
    x, beta, st = oracle.pd(H[None], s, 0.0, [8], zf=True)
    assert st[0] == 1 and beta[0] == 0.0 and not np.any(x)


def test_zero_channel_sets_status():
    H = np.zeros((1, 8, 3), np.complex128)
    s = np.ones((1, 1, 3), np.complex128)
    x, beta, st = oracle.pd(H, s, 0.5, [8])
    # Lemma 1 evaluates tr(A^-1) - kappa ||A^-1||_F^2 = 0 up to rounding here,
    # so beta may come out as a rounding-level positive number: x must be 0
    assert not np.any(x) and (st[0] == 1 or beta[0] < 1e-6)
    x, w, st = oracle.fd(H, s, 0.5, [4, 4])
    assert (st == 1).all() and not np.any(x)


def test_bad_sizes_rejected():
    H = np.zeros((1, 8, 3), np.complex128)
    s = np.ones((1, 1, 3), np.complex128)
    with pytest.raises(ValueError):
        oracle.pd(H, s, 0.5, [4, 3])
