"""FP64 oracle of the uncoded-BER link of Sec. III-D (downlink model of
Sec. II-A, UE scaling of Sec. II-B).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

One channel use per (symbol k, subcarrier n), with this package's H = H_dl^H
([n_sc][B][U]) and precoded x ([K][n_sc][B]):

    y = H_dl x + sqrt(N0) w,   w ~ CN(0, I_U)          (eq. downlinkmodel)
    s_hat_u = beta_ue y_u                               (UE scaling, Sec. II-B)

followed by nearest-point demapping of Gray-labelled square QAM and a count
of differing bits.  The noise variance follows from the SNR rho^2 / N0 (E_s = 1
symbols), and the WF regularizer is kappa = U N0 / rho^2 (Theorem 1).

UE scaling (a reading: the paper fixes beta_ue only for the WF precoder).
The MSE of Sec. II-B, E||s - beta H_dl P s||^2 + |beta|^2 U N0, is minimized
over beta for a given precoder P at

    beta = Es conj(tr E) / (Es ||E||_F^2 + U N0),   E = H_dl P  (U x U).

For P = P_WF this is beta_WF itself (the joint optimum of Theorem 1), so one
rule covers PD, centralized WF, FD and MRT; E is what the UEs would see on U
noise-free pilot symbols s = e_u.
"""
from __future__ import annotations

import numpy as np


def bits_per_symbol(order: int) -> int:
    q = int(order).bit_length() - 1
    if order < 4 or (1 << q) != order or q % 2:
        raise ValueError("square QAM with 4, 16, 64, 256 ... points expected")
    return q


def _gray_to_index(code: np.ndarray) -> np.ndarray:
    """The PAM level index i whose binary-reflected Gray code i ^ (i >> 1) is code."""
    i = code.copy()
    shift = code >> 1
    while np.any(shift):
        i ^= shift
        shift >>= 1
    return i


def pam_spacing(order: int) -> float:
    """Half the distance between neighbouring levels for unit average energy:
    E|s|^2 = 2 d^2 (m^2 - 1) / 3 = 1 with m = sqrt(order) levels per axis."""
    return float(np.sqrt(3.0 / (2.0 * (order - 1))))


def qam_map(labels: np.ndarray, order: int) -> np.ndarray:
    """Label l (an integer in [0, order)) -> unit-energy square QAM point.  The
    upper half of l's bits is the Gray code of the in-phase level, the lower
    half that of the quadrature level; level i sits at (2 i - (m - 1)) d."""
    q = bits_per_symbol(order)
    m = 1 << (q // 2)
    d = pam_spacing(order)
    lab = np.asarray(labels, dtype=np.int64)
    i_re = _gray_to_index(lab >> (q // 2))
    i_im = _gray_to_index(lab & (m - 1))
    return ((2 * i_re - (m - 1)) * d) + 1j * ((2 * i_im - (m - 1)) * d)


def demap(s_hat: np.ndarray, order: int) -> np.ndarray:
    """Nearest QAM point of every estimate, returned as its label."""
    q = bits_per_symbol(order)
    m = 1 << (q // 2)
    d = pam_spacing(order)

    def axis(v):
        i = np.floor((v / d + (m - 1)) / 2.0 + 0.5).astype(np.int64)
        i = np.clip(i, 0, m - 1)
        return i ^ (i >> 1)

    return (axis(np.real(s_hat)) << (q // 2)) | axis(np.imag(s_hat))


def bit_errors(labels_tx: np.ndarray, labels_rx: np.ndarray) -> int:
    diff = np.bitwise_xor(np.asarray(labels_tx, np.int64), np.asarray(labels_rx, np.int64))
    count = 0
    while np.any(diff):
        count += int(np.sum(diff & 1))
        diff >>= 1
    return count


def receive(H: np.ndarray, x: np.ndarray, noise, N0: float, scale) -> np.ndarray:
    """s_hat[k][n][u] = scale[n] (sum_b conj(H[n][b][u]) x[k][n][b] + sqrt(N0) w[k][n][u])."""
    H = np.asarray(H, np.complex128)
    x = np.asarray(x, np.complex128)
    y = np.einsum("nbu,knb->knu", H.conj(), x)
    if noise is not None:
        y = y + np.sqrt(N0) * np.asarray(noise, np.complex128)
    sc = np.ones(H.shape[0]) if scale is None else np.asarray(scale, np.float64)
    return y * sc[None, :, None]


def joint_beta(E: np.ndarray, N0: float, Es: float = 1.0) -> np.ndarray:
    """MSE-optimal joint UE factor per subcarrier from E [n_sc][U][U] = H_dl P;
    real part (tr E is real and positive for the WF, FD and MRT precoders)."""
    E = np.asarray(E, np.complex128)
    U = E.shape[-1]
    tr = np.trace(E, axis1=-2, axis2=-1)
    fro = np.sum(np.abs(E) ** 2, axis=(-2, -1))
    return (Es * tr.conj() / (Es * fro + U * N0)).real


def pilots(n_sc: int, U: int) -> np.ndarray:
    """U noise-free pilot symbols per subcarrier: s[u][n] = e_u ([U][n_sc][U])."""
    return np.broadcast_to(np.eye(U, dtype=np.complex128)[:, None, :], (U, n_sc, U)).copy()


def effective_channel(H: np.ndarray, x_pilot: np.ndarray) -> np.ndarray:
    """E[n] = H_dl P from the precoded pilots x_pilot [U][n_sc][B]: column u of
    E is H_dl P e_u, so E[n][:, u] = receive(...)[u][n]."""
    r = receive(H, x_pilot, None, 0.0, None)  # [U(pilot)][n_sc][U(user)]
    return np.transpose(r, (1, 2, 0))
