"""Uncoded-BER link of Sec. III-D on the library's kernels.

Argument marshalling and orchestration only: the precoders (precode_pd,
precode_fd, precode_central, precode_mrt), the QAM mapping, the receive
model y = H_dl x + n of Sec. II-A, the UE factor and the bit-error count all
run in the library (include/precode.h).

SNR = rho^2 / N0 with E_s = 1 symbols, so N0 = rho^2 / SNR and the WF
regularizer of Theorem 1 is kappa = U N0 / rho^2.  The UE factor (Sec. II-B):
PD and centralized WF use their beta_WF; FD and MRT, whose precoders the
paper gives no UE factor for, use the MSE-optimal joint factor measured on U
noise-free pilots (for a WF precoder this equals beta_WF).
"""
from __future__ import annotations

import math

from . import Context, params, qam_errors, qam_map, ue_gain, ue_receive

SCHEMES = ("pd", "fd", "central", "mrt")


def noise_var(snr_db: float, power: float = 1.0) -> float:
    return power / (10.0 ** (snr_db / 10.0))


def _pilots(torch, n_sc, U, device):
    eye = torch.eye(U, dtype=torch.complex64, device=device)
    return eye[:, None, :].expand(U, n_sc, U).contiguous()


def precode(ctx: Context, scheme: str, H, s, kappa: float, sizes, mode="wf", tau=0.125, power=1.0, Es=1.0,
            precision="fp32", stream=None):
    """x of one precoder, with its own factor (beta, or None for FD / MRT)."""
    prm = params(power=power, Es=Es, tau=tau, precision=precision)
    if scheme == "pd":
        x, beta, _ = ctx.pd(H, s, kappa, sizes, mode, prm, stream=stream)
        return x, beta
    if scheme == "fd":
        x, _, _ = ctx.fd(H, s, kappa, sizes, mode, prm, stream=stream)
        return x, None
    if scheme == "central":
        x, beta, _ = ctx.central(H, s, kappa, params(power=power, Es=Es), stream=stream)
        return x, beta
    if scheme == "mrt":
        x, _, _ = ctx.mrt(H, s, sizes, params(power=power, Es=Es), stream=stream)
        return x, None
    raise ValueError("scheme must be one of %s" % (SCHEMES,))


def frame_errors(ctx: Context, scheme: str, H, labels, noise, snr_db: float, order: int, sizes, mode="wf",
                 tau=0.125, power=1.0, Es=1.0, precision="fp32", joint=False, count=None, labels_out=None,
                 stream=None):
    """Bit errors of one frame, added to the device counter `count` (created if
    None).  joint=True uses the pilot-measured joint factor for every scheme.
    Returns (count, s_hat, ue_scale)."""
    import torch

    n_sc, B, U = H.shape
    N0 = noise_var(snr_db, power)
    kappa = U * N0 / power
    s = qam_map(labels, order, stream=stream)
    x, scale = precode(ctx, scheme, H, s, kappa, sizes, mode, tau, power, Es, precision, stream)
    if scale is None or joint:
        xp, _ = precode(ctx, scheme, H, _pilots(torch, n_sc, U, H.device), kappa, sizes, mode, tau, power, Es,
                        precision, stream)
        scale = ue_gain(ue_receive(H, xp, stream=stream), N0, Es, stream=stream)
    s_hat = ue_receive(H, x, noise, N0, scale, stream=stream)
    count, _ = qam_errors(s_hat, labels, order, count=count, labels_out=labels_out, stream=stream)
    return count, s_hat, scale


def ber(ctx: Context, scheme: str, cell, snr_db: float, frames: int, seed: int = 0, tau=0.125, power=1.0,
        precision="fp32", joint=False) -> float:
    """Uncoded BER of a scheme on `frames` seeded device-drawn frames of a cell
    (synth.device_link_frame), counted on the device."""
    import torch

    import synth

    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    for f in range(frames):
        H, lab, w = synth.device_link_frame(cell, "cuda", seed, f)
        frame_errors(ctx, scheme, H, lab, w, snr_db, cell.qam, cell.sizes, "wf", tau, power, 1.0, precision, joint,
                     count=count)
    bits = frames * cell.K * cell.n_sc * cell.U * int(math.log2(cell.qam))
    return int(count.item()) / bits
