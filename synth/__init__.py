"""Seeded synthetic workloads for decentralized precoding.

This module only draws inputs: channels, symbols, cluster splits, cell mixes
and arrival times.  It holds none of the precoding arithmetic, so both the
HIP library's tests/benchmarks and the FP64 oracle can use it.

Shapes follow the paper's system model and LTE framing (Sec. II-A, III-D,
IV-C): i.i.d. Rayleigh (or exponentially correlated) channels that stay fixed
over the K OFDM symbols of a frame, unit-energy QAM symbols, and the channel
stored antenna-major as H[n_sc][B][U] (B x U per subcarrier).

Regularizer: with unit power budget rho^2 = 1 and SNR = rho^2 / N0, the WF
regularizer U N0 / rho^2 of Theorem 1 equals U / SNR; ``Cell.kappa`` holds it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

QAM_ORDERS = (4, 16, 64)


@dataclasses.dataclass(frozen=True)
class Cell:
    """One precoding problem: n_sc subcarriers x K symbols of one cell."""

    B: int
    sizes: tuple
    U: int
    n_sc: int
    K: int = 14
    snr_db: float = 10.0
    channel: str = "rayleigh"  # or "kron" (exponential correlation over antennas)
    r: float = 0.5
    qam: int = 16

    @property
    def C(self) -> int:
        return len(self.sizes)

    @property
    def kappa(self) -> float:
        return self.U / (10.0 ** (self.snr_db / 10.0))

    def with_(self, **kw) -> "Cell":
        return dataclasses.replace(self, **kw)


def config(i: int) -> Cell:
    """The paper-shaped workloads (index 1..3; 4 and 5 are mixes, see ``mix``)."""
    if i == 1:  # tiny: seconds for the oracle
        return Cell(B=64, sizes=(32, 32), U=8, n_sc=64, K=14, snr_db=10.0, qam=4)
    if i == 2:  # B=256 as 8 clusters of 32, U=16, 20 MHz LTE (1200 subcarriers)
        return Cell(B=256, sizes=(32,) * 8, U=16, n_sc=1200, K=14, snr_db=10.0, qam=16)
    if i == 3:  # precision workload: correlated channel
        return Cell(B=512, sizes=(32,) * 16, U=32, n_sc=3300, K=14, snr_db=10.0,
                    channel="kron", r=0.5, qam=16)
    raise ValueError("config index must be 1, 2 or 3")


def _rng(*key) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


def rayleigh(n_sc: int, B: int, U: int, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. CN(0,1) entries: re, im ~ N(0, 1/2)."""
    re = rng.standard_normal((n_sc, B, U), dtype=np.float32)
    im = rng.standard_normal((n_sc, B, U), dtype=np.float32)
    h = np.empty((n_sc, B, U), np.complex64)
    h.real = re * np.float32(math.sqrt(0.5))
    h.imag = im * np.float32(math.sqrt(0.5))
    return h


def kron_exp(n_sc: int, B: int, U: int, r: float, rng: np.random.Generator) -> np.ndarray:
    """Kronecker channel with exponential correlation r^|i-j| over the antenna
    index and independent users, drawn as the AR(1) recursion
    h_0 = w_0, h_b = r h_{b-1} + sqrt(1-r^2) w_b (unit variance, exact)."""
    w = rayleigh(n_sc, B, U, rng).astype(np.complex128)
    h = np.empty_like(w)
    h[:, 0] = w[:, 0]
    a = math.sqrt(1.0 - r * r)
    for b in range(1, B):
        h[:, b] = r * h[:, b - 1] + a * w[:, b]
    return h.astype(np.complex64)


def qam(shape, order: int, rng: np.random.Generator) -> np.ndarray:
    """Unit-average-energy square QAM symbols (QPSK, 16-QAM, 64-QAM)."""
    m = int(round(math.sqrt(order)))
    if m * m != order or order not in QAM_ORDERS:
        raise ValueError("order must be 4, 16 or 64")
    levels = np.arange(-(m - 1), m, 2, dtype=np.float64)
    scale = math.sqrt(2.0 * (order - 1) / 3.0)
    re = levels[rng.integers(0, m, size=shape)]
    im = levels[rng.integers(0, m, size=shape)]
    return ((re + 1j * im) / scale).astype(np.complex64)


def channel(cell: Cell, seed: int = 0, cell_id: int = 0, frame: int = 0) -> np.ndarray:
    rng = _rng(1, seed, cell_id, frame)
    if cell.channel == "kron":
        return kron_exp(cell.n_sc, cell.B, cell.U, cell.r, rng)
    return rayleigh(cell.n_sc, cell.B, cell.U, rng)


def symbols(cell: Cell, seed: int = 0, cell_id: int = 0, frame: int = 0) -> np.ndarray:
    rng = _rng(2, seed, cell_id, frame)
    return qam((cell.K, cell.n_sc, cell.U), cell.qam, rng)


def make_cell(cell: Cell, seed: int = 0, cell_id: int = 0, frame: int = 0):
    """(H [n_sc][B][U], s [K][n_sc][U]) complex64 for one frame of a cell."""
    return channel(cell, seed, cell_id, frame), symbols(cell, seed, cell_id, frame)


def uneven_sizes(B: int, C: int, rng: np.random.Generator, min_size: int = 1) -> tuple:
    """A random composition of B into C positive parts (w_c != 1/C, Sec. III-A)."""
    cuts = np.sort(rng.choice(np.arange(1, B - (min_size - 1) * C), size=C - 1, replace=False))
    parts = np.diff(np.concatenate([[0], cuts, [B - (min_size - 1) * C]])) + (min_size - 1)
    return tuple(int(p) for p in parts)


def mix(n_cells: int = 64, seed: int = 0, uneven: bool = False,
        B_choices: Sequence[int] = (64, 128, 256, 512), Bc_choices: Sequence[int] = (16, 32, 64),
        U_range=(4, 64), nsc_choices: Sequence[int] = (300, 1200, 3300), K: int = 14,
        snr_range=(0.0, 20.0)) -> List[Cell]:
    """Heterogeneous batch of cells: B, cluster size, U, subcarrier count and SNR
    drawn per cell (U <= B); optionally uneven cluster sizes."""
    rng = _rng(4, seed)
    cells = []
    for _ in range(n_cells):
        B = int(rng.choice(B_choices))
        Bc = int(rng.choice([b for b in Bc_choices if b <= B]))
        C = B // Bc
        U = int(rng.integers(U_range[0], min(U_range[1], B) + 1))
        n_sc = int(rng.choice(nsc_choices))
        snr = float(rng.uniform(*snr_range))
        sizes = uneven_sizes(B, C, rng) if (uneven and C > 1) else (Bc,) * C
        cells.append(Cell(B=B, sizes=sizes, U=U, n_sc=n_sc, K=K, snr_db=snr, qam=16))
    return cells


def poisson_arrivals(rate_hz: float, n_jobs: int, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = _rng(5, seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n_jobs))


def device_cell(cell: Cell, device, seed: int = 0, cell_id: int = 0):
    """(H, s) like make_cell, drawn directly in device memory with a seeded
    torch generator (i.i.d. CN(0,1) channel, uniform QAM symbols): for large
    serving mixes where host generation would dominate.  Not bit-identical to
    make_cell."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed((seed * 1_000_003 + cell_id) & 0x7FFFFFFF)
    H = torch.randn((cell.n_sc, cell.B, cell.U, 2), generator=g, device=device) * math.sqrt(0.5)
    m = int(round(math.sqrt(cell.qam)))
    lv = torch.randint(0, m, (cell.K, cell.n_sc, cell.U, 2), generator=g, device=device).float() * 2 - (m - 1)
    lv = lv / math.sqrt(2.0 * (m * m - 1) / 3.0)
    return torch.view_as_complex(H.contiguous()), torch.view_as_complex(lv.contiguous())


# ---------------------------------------------------------------------------
# uncoded-BER link inputs (Sec. III-D): random labels and receiver noise only
# ---------------------------------------------------------------------------
def labels(shape, order: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform QAM labels in [0, order) (the information bits), int32."""
    return rng.integers(0, order, size=shape, dtype=np.int64).astype(np.int32)


def cn_noise(shape, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. CN(0, 1) samples (unit variance per complex entry), complex64."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return ((re + 1j * im) / math.sqrt(2.0)).astype(np.complex64)


def link_frame(cell: Cell, seed: int = 0, frame: int = 0):
    """(H [n_sc][B][U], labels [K][n_sc][U] int32, noise [K][n_sc][U]) for one
    frame of an uncoded-BER run on the cell (labels in [0, cell.qam))."""
    H = channel(cell, seed, 0, frame)
    rng = _rng(6, seed, frame)
    return H, labels((cell.K, cell.n_sc, cell.U), cell.qam, rng), cn_noise((cell.K, cell.n_sc, cell.U), rng)


def device_link_frame(cell: Cell, device, seed: int = 0, frame: int = 0):
    """link_frame drawn in device memory with a seeded torch generator
    (i.i.d. CN(0,1) channel): for long Monte Carlo runs.  Not bit-identical
    to link_frame."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed((seed * 1_000_003 + frame * 7919 + 17) & 0x7FFFFFFF)
    H = torch.randn((cell.n_sc, cell.B, cell.U, 2), generator=g, device=device) * math.sqrt(0.5)
    lab = torch.randint(0, cell.qam, (cell.K, cell.n_sc, cell.U), generator=g, device=device, dtype=torch.int32)
    w = torch.randn((cell.K, cell.n_sc, cell.U, 2), generator=g, device=device) * math.sqrt(0.5)
    return torch.view_as_complex(H.contiguous()), lab, torch.view_as_complex(w.contiguous())
