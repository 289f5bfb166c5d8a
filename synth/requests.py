"""Seeded serving workload: slot requests of uneven PRB allocations, antenna counts and
modulations, and Poisson arrival times."""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from .ofdm import SimConfig, simulate_slot

N_RX = (2, 4)
BITS = (2, 4, 6)          # QPSK, 16-QAM, 64-QAM


@dataclass
class Request:
    n_prb: int
    n_rx: int
    m: int
    x: np.ndarray           # [14, 12 n_prb, 4 n_rx] float32 features
    bits: np.ndarray        # [14, 12 n_prb, m] uint8
    seed: int
    y: np.ndarray = None    # [14, 12 n_prb, n_rx, 2] float32 received grid (Re, Im)


def make_requests(n: int, seed: int = 5, prb_range=(4, 273)) -> List[Request]:
    """n requests: n_prb ~ U{lo..hi}, n_rx ~ U{2,4}, m ~ U{2,4,6}; request i's slot is
    simulated with the 8-tap Jakes channel and SNR U[-5, 25] dB from SeedSequence([seed, i])."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 1 << 20])))
    out = []
    for i in range(n):
        n_prb = int(rng.integers(prb_range[0], prb_range[1] + 1))
        n_rx = int(N_RX[rng.integers(0, 2)])
        m = int(BITS[rng.integers(0, 3)])
        sim = SimConfig(F=12 * n_prb, n_rx=n_rx, bits_per_symbol=m, n_taps=8, max_doppler_hz=400.0, seed=seed)
        sl = simulate_slot(sim, i)
        y = np.stack([sl.y.real, sl.y.imag], axis=-1).astype(np.float32)
        out.append(Request(n_prb, n_rx, m, sl.features, sl.bits, i, y))
    return out


def poisson_arrivals(rate_per_s: float, n: int, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 2 << 20])))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
