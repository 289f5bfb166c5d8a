"""Counter-based OFDM slot generator: the reference for the GPU's on-device simulator.

Training draws many slots; generating them on the GPU (conet_simulate) keeps the host out of
the training loop. Both sides implement the same generator from its definition, so a slot is
the same on either (bits exactly, samples to FP32 rounding), whatever the batch it belongs to.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011): 10 rounds of two 32x32->64-bit multiplies (multipliers 0xD2511F53
and 0xCD9E8D57) on a 4-word counter, the 2-word key bumped by the Weyl constants 0x9E3779B9,
0xBB67AE85 between rounds. Key = the 64-bit seed (low word first); counter = (slot, stream,
index, 0). A uniform in (0, 1) is (2 (w >> 9) + 1) 2^-24 (exact in FP32); a complex CN(0, 1)
sample is Box-Muller on two uniforms: sqrt(-ln u1) (cos 2 pi u2 + j sin 2 pi u2).

Slot model (the same structure as synth.ofdm, with a sum-of-sinusoids time variation):
  * bits uniform, m per RE (stream 2, index t F + f: word 0's bits 0..m-1); Gray QAM as
    synth.ofdm.qam_map; pilots (1 + j)/sqrt(2) on symbols 2 and 11, even subcarriers;
  * per slot (stream 1, index 0): Doppler f_D = U[0, f_max] (word 0), SNR = U[lo, hi] dB (word 1);
  * tap l of antenna n, exponential power delay profile as synth.ofdm.tap_powers:
    g(t) = sqrt(1/M) sum_{s<M} exp(j (2 pi f_D T_sym t cos(alpha_s) + phi_s)), M = 16 paths
    with alpha_s, phi_s uniform on [0, 2 pi) (stream 4, index (l N + n) M + s: words 0, 1)
    -- Clarke's isotropic scattering, whose time correlation over the path draws is
    J0(2 pi f_D T_sym dt), as the eigen-split colouring in synth.ofdm has exactly;
  * H(t, f, n) = sum_l sqrt(p_l) g_{l,n}(t) exp(-j 2 pi f df tau_l);
  * noise CN(0, sigma^2), sigma^2 = 10^(-SNR/10) (stream 3, index (t F + f) N + n).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ofdm import PILOT_SYMBOLS, PILOT_VALUE, SUBCARRIER_SPACING_HZ, SYMBOL_PERIOD_S, TAP_SPACING_S, pilot_mask, \
    qam_map, tap_powers

M_PATHS = 16
STREAM_SLOT, STREAM_BITS, STREAM_NOISE, STREAM_PATHS = 1, 2, 3, 4

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """ctr: (..., 4) uint32 counters; key: two uint32 words. Returns (..., 4) uint32."""
    c = np.asarray(ctr, dtype=np.uint32)
    x0, x1, x2, x3 = (c[..., i].astype(np.uint64) for i in range(4))
    k0, k1 = np.uint32(key[0]), np.uint32(key[1])
    for r in range(10):
        if r:
            k0 = np.uint32((int(k0) + int(_W0)) & 0xFFFFFFFF)
            k1 = np.uint32((int(k1) + int(_W1)) & 0xFFFFFFFF)
        p0 = _M0 * x0
        p1 = _M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _LO
        hi1, lo1 = p1 >> np.uint64(32), p1 & _LO
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0)), lo1, (hi0 ^ x3 ^ np.uint64(k1)), lo0
    return np.stack([x0, x1, x2, x3], axis=-1).astype(np.uint32)


def _key(seed: int):
    s = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (s & 0xFFFFFFFF, s >> 32)


def draws(seed: int, slot: int, stream: int, n: int) -> np.ndarray:
    """(n, 4) uint32 words of counters (slot, stream, i, 0), i = 0..n-1."""
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.uint32(slot & 0xFFFFFFFF)
    ctr[:, 1] = np.uint32(stream)
    ctr[:, 2] = np.arange(n, dtype=np.uint64).astype(np.uint32)
    return philox4x32_10(ctr, _key(seed))


def uniform(w: np.ndarray) -> np.ndarray:
    return ((np.asarray(w, dtype=np.uint32) >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def cnormal(w0: np.ndarray, w1: np.ndarray) -> np.ndarray:
    u1, u2 = uniform(w0), uniform(w1)
    r = np.sqrt(-np.log(u1))
    return r * (np.cos(2 * np.pi * u2) + 1j * np.sin(2 * np.pi * u2))


@dataclass(frozen=True)
class DevSimConfig:
    F: int
    n_rx: int
    bits_per_symbol: int
    n_taps: int = 8
    max_doppler_hz: float = 400.0
    snr_lo_db: float = -5.0
    snr_hi_db: float = 25.0
    seed: int = 0
    T: int = 14


def slot_params(cfg: DevSimConfig, slot: int):
    w = draws(cfg.seed, slot, STREAM_SLOT, 1)[0]
    fd = uniform(w[0:1])[0] * cfg.max_doppler_hz
    snr = cfg.snr_lo_db + uniform(w[1:2])[0] * (cfg.snr_hi_db - cfg.snr_lo_db)
    return float(fd), float(snr)


def simulate(cfg: DevSimConfig, slot: int):
    """One slot: (y (T, F, N) complex128, bits (T, F, m) uint8, H, noise_var)."""
    T, F, N, m, L = cfg.T, cfg.F, cfg.n_rx, cfg.bits_per_symbol, cfg.n_taps
    fd, snr = slot_params(cfg, slot)
    wb = draws(cfg.seed, slot, STREAM_BITS, T * F)[:, 0]
    bits = ((wb[:, None] >> np.arange(m, dtype=np.uint32)[None, :]) & np.uint32(1)).astype(np.uint8).reshape(T, F, m)
    x = np.where(pilot_mask(T, F), PILOT_VALUE, qam_map(bits))
    wp = draws(cfg.seed, slot, STREAM_PATHS, L * N * M_PATHS).reshape(L, N, M_PATHS, 4)
    alpha = 2 * np.pi * uniform(wp[..., 0])
    phi = 2 * np.pi * uniform(wp[..., 1])
    t = np.arange(T, dtype=np.float64)
    om = 2 * np.pi * fd * SYMBOL_PERIOD_S * np.cos(alpha)                          # (L, N, M)
    g = np.exp(1j * (om[..., None] * t + phi[..., None])).sum(axis=2) / np.sqrt(M_PATHS)  # (L, N, T)
    p = tap_powers(L)
    tau = np.arange(L) * TAP_SPACING_S
    ph = np.exp(-2j * np.pi * np.arange(F)[:, None] * SUBCARRIER_SPACING_HZ * tau[None, :])  # (F, L)
    H = np.einsum("fl,lnt->tfn", ph, g * np.sqrt(p)[:, None, None])
    nv = 10.0 ** (-snr / 10.0)
    wn = draws(cfg.seed, slot, STREAM_NOISE, T * F * N)
    noise = np.sqrt(nv) * cnormal(wn[:, 0], wn[:, 1]).reshape(T, F, N)
    y = H * x[..., None] + noise
    return y, bits, H, nv
