"""Seeded OFDM uplink simulator: the synthetic input generator for CoNet-Rx.

This module makes the receiver's inputs. It holds none of the receiver network's
arithmetic, and both the FP64 oracle's tests and the GPU path's tests/bench draw
their inputs from it.

What it simulates (paper, Sec. II, Eq. (1), and the simulation setup of Sec. IV):
  * uniformly random information bits (Sec. II, first paragraph);
  * square Gray M-QAM mapping with unit average energy (Sec. II; 64-QAM in Sec. IV);
  * a TTI of T = 14 OFDM symbols over F subcarriers, with fixed DMRS pilots on
    designated subcarriers (Sec. II; Sec. II-A says the pilots are fixed);
  * the per-RE SIMO observation y = h x + g z + n of Eq. (1); the interference term g z
    (another transmitter's QAM symbols through its own Rayleigh channel, a random share
    of the noise-plus-interference power) only where a configuration asks for it, and
    the FFT/IFFT pair omitted (without ICI or timing offset the
    pair is the identity on a per-RE model);
  * LS channel estimates at the pilots, linearly interpolated over the grid (Sec. I);
  * the real NHWC input tensor: Re/Im of Y and of the LS estimate per rx antenna
    (Sec. II-A builds the input from Re/Im parts of Y).

Readings where the paper is silent (each is listed in the design notes):
  * channel: exponential power-delay profile Rayleigh taps at 200 ns spacing with a
    300 ns decay constant, i.i.d. across antennas, Jakes/Clarke time correlation
    J0(2 pi f_D dt) sampled at the OFDM symbol period, 30 kHz subcarrier spacing;
  * SNR per RE per antenna with unit symbol and channel power, sigma^2 = 10^(-SNR/10);
  * pilots on 0-based symbols 2 and 11, even subcarriers, value (1+j)/sqrt(2);
  * NR-style Gray labelling: even bits drive I, odd bits drive Q.

Random-number contract: slot s of a configuration with seed S draws from
numpy.random.Generator(PCG64(SeedSequence([S, s]))) in this order:
bits (T, F, m) -> Doppler f_D (if the channel is time-varying) -> SNR (if ranged)
-> tap gains (n_taps, N, T) real part then imaginary part -> noise (T, F, N) real
part then imaginary part [-> with an interferer: its power share, its bits (T, F, m),
its Doppler, its tap gains real then imaginary]. Any slot can therefore be regenerated
alone, and configurations without an interferer draw exactly what they drew before it
existed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

T_SYMBOLS = 14
PILOT_SYMBOLS = (2, 11)
SUBCARRIER_SPACING_HZ = 30e3
SYMBOL_PERIOD_S = 0.5e-3 / 14.0
TAP_SPACING_S = 200e-9
PDP_DECAY_S = 300e-9
PILOT_VALUE = (1.0 + 1.0j) / np.sqrt(2.0)


@dataclass(frozen=True)
class SimConfig:
    """One workload's simulator settings."""
    F: int                      # subcarriers
    n_rx: int                   # receive antennas N
    bits_per_symbol: int        # m = log2 M (even: square QAM)
    n_taps: int = 8
    max_doppler_hz: float = 400.0   # f_D ~ U[0, max]; 0 => block fading
    snr_db: Optional[float] = None  # fixed SNR, or None for a uniform range
    snr_range_db: Tuple[float, float] = (-5.0, 25.0)
    seed: int = 0
    T: int = T_SYMBOLS
    # Interference g z of Eq. (1): a second transmitter's QAM symbols (same modulation, data on
    # every RE) through its own Rayleigh channel. Per slot its share of the noise-plus-
    # interference power is U[lo, hi] (the paper trains with 10-90 %); None: no interferer.
    interference_share: Optional[Tuple[float, float]] = None
    # Append the known noise and interference variances to the input (Sec. II-A): 8 more
    # channels (sigma_n^2, sigma_i^2, then zeros, so the width stays a multiple of 8).
    variance_channels: bool = False


VARIANCE_CHANNELS = 8


@dataclass
class Slot:
    """One simulated TTI (all arrays for a single slot)."""
    bits: np.ndarray         # (T, F, m) uint8
    x: np.ndarray            # (T, F) complex128, transmitted symbols (pilots included)
    H: np.ndarray            # (T, F, N) complex128, true channel
    y: np.ndarray            # (T, F, N) complex128, received grid
    H_ls: np.ndarray         # (T, F, N) complex128, LS + linear interpolation
    noise_var: float         # noise + interference variance per RE and antenna (1 / SINR)
    snr_db: float
    doppler_hz: float
    features: np.ndarray     # (T, F, 4N [+ 8]) float32, NHWC input of the network
    interf_var: float = 0.0  # the interference's part of noise_var


# ----------------------------------------------------------------------------- QAM

def qam_axis_levels(bits_axis: np.ndarray) -> np.ndarray:
    """Amplitude of one QAM axis from its k Gray-coded bits (last axis, c0 first).

    Follows the nested form A = s0 (2^{k-1} - s1 (2^{k-2} - ... (2 - s_{k-1}))),
    s_i = 1 - 2 c_i, used for the NR square constellations.
    """
    c = np.asarray(bits_axis, dtype=np.int64)
    k = c.shape[-1]
    s = 1 - 2 * c
    tail = np.ones(c.shape[:-1], dtype=np.int64)
    for i in range(k - 1, 0, -1):
        tail = (1 << (k - i)) - s[..., i] * tail
    return (s[..., 0] * tail).astype(np.float64)


def qam_norm(bits_per_symbol: int) -> float:
    M = 1 << bits_per_symbol
    return float(np.sqrt(2.0 * (M - 1) / 3.0))


def qam_map(bits: np.ndarray) -> np.ndarray:
    """Map (..., m) bits to unit-energy square Gray QAM symbols.

    Even-indexed bits (b0, b2, ...) set the in-phase level, odd ones the quadrature.
    """
    bits = np.asarray(bits)
    m = bits.shape[-1]
    if m % 2 != 0 or m < 2:
        raise ValueError("square QAM needs an even number of bits per symbol")
    a_i = qam_axis_levels(bits[..., 0::2])
    a_q = qam_axis_levels(bits[..., 1::2])
    return (a_i + 1j * a_q) / qam_norm(m)


def constellation(bits_per_symbol: int) -> Tuple[np.ndarray, np.ndarray]:
    """All M points and their bit labels, label index = sum b_i 2^i."""
    m = bits_per_symbol
    M = 1 << m
    labels = ((np.arange(M)[:, None] >> np.arange(m)[None, :]) & 1).astype(np.uint8)
    return qam_map(labels), labels


# ----------------------------------------------------------------------------- grid

def pilot_mask(T: int, F: int) -> np.ndarray:
    """Boolean (T, F): True on DMRS pilot REs (symbols 2 and 11, even subcarriers)."""
    mask = np.zeros((T, F), dtype=bool)
    for t in PILOT_SYMBOLS:
        if t < T:
            mask[t, 0::2] = True
    return mask


def data_mask(T: int, F: int) -> np.ndarray:
    return ~pilot_mask(T, F)


# ----------------------------------------------------------------------------- channel

def tap_powers(n_taps: int) -> np.ndarray:
    tau = np.arange(n_taps) * TAP_SPACING_S
    p = np.exp(-tau / PDP_DECAY_S)
    return p / p.sum()


def jakes_covariance(T: int, doppler_hz: float) -> np.ndarray:
    """R[t, t'] = J0(2 pi f_D (t - t') T_sym) (Clarke's isotropic scattering)."""
    from scipy.special import j0
    dt = np.arange(T)[:, None] - np.arange(T)[None, :]
    return j0(2.0 * np.pi * doppler_hz * dt * SYMBOL_PERIOD_S)


def correlated_gains(w: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Colour i.i.d. CN(0,1) samples w[..., T] with covariance R via its eigen-split."""
    lam, V = np.linalg.eigh(R)
    A = V * np.sqrt(np.maximum(lam, 0.0))[None, :]
    return np.einsum("ts,...s->...t", A, w)


def freq_response(gains: np.ndarray, n_taps: int, F: int) -> np.ndarray:
    """H[t, f, n] = sum_l sqrt(p_l) g_{l,n}[t] exp(-j 2 pi f df tau_l).

    gains: (n_taps, N, T) complex.
    """
    p = tap_powers(n_taps)
    tau = np.arange(n_taps) * TAP_SPACING_S
    f = np.arange(F)
    phase = np.exp(-2j * np.pi * f[:, None] * SUBCARRIER_SPACING_HZ * tau[None, :])  # (F, L)
    g = gains * np.sqrt(p)[:, None, None]                                          # (L, N, T)
    return np.einsum("fl,lnt->tfn", phase, g)


# ----------------------------------------------------------------------------- LS

def ls_estimate(y: np.ndarray) -> np.ndarray:
    """LS at pilots, linear interpolation along f then along t (Sec. I: LS estimation).

    y: (T, F, N). Pilot REs: symbols 2 and 11, even subcarriers, value (1+j)/sqrt(2).
    Along f (on each pilot symbol) odd subcarriers take the mean of both even
    neighbours; a trailing odd subcarrier copies its left neighbour. Along t every
    symbol lies on the line through symbols 2 and 11 (extrapolated at the edges).
    """
    T, F, N = y.shape
    t0, t1 = PILOT_SYMBOLS
    rows = []
    for t in (t0, t1):
        h = np.zeros((F, N), dtype=np.complex128)
        h[0::2] = y[t, 0::2] / PILOT_VALUE
        for f in range(1, F, 2):
            if f + 1 < F:
                h[f] = 0.5 * (h[f - 1] + h[f + 1])
            else:
                h[f] = h[f - 1]
        rows.append(h)
    h0, h1 = rows
    t = np.arange(T, dtype=np.float64)[:, None, None]
    return h0[None] + (t - t0) / float(t1 - t0) * (h1 - h0)[None]


def make_features(y: np.ndarray, H_ls: np.ndarray, variances: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """X[t, f, 4n + (0,1,2,3)] = (Re y_n, Im y_n, Re H_n, Im H_n), float32, antenna-major;
    with variances = (sigma_n^2, sigma_i^2) also channels 4N, 4N + 1 = those (constant over
    the slot) and 4N + 2 .. 4N + 7 = 0."""
    T, F, N = y.shape
    X = np.empty((T, F, N, 4), dtype=np.float64)
    X[..., 0] = y.real
    X[..., 1] = y.imag
    X[..., 2] = H_ls.real
    X[..., 3] = H_ls.imag
    X = X.reshape(T, F, 4 * N)
    if variances is not None:
        V = np.zeros((T, F, VARIANCE_CHANNELS))
        V[..., 0], V[..., 1] = variances
        X = np.concatenate([X, V], axis=-1)
    return X.astype(np.float32)


# ----------------------------------------------------------------------------- slots

def slot_rng(seed: int, slot: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(slot)])))


def simulate_slot(cfg: SimConfig, slot: int, noise_var_override: Optional[float] = None,
                  channel_override: Optional[np.ndarray] = None) -> Slot:
    """Simulate one TTI. Overrides exist for the noiseless and known-channel pins."""
    T, F, N, m = cfg.T, cfg.F, cfg.n_rx, cfg.bits_per_symbol
    rng = slot_rng(cfg.seed, slot)
    bits = rng.integers(0, 2, size=(T, F, m), dtype=np.uint8)
    doppler = float(rng.uniform(0.0, cfg.max_doppler_hz)) if cfg.max_doppler_hz > 0 else 0.0
    if cfg.snr_db is None:
        snr_db = float(rng.uniform(*cfg.snr_range_db))
    else:
        snr_db = float(cfg.snr_db)
    wr = rng.standard_normal((cfg.n_taps, N, T))
    wi = rng.standard_normal((cfg.n_taps, N, T))
    nr = rng.standard_normal((T, F, N))
    ni = rng.standard_normal((T, F, N))

    x = qam_map(bits)
    pm = pilot_mask(T, F)
    x = np.where(pm, PILOT_VALUE, x)

    if channel_override is not None:
        H = np.broadcast_to(channel_override, (T, F, N)).astype(np.complex128)
    else:
        w = (wr + 1j * wi) / np.sqrt(2.0)
        if cfg.max_doppler_hz > 0:
            gains = correlated_gains(w, jakes_covariance(T, doppler))
        else:  # block fading: one draw per tap and antenna, held over the TTI
            gains = np.repeat(w[..., :1], T, axis=-1)
        H = freq_response(gains, cfg.n_taps, F)

    total = 10.0 ** (-snr_db / 10.0) if noise_var_override is None else float(noise_var_override)
    share, gz = 0.0, 0.0
    if cfg.interference_share is not None:
        share = float(rng.uniform(*cfg.interference_share))
        zbits = rng.integers(0, 2, size=(T, F, m), dtype=np.uint8)
        doppler_i = float(rng.uniform(0.0, cfg.max_doppler_hz)) if cfg.max_doppler_hz > 0 else 0.0
        gr = rng.standard_normal((cfg.n_taps, N, T))
        gi = rng.standard_normal((cfg.n_taps, N, T))
        wg = (gr + 1j * gi) / np.sqrt(2.0)
        if cfg.max_doppler_hz > 0:
            ggains = correlated_gains(wg, jakes_covariance(T, doppler_i))
        else:
            ggains = np.repeat(wg[..., :1], T, axis=-1)
        G = freq_response(ggains, cfg.n_taps, F)
        gz = np.sqrt(share * total) * G * qam_map(zbits)[..., None]   # unit-power z and G
    interf_var = share * total
    n = np.sqrt((total - interf_var) / 2.0) * (nr + 1j * ni)
    y = H * x[..., None] + gz + n
    H_ls = ls_estimate(y)
    var = ((total - interf_var), interf_var) if cfg.variance_channels else None
    return Slot(bits=bits, x=x, H=H, y=y, H_ls=H_ls, noise_var=total, snr_db=snr_db,
                doppler_hz=doppler, features=make_features(y, H_ls, var), interf_var=interf_var)


def simulate_batch(cfg: SimConfig, n_slots: int, first_slot: int = 0):
    """Features (B, T, F, 4N) float32, bits (B, T, F, m) uint8, data mask (T, F), slots."""
    slots = [simulate_slot(cfg, first_slot + s) for s in range(n_slots)]
    X = np.stack([s.features for s in slots])
    bits = np.stack([s.bits for s in slots])
    return X, bits, data_mask(cfg.T, cfg.F), slots


def features_fast(cfg: SimConfig, n_slots: int, first_slot: int = 0, n_distinct: int = 4):
    """Large batches: simulate n_distinct slots and tile them to n_slots.

    Throughput runs need hundreds of MB of realistic input; simulating every slot on
    the host would dominate set-up time, and the receiver's cost does not depend on
    the values. Slot s of the result equals simulated slot first_slot + (s mod n_distinct).
    """
    n_distinct = max(1, min(n_distinct, n_slots))
    base = np.stack([simulate_slot(cfg, first_slot + s).features for s in range(n_distinct)])
    reps = -(-n_slots // n_distinct)
    return np.concatenate([base] * reps, axis=0)[:n_slots]
