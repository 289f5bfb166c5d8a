"""Classical receiver and metrics in FP64 (test infrastructure only).

The paper compares its network with LMMSE receivers using imperfect (LS) and perfect
channel knowledge (Sec. I, Sec. IV). For a single transmit stream and N receive
antennas the LMMSE equaliser followed by unbiasing is maximum-ratio combining:
z = h^H y / ||h||^2 with effective noise variance sigma^2 / ||h||^2. Soft bits are
max-log LLRs over the M constellation points, signed as ln P(b=1)/P(b=0).
"""
from __future__ import annotations

from math import comb
from typing import Tuple

import numpy as np


def _gray_axis(c: np.ndarray) -> np.ndarray:
    """One QAM axis level from Gray bits c0..c_{k-1} (last axis), NR nesting."""
    k = c.shape[-1]
    s = 1 - 2 * c.astype(np.int64)
    v = np.ones(c.shape[:-1], dtype=np.int64)
    for i in range(k - 1, 0, -1):
        v = (1 << (k - i)) - s[..., i] * v
    return (s[..., 0] * v).astype(np.float64)


def constellation(m: int) -> Tuple[np.ndarray, np.ndarray]:
    """Square Gray M-QAM points (unit mean energy) and labels; even bits -> I, odd -> Q."""
    M = 1 << m
    labels = ((np.arange(M)[:, None] >> np.arange(m)[None, :]) & 1).astype(np.uint8)
    pts = (_gray_axis(labels[:, 0::2]) + 1j * _gray_axis(labels[:, 1::2])) / np.sqrt(2.0 * (M - 1) / 3.0)
    return pts, labels


def mrc(y: np.ndarray, h: np.ndarray, noise_var: float) -> Tuple[np.ndarray, np.ndarray]:
    """MRC/LMMSE-unbiased combining per RE: returns (z, effective noise variance)."""
    g = np.sum(np.abs(h) ** 2, axis=-1)
    z = np.sum(np.conj(h) * y, axis=-1) / g
    return z, noise_var / g


def maxlog_llr(z: np.ndarray, noise_eff: np.ndarray, m: int) -> np.ndarray:
    """Max-log LLRs (..., m): [min_{s: b_i=0} |z-s|^2 - min_{s: b_i=1} |z-s|^2] / sigma_eff^2."""
    pts, labels = constellation(m)
    d = np.abs(z[..., None] - pts) ** 2                 # (..., M)
    out = np.empty(z.shape + (m,))
    for i in range(m):
        d0 = np.where(labels[:, i] == 0, d, np.inf).min(axis=-1)
        d1 = np.where(labels[:, i] == 1, d, np.inf).min(axis=-1)
        out[..., i] = (d0 - d1) / noise_eff
    return out


def classical_rx(y: np.ndarray, h: np.ndarray, noise_var: float, m: int) -> np.ndarray:
    """LLRs (T, F, m) of the MRC + max-log receiver for one slot."""
    z, ne = mrc(y, h, noise_var)
    return maxlog_llr(z, ne, m)


def hard_bits(llr: np.ndarray) -> np.ndarray:
    """b = 1 iff LLR > 0 (an LLR of exactly 0 decides 0)."""
    return (np.asarray(llr) > 0).astype(np.uint8)


def ber(llr: np.ndarray, bits: np.ndarray, data_mask: np.ndarray) -> float:
    """Bit error rate over data REs. llr/bits: (..., T, F, m); data_mask (T, F)."""
    err = hard_bits(llr) != np.asarray(bits)
    m = np.broadcast_to(np.asarray(data_mask, bool)[..., None], err.shape[-3:])
    m = np.broadcast_to(m, err.shape)
    return float(err[m].mean())


def mrc_rayleigh_ber(snr_bit_per_branch: float, n_branches: int) -> float:
    """Textbook BER of BPSK with N-branch MRC over i.i.d. Rayleigh fading (Proakis).

    P_b = ((1-mu)/2)^N sum_{k<N} C(N-1+k, k) ((1+mu)/2)^k, mu = sqrt(g/(1+g)).
    Gray QPSK is two independent BPSK axes, each with g = Es/N0 / 2 per branch.
    """
    g = snr_bit_per_branch
    mu = np.sqrt(g / (1.0 + g))
    N = n_branches
    return float(((1 - mu) / 2) ** N * sum(comb(N - 1 + k, k) * ((1 + mu) / 2) ** k for k in range(N)))


def llr_errors(llr_x: np.ndarray, llr_ref: np.ndarray, data_mask=None) -> dict:
    """rel-L2, max-abs / RMS(ref) and sign agreement of llr_x against llr_ref."""
    a = np.asarray(llr_x, dtype=np.float64)
    r = np.asarray(llr_ref, dtype=np.float64)
    if data_mask is not None:
        m = np.broadcast_to(np.asarray(data_mask, bool)[..., None], r.shape[-3:])
        m = np.broadcast_to(m, r.shape)
        a, r = a[m], r[m]
    d = a - r
    rms = float(np.sqrt(np.mean(r ** 2)))
    return {"rel_l2": float(np.linalg.norm(d) / max(np.linalg.norm(r), 1e-300)),
            "max_abs_over_rms": float(np.abs(d).max() / max(rms, 1e-300)),
            "sign_agree": float(np.mean((a > 0) == (r > 0)))}


def snr_gap_db(snr_grid, ber_a, ber_b, target: float) -> float:
    """Horizontal gap (dB) between two BER curves at a target BER (log-linear interpolation)."""
    def cross(ber):
        lb = np.log10(np.maximum(np.asarray(ber, float), 1e-12))
        s = np.asarray(snr_grid, float)
        for i in range(len(s) - 1):
            if (lb[i] - np.log10(target)) * (lb[i + 1] - np.log10(target)) <= 0 and lb[i] != lb[i + 1]:
                return s[i] + (np.log10(target) - lb[i]) * (s[i + 1] - s[i]) / (lb[i + 1] - lb[i])
        return np.nan
    return float(cross(ber_a) - cross(ber_b))
