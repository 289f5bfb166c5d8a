"""Shared test helpers: seeded inputs and the comparison metrics used by the parity tests."""
from __future__ import annotations

import sys

import numpy as np

from synth import ModelConfig, SimConfig, make_blob, simulate_slot


def say(*a):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print(*a, flush=True)
    sys.stdout.flush()


def features(sim: SimConfig, n_slots: int, first: int = 0) -> np.ndarray:
    return np.stack([simulate_slot(sim, first + s).features for s in range(n_slots)])


def rel_l2(a, r) -> float:
    a = np.asarray(a, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300))


def max_over_rms(a, r) -> float:
    a = np.asarray(a, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.abs(a - r).max() / max(np.sqrt(np.mean(r ** 2)), 1e-300))


def sign_agree(a, r) -> float:
    return float(np.mean((np.asarray(a) > 0) == (np.asarray(r) > 0)))
