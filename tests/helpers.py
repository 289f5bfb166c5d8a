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


def emulation_with_bound(p, X64, quant, draws: int = 2, kappa: float = 4.0, sel=None, **kw):
    """The oracle's emulation of a reduced-precision contract and tolerances for a GPU run of it.

    The oracle's error model (forward's acc_noise) perturbs each conv sum and the head the way
    the GPU's accumulation does (FP32 rounding; for FP8 also the matrix instruction's truncation
    within groups of 8 products) and every value rounded to BF16 or e4m3 by the FP32 error of
    the operations forming it. Over `draws` noise draws, the element-wise tolerance is kappa
    times the largest element-wise move and the rel-L2 tolerance twice the largest rel-L2 move.
    A kernel mistake (a wrong tap, channel, tile column or slot edge) is not of that kind.
    sel (optional) picks the outputs compared (e.g. a window's own subcarriers).
    Returns (emulation, element-wise bound, rel-L2 bound)."""
    from oracle import conet64 as o
    sel = sel or (lambda a: a)
    emu = sel(o.forward_slots(p, X64, quant=quant, **kw))
    dev, rel = 0.0, 0.0
    for j in range(draws):
        noisy = sel(o.forward_slots(p, X64, quant=quant, acc_noise=np.random.default_rng(7919 + j), **kw))
        dev = max(dev, float(np.abs(noisy - emu).max()))
        rel = max(rel, rel_l2(noisy, emu))
    return emu, kappa * dev, 2.0 * rel


def elementwise_report(got, ref, tw: int, label: str = "") -> dict:
    """Worst |got - ref| over all LLRs and separately over the REs where a tiling or padding
    mistake would show first: the first and last subcarrier of every tile of width tw (tile
    seams), the slot's first and last subcarrier and its first and last symbol (zero padding),
    and the remaining interior. got/ref: (B, T, F, m). Printed and returned."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.abs(got - ref)
    B, T, F, m = d.shape
    f = np.arange(F)
    seam = np.zeros(F, bool)
    if tw > 0:
        seam = (f % tw == 0) | (f % tw == tw - 1) | (f == F - 1)
    fedge = (f == 0) | (f == F - 1)
    tedge = np.zeros(T, bool)
    tedge[[0, T - 1]] = True
    groups = {"all": np.ones((T, F), bool), "tile_seams": np.broadcast_to(seam[None, :], (T, F)),
              "slot_edge_subcarriers": np.broadcast_to(fedge[None, :], (T, F)),
              "slot_edge_symbols": np.broadcast_to(tedge[:, None], (T, F))}
    groups["interior"] = ~(groups["tile_seams"] | groups["slot_edge_subcarriers"] | groups["slot_edge_symbols"])
    out = {}
    for name, msk in groups.items():
        sel = d[:, msk, :] if msk.any() else np.zeros(1)
        out[name] = (float(sel.max()), float(sel.mean()))
    i = np.unravel_index(int(np.argmax(d)), d.shape)
    out["worst_index"] = tuple(int(v) for v in i)
    say(f"  {label} max|d| {out['all'][0]:.3e} at (slot, t, f, bit) = {out['worst_index']}; "
        + ", ".join(f"{k} max {v[0]:.2e} mean {v[1]:.2e}" for k, v in out.items() if k not in ("all", "worst_index")))
    return out


def check_vs_emulation(got, p, X64, quant, tw, label, **kw):
    """Parity against the emulating oracle with the tolerances its GPU error model gives
    (emulation_with_bound): every LLR within the element-wise bound, rel-L2 within the rel
    bound, and tile seams no worse on average than the interior (the per-RE arithmetic does
    not depend on the tiling). Returns the emulation."""
    emu, bound, rel_bound = emulation_with_bound(p, X64, quant, **kw)
    rms = float(np.sqrt(np.mean(emu ** 2)))
    bound = max(bound, 1e-6 * rms)
    rel_bound = max(rel_bound, 1e-6)
    rep = elementwise_report(got, emu, tw, f"{label} (bound {bound:.2e} = {bound / rms:.2e} RMS)")
    say(f"  {label}: rel-L2 vs emulated {rel_l2(got, emu):.2e} (bound {rel_bound:.2e})")
    assert rep["all"][0] <= bound, (label, rep["all"][0], bound, rep["worst_index"])
    assert rel_l2(got, emu) <= rel_bound, (label, rel_l2(got, emu), rel_bound)
    assert rep["tile_seams"][1] <= 3.0 * rep["interior"][1] + 1e-6 * rms, (label, rep["tile_seams"], rep["interior"])
    return emu
