"""Pins of the oracle's BF16 / e4m3 rounding (against torch's CPU casts) and its emulation modes."""
import numpy as np
import torch

from oracle import conet64 as o
from synth import ModelConfig, make_blob


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-6, 6, 20000),
                        # exact ties: lowest kept bit 0 and 1, dropped bits exactly half
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.0 + 2 ** -7])])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(o.round_bf16(v), ref)


def test_round_e4m3_matches_torch_in_range():
    rng = np.random.default_rng(1)
    v = rng.standard_normal(20000) * 10 ** rng.uniform(-4, 2.3, 20000)
    v = np.clip(v, -448, 448)
    ties = np.array([1.0 + 1 / 16, 1.0 + 3 / 16, 2 ** -9 * 1.5, 2 ** -9 * 2.5, 240.0 + 8.0])
    v = np.concatenate([v, ties, -ties])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(o.round_e4m3(v), ref)


def test_round_e4m3_saturates():
    np.testing.assert_array_equal(o.round_e4m3(np.array([449.0, 1e6, -500.0, 464.0])),
                                  np.array([448.0, 448.0, -448.0, 448.0]))


def test_emulation_modes_stay_close_to_fp64():
    cfg = ModelConfig(K=2, L=2, C=8, C_in=8, m=2)
    p = o.unpack(make_blob(cfg, seed=2, perturb=True), 2, 2, 8, 8, 2)
    X = np.random.default_rng(3).standard_normal((1, 14, 16, 8))
    ref = o.forward(p, X)
    bf = o.forward(p, X, quant=o.Quant("bf16"))
    rel = np.linalg.norm(bf - ref) / np.linalg.norm(ref)
    assert 1e-4 < rel < 3e-2          # rounding happened and stayed at BF16 scale
    sc = o.calibrate(p, X)
    f8 = o.forward(p, X, quant=o.Quant("fp8", sc))
    rel8 = np.linalg.norm(f8 - ref) / np.linalg.norm(ref)
    assert rel < rel8 < 0.25
