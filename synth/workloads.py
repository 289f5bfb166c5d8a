"""The six named workloads: grid, antennas, modulation, channel, model and seeds."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

from .ofdm import SimConfig
from .weights import ModelConfig


@dataclass(frozen=True)
class Workload:
    name: str
    batch: int
    sim: SimConfig
    model: ModelConfig
    dtype: str            # conv arithmetic: "f32", "bf16", "fp8"
    weight_seed: int = 0


WORKLOADS = {
    # Plain FP32 forward of one slot: 72 x 14 grid, 2 rx, QPSK, 4-tap block-fading channel.
    "fp32_b1_f72": Workload("fp32_b1_f72", 1,
                            SimConfig(F=72, n_rx=2, bits_per_symbol=2, n_taps=4, max_doppler_hz=0.0,
                                      snr_db=10.0, seed=1),
                            ModelConfig(K=2, L=2, C=32, C_in=8, m=2), "f32"),
    # BF16 batched inference: 64 slots of 3276 x 14, 4 rx, 16-QAM, K=3 L=4 C=64.
    "bf16_b64_f3276": Workload("bf16_b64_f3276", 64,
                               SimConfig(F=3276, n_rx=4, bits_per_symbol=4, n_taps=8, max_doppler_hz=400.0,
                                         seed=2),
                               ModelConfig(K=3, L=4, C=64, C_in=16, m=4), "bf16"),
    # FP8 e4m3 inference: 128 slots of 3276 x 14, 8 rx, 256-QAM, K=4 L=6 C=96.
    "fp8_b128_f3276": Workload("fp8_b128_f3276", 128,
                               SimConfig(F=3276, n_rx=8, bits_per_symbol=8, n_taps=8, max_doppler_hz=400.0,
                                         seed=3),
                               ModelConfig(K=4, L=6, C=96, C_in=32, m=8), "fp8"),
    # Training step: 128 slots of 1024 x 14, 4 rx, 16-QAM, K=3 L=4 C=64.
    "train_b128_f1024": Workload("train_b128_f1024", 128,
                                 SimConfig(F=1024, n_rx=4, bits_per_symbol=4, n_taps=8, max_doppler_hz=400.0,
                                           seed=4),
                                 ModelConfig(K=3, L=4, C=64, C_in=16, m=4), "bf16"),
    # Interference-limited uplink (Sec. IV): 64 slots of 3276 x 14, 4 rx, 64-QAM; an interferer
    # holds 10-90 % of the noise-plus-interference power, and its variance and the noise's
    # feed 8 more input channels (C_in = 16 + 8). K=3 L=4 C=64.
    "interf_bf16_b64_f3276": Workload("interf_bf16_b64_f3276", 64,
                                      SimConfig(F=3276, n_rx=4, bits_per_symbol=6, n_taps=8, max_doppler_hz=400.0,
                                                seed=6, interference_share=(0.1, 0.9), variance_channels=True),
                                      ModelConfig(K=3, L=4, C=64, C_in=24, m=6), "bf16"),
    # Serving trunk: K=3 L=4 C=64, inputs padded to 16 channels, head width 6.
    "serve_bf16": Workload("serve_bf16", 1,
                           SimConfig(F=3276, n_rx=4, bits_per_symbol=6, n_taps=8, max_doppler_hz=400.0,
                                     seed=5),
                           ModelConfig(K=3, L=4, C=64, C_in=16, m=6), "bf16"),
}


def workload(name: str, F: Optional[int] = None, batch: Optional[int] = None) -> Workload:
    """A named workload, optionally with a smaller grid or batch for tests."""
    w = WORKLOADS[name]
    if F is None and batch is None:
        return w
    sim = w.sim if F is None else SimConfig(**{**w.sim.__dict__, "F": F})
    return Workload(w.name, w.batch if batch is None else batch, sim, w.model, w.dtype, w.weight_seed)
