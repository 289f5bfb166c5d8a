"""Seeded CoNet weight blobs (the packed FP32 parameter vector crossing the C ABI).

Blob order (little-endian FP32, fixed; the C header states the same order):
  for each branch k = 0..K-1 (k = 0 is the main net):
      W_in  (C, C_in, 3, 3)  input conv, OIHW with H = OFDM symbol, W = subcarrier
      b_in  (C,)
      for each block l = 1..L:
          s0, o0 (C,)  leading pre-activation affine (ignored where the block is an MRB)
          W1 (C, C, 3, 3), b1 (C,)
          s1, o1 (C,)  middle pre-activation affine
          W2 (C, C, 3, 3), b2 (C,)
  for each block l = 1..L: gamma_l, beta_l (C,)   norm after the product fusion
  W_h (m, C), b_h (m,)                            1x1 LLR head
Variants: support branches may have fewer blocks (support_blocks); depthwise-separable
blocks replace each W (C, C, 3, 3) by D (C, 3, 3) then P (C, C); fusion by concatenation
appends Wc_l (C, K C), bc_l (C,) for l = 1..L after the head.

Draws are random numbers the method consumes, so they are made here and passed to
both the oracle and the GPU library. The default is the He-normal initialisation:
every conv and the head draw N(0, 2/fan_in) (fan_in = C_in_layer * 9, or C for the
head), biases are 0 and every affine is the identity. ``perturb=True`` additionally
draws non-trivial biases, affines and norm parameters so that parity tests exercise
every parameter.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np


@dataclass(frozen=True)
class ModelConfig:
    K: int                 # branches (k = 0 main, 1..K-1 support)
    L: int                 # residual blocks per branch
    C: int                 # channels
    C_in: int              # input channels = 4 N_rx
    m: int                 # head width (bits per symbol)
    fuse_mask: int = -1    # bit l-1 => fusion after block l; -1 => all blocks
    support_blocks: int = 0  # blocks of each support branch (0 => L)
    fusion: str = "product"  # "concat" adds the projection Wc_l (C, K C), bc_l (C) per block
    block: str = "standard"  # "ds": depthwise-separable convs (D (C,3,3) then P (C,C))

    @property
    def mask(self) -> int:
        if self.fuse_mask >= 0:
            return int(self.fuse_mask)
        return (1 << (self.L if self.support_blocks <= 0 else self.support_blocks)) - 1

    @property
    def Ls(self) -> int:
        return self.L if self.support_blocks <= 0 else self.support_blocks


def blob_layout(cfg: ModelConfig) -> List[Tuple[str, Tuple[int, ...]]]:
    K, L, C, Ci, m = cfg.K, cfg.L, cfg.C, cfg.C_in, cfg.m
    out: List[Tuple[str, Tuple[int, ...]]] = []
    for k in range(K):
        out.append((f"b{k}.W_in", (C, Ci, 3, 3)))
        out.append((f"b{k}.b_in", (C,)))
        for l in range(1, (L if k == 0 else cfg.Ls) + 1):
            p = f"b{k}.l{l}."
            if cfg.block == "ds":
                c1 = [(p + "D1", (C, 3, 3)), (p + "P1", (C, C))]
                c2 = [(p + "D2", (C, 3, 3)), (p + "P2", (C, C))]
            else:
                c1, c2 = [(p + "W1", (C, C, 3, 3))], [(p + "W2", (C, C, 3, 3))]
            out += [(p + "s0", (C,)), (p + "o0", (C,))] + c1 + [(p + "b1", (C,)), (p + "s1", (C,)), (p + "o1", (C,))] \
                + c2 + [(p + "b2", (C,))]
    for l in range(1, L + 1):
        out += [(f"l{l}.gamma", (C,)), (f"l{l}.beta", (C,))]
    out += [("W_h", (m, C)), ("b_h", (m,))]
    if cfg.fusion == "concat":
        for l in range(1, L + 1):
            out += [(f"l{l}.Wc", (C, K * C)), (f"l{l}.bc", (C,))]
    return out


def blob_size(cfg: ModelConfig) -> int:
    return int(sum(int(np.prod(s)) for _, s in blob_layout(cfg)))


def make_blob(cfg: ModelConfig, seed: int = 0, perturb: bool = False, scale: float = 1.0) -> np.ndarray:
    """Draw a weight blob in blob order from SeedSequence([seed])."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed)])))
    parts = []
    for name, shape in blob_layout(cfg):
        leaf = name.split(".")[-1]
        n = int(np.prod(shape))
        if leaf in ("W_in", "W1", "W2"):
            fan_in = shape[1] * 9
            v = rng.standard_normal(n) * np.sqrt(2.0 / fan_in) * scale
        elif leaf in ("D1", "D2"):  # depthwise: fan-in 9
            v = rng.standard_normal(n) * np.sqrt(2.0 / 9) * scale
        elif leaf in ("P1", "P2", "Wc"):  # 1x1 convs: fan-in = input channels
            v = rng.standard_normal(n) * np.sqrt(2.0 / shape[1]) * scale
        elif leaf == "W_h":
            v = rng.standard_normal(n) * np.sqrt(2.0 / shape[1])
        elif leaf in ("s0", "s1", "gamma"):
            v = rng.uniform(0.6, 1.4, n) if perturb else np.ones(n)
        else:  # biases, o0, o1, beta
            v = rng.standard_normal(n) * 0.1 if perturb else np.zeros(n)
        parts.append(v)
    return np.concatenate(parts).astype(np.float32)


def split_blob(cfg: ModelConfig, blob: np.ndarray) -> Dict[str, np.ndarray]:
    """Named views of a blob (used by tests to plant values; the oracle parses on its own)."""
    out, off = {}, 0
    for name, shape in blob_layout(cfg):
        n = int(np.prod(shape))
        out[name] = blob[off:off + n].reshape(shape)
        off += n
    assert off == blob.size
    return out
