"""CPU trainer of CoNet weights for the BER experiments (test infrastructure only).

The BER comparisons between arithmetic precisions need a receiver that has learnt
something: with random weights the LLRs carry no information about the bits and a BER
curve is flat. The paper trains its networks on simulated link-level data with the same
dataset for every model (Sec. IV) but ships no weights, so this module trains them. It
produces an INPUT (a weight blob) shared by the FP64 oracle and the GPU library; no
parity claim rests on its own arithmetic, and it shares no code with the GPU library.

Like the rest of ``oracle/`` it is plain and CPU-only, but it runs in FP32 through
torch's CPU convolutions and autograd, because FP64 training is too slow to reach a
useful receiver in the time available. ``TorchConet`` can run in FP64, and the test
suite pins it there against ``conet64.forward`` and ``conet64.backward``.

The network is the one ``conet64.forward`` computes with its defaults (product fusion
after the blocks in ``fuse_mask``, per-RE LayerNorm, linear head): input layer 3x3 conv +
ReLU per branch; pre-activation residual blocks, the main net's block after a fusion
without its leading affine; product of the K block outputs, LayerNorm over C, fed to
the main net; 1x1 head. Loss: BCE-with-logits on the data bits (LLR = logit of b = 1),
averaged over slots, data REs and bits. Optimiser: Adam (beta 0.9 / 0.999, eps 1e-8)
with a cosine-decayed learning rate and gradient-norm clipping.
"""
from __future__ import annotations

import json
import math
import multiprocessing as mp
import os
import time
from typing import Dict, Optional

import numpy as np
import torch
import torch.nn.functional as Fn

from . import conet64 as o


def _ste(x: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
    """q in the forward, the identity's gradient in the backward (straight-through)."""
    return x + (q - x).detach()


def fq_e4m3(x: torch.Tensor, per_channel: bool = False) -> torch.Tensor:
    """Fake e4m3 quantisation of a conv operand (per tensor) or filter (per output channel):
    scale amax / 448, saturating round to nearest even onto e4m3, rescaled."""
    a = x.detach().abs()
    amax = a.flatten(1).amax(dim=1).view(-1, *([1] * (x.dim() - 1))) if per_channel else a.amax()
    s = torch.where(amax > 0, amax / o.E4M3_MAX, torch.ones_like(amax))
    q = (x / s).clamp(-o.E4M3_MAX, o.E4M3_MAX).to(torch.float8_e4m3fn).to(x.dtype) * s
    return _ste(x, q)


def fq_bf16(x: torch.Tensor) -> torch.Tensor:
    return _ste(x, x.to(torch.bfloat16).to(x.dtype))


class TorchConet(torch.nn.Module):
    """CoNet with its parameters held as torch tensors in the blob's structure.

    fake_quant="fp8": the forward applies the FP8 contract's roundings (conv operands per
    tensor and filters per output channel onto e4m3, stored block outputs to BF16) with
    straight-through gradients, for fine-tuning a network that will run in FP8 (activation
    scales here come from each batch; deployment calibrates static ones)."""

    def __init__(self, p: Dict, fuse_mask: Optional[int] = None, dtype=torch.float32, fake_quant: Optional[str] = None):
        super().__init__()
        self.fq = fake_quant
        self.K, self.L, self.C = p["K"], p["L"], p["C"]
        self.mask = ((1 << self.L) - 1) if fuse_mask is None else int(fuse_mask)
        P = lambda a: torch.nn.Parameter(torch.tensor(np.asarray(a), dtype=dtype))
        self.W_in = torch.nn.ParameterList([P(br["W_in"]) for br in p["branch"]])
        self.b_in = torch.nn.ParameterList([P(br["b_in"]) for br in p["branch"]])
        names = ("s0", "o0", "W1", "b1", "s1", "o1", "W2", "b2")
        self.blk = torch.nn.ParameterList(
            [P(p["branch"][k]["blocks"][l][n]) for k in range(self.K) for l in range(self.L) for n in names])
        self.gamma = torch.nn.ParameterList([P(g) for g in p["gamma"]])
        self.beta = torch.nn.ParameterList([P(b) for b in p["beta"]])
        self.W_h = P(p["W_h"])
        self.b_h = P(p["b_h"])
        self.meta = {k: p[k] for k in ("K", "L", "C", "C_in", "m")}

    def _b(self, k: int, l: int, n: str) -> torch.Tensor:
        i = ("s0", "o0", "W1", "b1", "s1", "o1", "W2", "b2").index(n)
        return self.blk[(k * self.L + l) * 8 + i]

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        """X: (B, T, F, C_in) -> LLR (B, T, F, m)."""
        ch = lambda v: v[None, :, None, None]
        fq = self.fq == "fp8"
        conv = (lambda z, W, bias: Fn.conv2d(fq_e4m3(z), fq_e4m3(W, True), bias, padding=1)) if fq else \
            (lambda z, W, bias: Fn.conv2d(z, W, bias, padding=1))
        st = fq_bf16 if fq else (lambda z: z)
        x = X.permute(0, 3, 1, 2)
        a = [st(torch.relu(conv(x, self.W_in[k], self.b_in[k]))) for k in range(self.K)]
        fused_prev = False
        for l in range(self.L):
            outs = []
            last = l == self.L - 1
            for k in range(self.K):
                b = lambda n: self._b(k, l, n)
                pre = torch.relu(a[k]) if (k == 0 and fused_prev) else torch.relu(ch(b("s0")) * a[k] + ch(b("o0")))
                h = torch.relu(ch(b("s1")) * conv(pre, b("W1"), b("b1")) + ch(b("o1")))
                outs.append(a[k] + conv(h, b("W2"), b("b2")))
            fused = bool((self.mask >> l) & 1)
            if fused:
                P = outs[0]
                for k in range(1, self.K):
                    P = P * st(outs[k])
                mu = P.mean(dim=1, keepdim=True)
                var = ((P - mu) ** 2).mean(dim=1, keepdim=True)
                A = ch(self.gamma[l]) * (P - mu) / torch.sqrt(var + o.LN_EPS) + ch(self.beta[l])
                a = [A if last else st(A)] + [st(v) for v in outs[1:]]
            else:
                a = [outs[0] if last else st(outs[0])] + [st(v) for v in outs[1:]]
            fused_prev = fused
        return torch.einsum("bctf,mc->btfm", a[0], self.W_h) + self.b_h

    def to_blob(self) -> np.ndarray:
        """The current parameters in blob order, FP32."""
        K, L = self.K, self.L
        t = lambda v: v.detach().double().numpy()
        p = {"branch": [], "gamma": [t(g) for g in self.gamma], "beta": [t(b) for b in self.beta],
             "W_h": t(self.W_h), "b_h": t(self.b_h), "norm": "ln"}
        for k in range(K):
            br = {"W_in": t(self.W_in[k]), "b_in": t(self.b_in[k]), "blocks": []}
            for l in range(L):
                br["blocks"].append({n: t(self._b(k, l, n)) for n in ("s0", "o0", "W1", "b1", "s1", "o1", "W2", "b2")})
            p["branch"].append(br)
        return o.pack(p).astype(np.float32)


def bce_loss(llr: torch.Tensor, bits: torch.Tensor, data_mask: torch.Tensor) -> torch.Tensor:
    """Mean BCE-with-logits over (slots, data REs, bits); pilots excluded."""
    per = Fn.binary_cross_entropy_with_logits(llr, bits, reduction="none")
    m = data_mask[None, :, :, None].expand_as(per)
    return per[m].mean()


# ----------------------------------------------------------------------------- data

_SIM = None


def _init_worker(sim_kwargs):
    global _SIM
    from synth import SimConfig
    _SIM = SimConfig(**sim_kwargs)
    torch.set_num_threads(1)


def _make_batch(args):
    from synth import simulate_slot
    first, n = args
    slots = [simulate_slot(_SIM, first + s) for s in range(n)]
    return np.stack([s.features for s in slots]), np.stack([s.bits for s in slots])


def train(p0: Dict, sim_kwargs: Dict, steps: int, batch: int, out_path: str, lr: float = 1e-3,
          lr_final: float = 1e-5, clip: float = 1.0, threads: int = 6, workers: int = 2,
          save_every: int = 200, log_every: int = 50, max_seconds: Optional[float] = None,
          first_slot: int = 0, fake_quant: Optional[str] = None) -> np.ndarray:
    """Train from parameters p0 (conet64.unpack form) on simulator batches.

    sim_kwargs: synth.SimConfig fields of the training data (its seed must differ from
    every evaluation seed). Step s reads slots first_slot + s*batch ... + batch - 1.
    Writes the blob to out_path (.npy, FP32) every save_every steps and at the end, and a
    log next to it (.json). Stops early after max_seconds of wall time.
    """
    torch.set_num_threads(threads)
    torch.manual_seed(0)
    net = TorchConet(p0, fake_quant=fake_quant)
    opt = torch.optim.Adam(net.parameters(), lr=lr, betas=(0.9, 0.999), eps=1e-8)
    from synth import data_mask as dmask
    T = sim_kwargs.get("T", 14)
    dm = torch.from_numpy(dmask(T, sim_kwargs["F"]))
    log = {"sim": sim_kwargs, "steps": steps, "batch": batch, "lr": lr, "lr_final": lr_final, "clip": clip,
           "first_slot": first_slot, "fake_quant": fake_quant, "loss": []}
    t0 = time.time()
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_init_worker, initargs=(sim_kwargs,)) as pool:
        # at most 2 batches per worker in flight: the simulator outruns the optimiser, and an
        # unbounded imap would queue every step's batch in memory
        ahead = 2 * workers
        pending = [pool.apply_async(_make_batch, ((first_slot + s * batch, batch),)) for s in range(min(ahead, steps))]
        run = 0.0
        step = 0
        while pending:
            X, bits = pending.pop(0).get()
            nxt = step + len(pending) + 1
            if nxt < steps:
                pending.append(pool.apply_async(_make_batch, ((first_slot + nxt * batch, batch),)))
            frac = step / max(1, steps - 1)
            if max_seconds is not None:  # decay over whichever budget runs out first
                frac = max(frac, (time.time() - t0) / max_seconds)
            frac = min(frac, 1.0)
            cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
            for gparam in opt.param_groups:
                gparam["lr"] = cur
            llr = net(torch.from_numpy(X))
            loss = bce_loss(llr, torch.from_numpy(bits).float(), dm)
            opt.zero_grad(set_to_none=True)
            loss.backward()
            torch.nn.utils.clip_grad_norm_(net.parameters(), clip)
            opt.step()
            run = loss.item() if step == 0 else 0.98 * run + 0.02 * loss.item()
            step += 1
            if step % log_every == 0 or step == steps:
                log["loss"].append([step, round(run, 5), round(time.time() - t0, 1)])
                print(f"step {step} loss {run:.4f} lr {cur:.2e} {time.time() - t0:.0f}s", flush=True)
            done = step == steps or (max_seconds is not None and time.time() - t0 > max_seconds)
            if step % save_every == 0 or done:
                np.save(out_path + ".tmp.npy", net.to_blob())
                os.replace(out_path + ".tmp.npy", out_path)
                log["steps_done"] = step
                with open(os.path.splitext(out_path)[0] + ".json", "w") as f:
                    json.dump(log, f, indent=1)
            if done:
                pool.terminate()
                break
    return net.to_blob()
