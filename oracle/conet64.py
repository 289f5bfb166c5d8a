"""FP64 CPU oracle of the CoNet-Rx receiver network (test infrastructure only).

Plain, slow and meant to be read against the paper. Nothing in the product path may
import it: only tests, the smoke check and the bench's CPU-baseline leg do.

What it computes (paper Sec. II-A and Sec. III):
  * input layer of every branch: 3x3 conv + ReLU (Sec. III describes the input layers
    as convolutions with ReLU activations);
  * residual blocks in the pre-activation form of He et al. (Sec. II-A, Fig. 1):
    affine -> ReLU -> conv -> affine -> ReLU -> conv, plus the identity shortcut;
    the affine stands in for inference-form BN;
  * the modified block (MRB, Sec. III, Fig. 3): the main-net block that follows a
    fusion drops its leading normalisation, since its input is already normalised;
  * element-wise product of the branch block outputs, followed by a per-RE channel
    LayerNorm (Sec. III allows BN or LN after each product), fed to the main net;
    with M support nets the product runs over all K = M+1 outputs (Sec. III, the
    generalisation to more than two nets);
  * 1x1 output conv with one filter per bit of the symbol (Sec. III) -> LLRs.

Variants the paper also describes (Sec. III): fusion by addition instead of the
product (``fusion="sum"``: P = sum_k O[k], then the same LayerNorm), and Example II's
feedback from the main net to the support nets (``feedback=True``: after a fusion, each
support net continues from its own block output plus the main net's fused activation).
The normalisation after the fusion may be BatchNorm instead of LayerNorm (the paper
allows either): ``norm="bn"`` applies gamma (P - mean) / sqrt(var + eps) + beta per
channel with running statistics stored in the blob (``unpack(..., norm="bn")``), and
``norm="bn_batch"`` uses the batch's own per-channel statistics over every RE (biased
variance, as BN does while training), which is how running statistics are produced.

Readings of what the paper leaves open (all listed in the design notes): conv
biases everywhere; "same" zero padding inside each slot; LN over the C channels of
each RE with eps = 1e-5 and affine (gamma, beta); the head is linear with bias and
reads the last main-net activation; LLR = ln P(b=1)/P(b=0).

Optional precision emulation (``quant``), the reduced-precision contract written from
what the configurations fix (conv arithmetic in BF16 or FP8 e4m3 with per-output-channel
scales, FP32 accumulation) plus one rule for what is stored:
  * every conv operand is rounded: filters and input activations to BF16 ("bf16"), or to
    e4m3 of value / scale ("fp8": filter scale amax/448 per output channel, a static
    activation scale per conv input, saturating round-to-nearest-even);
  * a tensor that leaves a residual block -- the input layer's output, a block output
    that a net carries on (or that a support net hands to the fusion), the fused
    activation -- is stored in BF16 on both paths; a main-net output consumed by its own
    block's fusion, and the last activation feeding the head, are not;
  * everything else (accumulation, biases, affines, ReLU, residual adds, the fusion, the
    normalisation, the head) is exact here and FP32 on the GPU.
The pins construct this contract independently with torch's casts.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

LN_EPS = 1e-5


# ----------------------------------------------------------------------------- params

def unpack(blob: np.ndarray, K: int, L: int, C: int, C_in: int, m: int, norm: str = "ln",
           support_blocks: int = 0, fusion: str = "product", block: str = "standard") -> Dict:
    """Parse the packed FP32 parameter vector into FP64 arrays (blob order of the C header).
    support_blocks: blocks of each support net (0: L; Sec. III lets the support net be
    shallower). fusion="concat": after the head, per block l the projection Wc_l (C, K C),
    bc_l (C) of the concatenated branch outputs. norm="bn": the blob ends with the BatchNorm
    running mean and variance of every block. block="ds": depthwise-separable blocks (Sec. II-A), each
    conv a depthwise 3x3 filter D (C, 3, 3) followed by a 1x1 conv P (C, C) with bias."""
    v = np.asarray(blob, dtype=np.float64).ravel()
    pos = [0]

    def take(*shape):
        n = int(np.prod(shape))
        out = v[pos[0]:pos[0] + n].reshape(shape)
        pos[0] += n
        return out

    Ls = L if support_blocks in (0, None) else int(support_blocks)
    if not 1 <= Ls <= L:
        raise ValueError(f"support_blocks must be 1..L (got {support_blocks})")
    if block not in ("standard", "ds"):
        raise ValueError(f"unknown block {block!r}")
    if fusion not in ("product", "sum", "concat"):
        raise ValueError(f"unknown fusion {fusion!r}")
    p = {"K": K, "L": L, "C": C, "C_in": C_in, "m": m, "branch": [], "Ls": Ls, "block": block}
    for k in range(K):
        br = {"W_in": take(C, C_in, 3, 3), "b_in": take(C), "blocks": []}
        for _l in range(L if k == 0 else Ls):
            blk = {}
            blk["s0"] = take(C); blk["o0"] = take(C)
            if block == "ds":
                blk["D1"] = take(C, 3, 3); blk["P1"] = take(C, C)
            else:
                blk["W1"] = take(C, C, 3, 3)
            blk["b1"] = take(C)
            blk["s1"] = take(C); blk["o1"] = take(C)
            if block == "ds":
                blk["D2"] = take(C, 3, 3); blk["P2"] = take(C, C)
            else:
                blk["W2"] = take(C, C, 3, 3)
            blk["b2"] = take(C)
            br["blocks"].append(blk)
        p["branch"].append(br)
    p["gamma"] = []
    p["beta"] = []
    for _l in range(L):
        p["gamma"].append(take(C))
        p["beta"].append(take(C))
    p["W_h"] = take(m, C)
    p["b_h"] = take(m)
    if fusion == "concat":
        p["Wc"], p["bc"] = [], []
        for _l in range(L):
            p["Wc"].append(take(C, K * C))
            p["bc"].append(take(C))
    p["fusion"] = fusion
    p["norm"] = norm
    if norm == "bn":
        p["bn_mean"], p["bn_var"] = [], []
        for _l in range(L):
            p["bn_mean"].append(take(C))
            p["bn_var"].append(take(C))
    elif norm != "ln":
        raise ValueError(f"unknown norm {norm!r}")
    if pos[0] != v.size:
        raise ValueError(f"blob has {v.size} values, layout needs {pos[0]}")
    return p


def pack(p: Dict) -> np.ndarray:
    """Inverse of unpack (gradients are returned in blob order)."""
    parts = []
    keys = ("s0", "o0", "D1", "P1", "b1", "s1", "o1", "D2", "P2", "b2") if p.get("block") == "ds" else \
        ("s0", "o0", "W1", "b1", "s1", "o1", "W2", "b2")
    for br in p["branch"]:
        parts += [br["W_in"], br["b_in"]]
        for blk in br["blocks"]:
            parts += [blk[k] for k in keys]
    for g, b in zip(p["gamma"], p["beta"]):
        parts += [g, b]
    parts += [p["W_h"], p["b_h"]]
    if p.get("fusion") == "concat":
        for W, b in zip(p["Wc"], p["bc"]):
            parts += [W, b]
    if p.get("norm", "ln") == "bn":
        for mu, var in zip(p["bn_mean"], p["bn_var"]):
            parts += [mu, var]
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts])


# ----------------------------------------------------------------------------- rounding

def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even) via FP32, returned as FP64.

    BF16 keeps the top 16 bits of an FP32 word; the rounding adds 0x7FFF plus the
    lowest kept bit before truncating, which is round-half-to-even on the dropped bits.
    """
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


E4M3_MAX = 448.0


def round_e4m3(a: np.ndarray) -> np.ndarray:
    """Saturating round-to-nearest-even onto the OCP e4m3fn grid (max 448, subnormals).

    Normal numbers 2^e (1 + j/8), e in [-6, 8]; subnormals j 2^-9. The value is
    clamped to +-448 and then rounded on the quantum of its binade.
    """
    x = np.clip(np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64), -E4M3_MAX, E4M3_MAX)
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.maximum(e, -6.0)
    q = np.exp2(e - 3.0)
    return np.sign(x) * np.round(ax / q) * q


# ----------------------------------------------------------------------------- conv

def conv3x3(x: np.ndarray, W: np.ndarray, b: Optional[np.ndarray] = None) -> np.ndarray:
    """3x3 cross-correlation with zero "same" padding inside each slot.

    x: (B, T, F, Ci); W: (Co, Ci, 3, 3) with axes (out, in, symbol offset, subcarrier offset).
    out[b,t,f,o] = bias[o] + sum_{i,dt,df} W[o,i,dt+1,df+1] x[b,t+dt,f+df,i],
    x read as 0 outside [0,T) x [0,F) of its own slot. Computed by im2col + matmul.
    """
    B, T, F, Ci = x.shape
    Co = W.shape[0]
    xp = np.zeros((B, T + 2, F + 2, Ci), dtype=np.float64)
    xp[:, 1:-1, 1:-1, :] = x
    cols = np.empty((B, T, F, 3, 3, Ci), dtype=np.float64)
    for a in range(3):
        for c in range(3):
            cols[:, :, :, a, c, :] = xp[:, a:a + T, c:c + F, :]
    Wm = W.transpose(2, 3, 1, 0).reshape(9 * Ci, Co)
    out = cols.reshape(B * T * F, 9 * Ci) @ Wm
    if b is not None:
        out += b[None, :]
    return out.reshape(B, T, F, Co)


def conv3x3_bruteforce(x: np.ndarray, W: np.ndarray, b: Optional[np.ndarray] = None) -> np.ndarray:
    """The same operation written as nested loops (tiny grids only; pins conv3x3)."""
    B, T, F, Ci = x.shape
    Co = W.shape[0]
    out = np.zeros((B, T, F, Co))
    for bb in range(B):
        for t in range(T):
            for f in range(F):
                for o in range(Co):
                    s = 0.0 if b is None else float(b[o])
                    for i in range(Ci):
                        for dt in (-1, 0, 1):
                            for df in (-1, 0, 1):
                                tt, ff = t + dt, f + df
                                if 0 <= tt < T and 0 <= ff < F:
                                    s += W[o, i, dt + 1, df + 1] * x[bb, tt, ff, i]
                    out[bb, t, f, o] = s
    return out


def dwconv3x3(x: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Depthwise 3x3 cross-correlation (each channel filtered by its own 3x3 filter), zero
    "same" padding inside each slot: out[b,t,f,c] = sum_{dt,df} D[c,dt+1,df+1] x[b,t+dt,f+df,c].
    x: (B, T, F, C); D: (C, 3, 3)."""
    B, T, F, C = x.shape
    xp = np.zeros((B, T + 2, F + 2, C), dtype=np.float64)
    xp[:, 1:-1, 1:-1, :] = x
    out = np.zeros((B, T, F, C), dtype=np.float64)
    for a in range(3):
        for c in range(3):
            out += D[:, a, c][None, None, None, :] * xp[:, a:a + T, c:c + F, :]
    return out


def conv3x3_input_grad(dout: np.ndarray, W: np.ndarray) -> np.ndarray:
    """d/dx of conv3x3: correlation of dout with the flipped, channel-transposed filter."""
    Wt = W[:, :, ::-1, ::-1].transpose(1, 0, 2, 3)
    return conv3x3(dout, np.ascontiguousarray(Wt))


def conv3x3_weight_grad(x: np.ndarray, dout: np.ndarray) -> np.ndarray:
    """dW[o,i,a,c] = sum_{b,t,f} dout[b,t,f,o] x[b,t+a-1,f+c-1,i] (zero outside the slot)."""
    B, T, F, Ci = x.shape
    Co = dout.shape[-1]
    xp = np.zeros((B, T + 2, F + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    dW = np.empty((Co, Ci, 3, 3))
    d2 = dout.reshape(-1, Co)
    for a in range(3):
        for c in range(3):
            dW[:, :, a, c] = d2.T @ xp[:, a:a + T, c:c + F, :].reshape(-1, Ci)
    return dW


def relu(z):
    return np.maximum(z, 0.0)


# ----------------------------------------------------------------------------- forward

def fused_after(fuse_mask: int, l: int) -> bool:
    """True if the product fusion follows block l (1-based)."""
    return bool((fuse_mask >> (l - 1)) & 1)


FP32_UNIT = 2.0 ** -24


@dataclass
class Quant:
    """Precision emulation. kind: None, "bf16" or "fp8"; act_scales for fp8 (see act_scale_index).
    noise: set by forward(acc_noise=...) for the FP32 error model (see _fp32_formed)."""
    kind: Optional[str] = None
    act_scales: Optional[np.ndarray] = None
    noise: Optional[np.random.Generator] = None

    def store(self, a):
        """Rounding of an activation tensor that leaves a residual block (BF16 on both paths)."""
        return a if self.kind is None else round_bf16(_fp32_formed(self, a))


# FP32 operations that form a value before it is rounded to BF16 or e4m3 (bias, affine, ReLU,
# residual add, product, scale); each contributes a relative rounding error of at most 2^-24.
FP32_OPS_BEFORE_ROUNDING = 6


def _fp32_formed(q: "Quant", a: np.ndarray) -> np.ndarray:
    """With q.noise: a as an FP32 implementation may have formed it, each element carrying the
    relative rounding error of FP32_OPS_BEFORE_ROUNDING independent FP32 operations. Such errors
    decide the reduced-precision rounding of values that lie next to a rounding boundary; used
    for tolerances only (forward's acc_noise), never for results."""
    if q.noise is None:
        return a
    return a * (1.0 + FP32_UNIT * np.sqrt(FP32_OPS_BEFORE_ROUNDING) * q.noise.standard_normal(np.shape(a)))


def act_scale_index(K: int, L: int, k: int, l: int, which: int) -> int:
    """Index of a conv's input scale: 0 = input layer; then per (k, l): 1 + 2(kL + l-1) + which."""
    if l == 0:
        return 0
    return 1 + 2 * (k * L + (l - 1)) + which


def _operand(q: Quant, a: np.ndarray, idx: int) -> np.ndarray:
    if q.kind is None:
        return a
    a = _fp32_formed(q, a)
    if q.kind == "bf16":
        return round_bf16(a)
    s = float(q.act_scales[idx])
    return round_e4m3(a / s) * s


def _weights(q: Quant, W: np.ndarray) -> np.ndarray:
    if q.kind is None:
        return W
    if q.kind == "bf16":
        return round_bf16(W)
    Wf = W.astype(np.float32).astype(np.float64)
    amax = np.abs(Wf).reshape(Wf.shape[0], -1).max(axis=1)
    s = np.where(amax > 0, (amax / E4M3_MAX).astype(np.float32).astype(np.float64), 1.0)
    return round_e4m3(Wf / s[:, None, None, None]) * s[:, None, None, None]


# Fractional bits kept, relative to the largest product of its group of 8, by the FP8 matrix
# instructions when they sum the products of one group (the MI355X's 16x16x128 and 32x32x64
# e4m3 MFMAs, measured with in-bounds probes of the instructions: a product 2^-13 of the
# group's largest is kept whole, 2^-14 is dropped; products in other groups, and BF16 products,
# are kept down to FP32 resolution).
FP8_MFMA_GROUP_BITS = 13


def _conv_acc(xq: np.ndarray, Wq: np.ndarray, b: Optional[np.ndarray], noise, fp8: bool = False) -> np.ndarray:
    """conv3x3 of an operand; with `noise` (a numpy Generator), plus a model of the error a
    GPU accumulation of the same sum makes.

    Model: summing N terms in FP32, each partial sum carries a relative rounding error of at
    most 2^-24; treated as independent, the errors add up to a standard deviation of about
    2^-24 sqrt(N / 2) sqrt(sum_i term_i^2) (term_i = w_i x_i, N = 9 C_in). With fp8, the matrix
    instruction also truncates each product of a group of 8 to FP8_MFMA_GROUP_BITS fractional
    bits of the group's largest product (toward zero): per product an error of up to one such
    unit u, biased half a unit, about u sqrt(7/3) per group; with u about 0.7 2^-13 times the
    group's largest product and that about twice the typical product, the sum carries about
    0.75 2^-13 sqrt(sum_i term_i^2), taken here as 2^-13 sqrt(sum_i term_i^2). Used to bound
    how far a GPU implementation may lie from this FP64 one, never as a result.
    """
    c = conv3x3(xq, Wq, b)
    if noise is not None:
        n_terms = 9 * xq.shape[-1]
        sq = np.sqrt(np.maximum(conv3x3(xq * xq, Wq * Wq), 0.0))
        sd = FP32_UNIT * np.sqrt(n_terms / 2.0) * sq
        if fp8:
            sd = np.sqrt(sd * sd + (2.0 ** -FP8_MFMA_GROUP_BITS * sq) ** 2)
        c = c + sd * noise.standard_normal(c.shape)
    return c


def _ds_conv_acc(q: "Quant", xq: np.ndarray, D: np.ndarray, P: np.ndarray, b: np.ndarray, noise) -> np.ndarray:
    """Depthwise-separable conv (Sec. II-A): the depthwise 3x3 filter D, then the 1x1 conv P
    with bias b, on an operand xq already rounded. The depthwise output is the 1x1 conv's
    operand and is rounded as one; filters are rounded as conv operands. With `noise`, each
    sum carries _conv_acc's FP32-accumulation error model (9 terms, then C terms)."""
    Dq = D if q.kind is None else round_bf16(D)
    Pq = P if q.kind is None else round_bf16(P)
    d = dwconv3x3(xq, Dq)
    if noise is not None:
        sq = np.sqrt(np.maximum(dwconv3x3(xq * xq, Dq * Dq), 0.0))
        d = d + FP32_UNIT * np.sqrt(9 / 2.0) * sq * noise.standard_normal(d.shape)
    dq = d if q.kind is None else round_bf16(_fp32_formed(q, d))
    c = dq @ Pq.T + b
    if noise is not None:
        sq = np.sqrt(np.maximum((dq * dq) @ (Pq * Pq).T, 0.0))
        c = c + FP32_UNIT * np.sqrt(P.shape[1] / 2.0) * sq * noise.standard_normal(c.shape)
    return c


def forward(p: Dict, X: np.ndarray, fuse_mask: Optional[int] = None, quant: Optional[Quant] = None,
            keep: bool = False, calib: Optional[np.ndarray] = None, fusion: Optional[str] = None,
            feedback: bool = False, norm: Optional[str] = None, bn_stats: Optional[Dict] = None,
            acc_noise: Optional[np.random.Generator] = None):
    """CoNet forward for a batch X (B, T, F, C_in) -> LLR (B, T, F, m).

    keep=True also returns the intermediate tensors the backward needs.
    calib, if given, receives the running max |.| of every conv input operand
    (indexing of act_scale_index), which is how static activation scales are set.
    fusion: "product" (Example I), "sum" (fusion by addition) or "concat" (fusion by
    concatenation: the K outputs side by side, projected back to C channels by p's 1x1 conv
    Wc_l, bc_l); default: p's own. feedback: Example II's main -> support feedback after every
    fusion. Support nets shallower than the main net (p["Ls"] < L) take part in the fusions
    after their own blocks only. norm: "ln", "bn" (running statistics of
    p) or "bn_batch" (this batch's statistics, recorded into bn_stats[l - 1] = (mean, var)
    if given); default: p's own. The backward covers product fusion without feedback, standard
    blocks of full depth, with "ln" or "bn_batch".
    acc_noise: a numpy Generator; every conv and the head then carry the FP32-accumulation
    error model of _conv_acc, and every value rounded to BF16 or e4m3 the FP32 error of the
    operations that formed it (_fp32_formed); for deriving tolerances, never for results.
    """
    fusion = fusion or p.get("fusion", "product")
    if fusion not in ("product", "sum", "concat"):
        raise ValueError(f"unknown fusion {fusion!r}")
    if fusion == "concat" and "Wc" not in p:
        raise ValueError("fusion by concatenation needs the projection weights (unpack(..., fusion='concat'))")
    ds = p.get("block", "standard") == "ds"
    norm = norm or p.get("norm", "ln")
    if norm not in ("ln", "bn", "bn_batch"):
        raise ValueError(f"unknown norm {norm!r}")
    K, L = p["K"], p["L"]
    Ls = p.get("Ls", L)
    mask = ((1 << L) - 1) if fuse_mask is None else int(fuse_mask)
    if mask >> Ls:
        raise ValueError(f"fusion after block {mask.bit_length()} but the support nets have {Ls} blocks")
    q = quant or Quant()
    if q.kind == "fp8" and (ds or fusion == "concat"):
        raise ValueError("the FP8 contract covers standard blocks with product or sum fusion")
    if acc_noise is not None and q.kind is not None:  # the error model also perturbs rounding inputs
        q = Quant(q.kind, q.act_scales, noise=acc_noise)
    X = np.asarray(X, dtype=np.float64)
    cache = {"X": X, "mask": mask, "a0": [], "levels": []}

    if calib is not None:
        calib[0] = max(calib[0], float(np.abs(X).max()))
    Xq = _operand(q, X, 0)
    a = []
    for k in range(K):
        br = p["branch"][k]
        z = _conv_acc(Xq, _weights(q, br["W_in"]), br["b_in"], acc_noise, q.kind == "fp8")
        a.append(q.store(relu(z)))
    cache["a0"] = [t.copy() for t in a] if keep else None

    fused_prev = False
    for l in range(1, L + 1):
        lev = {"x": a, "pre": [], "c1": [], "z1": [], "h": [], "O": [], "mrb": []}
        O = []
        Kl = K if l <= Ls else 1  # branches that have block l
        for k in range(Kl):
            blk = p["branch"][k]["blocks"][l - 1]
            x = a[k]
            mrb = (k == 0 and fused_prev)
            pre = relu(x) if mrb else relu(blk["s0"] * x + blk["o0"])
            if calib is not None:
                i0 = act_scale_index(K, L, k, l, 0)
                calib[i0] = max(calib[i0], float(np.abs(pre).max()))
            if ds:
                c1 = _ds_conv_acc(q, _operand(q, pre, 0), blk["D1"], blk["P1"], blk["b1"], acc_noise)
            else:
                c1 = _conv_acc(_operand(q, pre, act_scale_index(K, L, k, l, 0)), _weights(q, blk["W1"]), blk["b1"],
                               acc_noise, q.kind == "fp8")
            z1 = blk["s1"] * c1 + blk["o1"]
            h = q.store(relu(z1)) if q.kind is None or q.kind == "bf16" else relu(z1)
            if calib is not None:
                i1 = act_scale_index(K, L, k, l, 1)
                calib[i1] = max(calib[i1], float(np.abs(h).max()))
            if ds:
                c2 = _ds_conv_acc(q, _operand(q, h, 0), blk["D2"], blk["P2"], blk["b2"], acc_noise)
            else:
                c2 = _conv_acc(_operand(q, h, act_scale_index(K, L, k, l, 1)), _weights(q, blk["W2"]), blk["b2"],
                               acc_noise, q.kind == "fp8")
            Ok = x + c2
            O.append(Ok)
            if keep:
                lev["pre"].append(pre); lev["c1"].append(c1); lev["z1"].append(z1)
                lev["h"].append(h); lev["mrb"].append(mrb)
        last = (l == L)
        if fused_after(mask, l):
            # the support outputs enter the fusion as stored (rounded under emulation)
            if fusion == "concat":  # a 1x1 conv over the K outputs side by side: conv operands
                cat = np.concatenate([_operand(q, O[0], 0)] + [q.store(O[k]) for k in range(1, K)], axis=-1)
                Wq = _weights(q, p["Wc"][l - 1][:, :, None, None])[:, :, 0, 0]
                P = cat @ Wq.T + p["bc"][l - 1]
                if acc_noise is not None:
                    sq = np.sqrt(np.maximum((cat * cat) @ (Wq * Wq).T, 0.0))
                    P = P + FP32_UNIT * np.sqrt(K * p["C"] / 2.0) * sq * acc_noise.standard_normal(P.shape)
            else:
                P = O[0].copy()
                for k in range(1, K):
                    P = P + q.store(O[k]) if fusion == "sum" else P * q.store(O[k])
            if norm == "ln":  # over the C channels of each RE
                mu = P.mean(axis=-1, keepdims=True)
                var = ((P - mu) ** 2).mean(axis=-1, keepdims=True)
            elif norm == "bn":  # per channel, running statistics
                mu, var = p["bn_mean"][l - 1], p["bn_var"][l - 1]
            else:  # per channel over every RE of the batch, biased variance
                mu = P.mean(axis=(0, 1, 2))
                var = ((P - mu) ** 2).mean(axis=(0, 1, 2))
                if bn_stats is not None:
                    bn_stats[l - 1] = (mu.copy(), var.copy())
            sig = np.sqrt(var + LN_EPS)
            ahat = (P - mu) / sig
            A0 = p["gamma"][l - 1] * ahat + p["beta"][l - 1]
            if feedback:  # Example II: each support continues from O[k] + the main net's A
                new = [A0 if last else q.store(A0)] + [q.store(q.store(O[k]) + A0) for k in range(1, K)]
            else:
                new = [A0 if last else q.store(A0)] + [q.store(O[k]) for k in range(1, K)]
            if keep:
                lev["P"] = P; lev["ahat"] = ahat; lev["sig"] = sig
        else:
            new = [O[0] if last else q.store(O[0])] + [q.store(O[k]) for k in range(1, Kl)]
        if keep:
            lev["O"] = O
            cache["levels"].append(lev)
        a = new
        fused_prev = fused_after(mask, l)

    llr = a[0] @ p["W_h"].T + p["b_h"]
    if acc_noise is not None:  # the head's C-term sums, same error model
        sq = (a[0] * a[0]) @ (p["W_h"] * p["W_h"]).T
        llr = llr + FP32_UNIT * np.sqrt(p["C"] / 2.0) * np.sqrt(sq) * acc_noise.standard_normal(llr.shape)
    if keep:
        cache["aL"] = a[0]
        cache["variant"] = (fusion, feedback, norm) + (() if (Ls == L and not ds) else (Ls, ds))
        return llr, cache
    return llr


def forward_slots(p: Dict, X: np.ndarray, **kw) -> np.ndarray:
    """forward() one slot at a time (bounds host memory on wide grids)."""
    return np.concatenate([forward(p, X[b:b + 1], **kw) for b in range(X.shape[0])], axis=0)


# ----------------------------------------------------------------------------- loss

def bce_with_logits(llr: np.ndarray, bits: np.ndarray, data_mask: np.ndarray) -> Tuple[float, np.ndarray]:
    """Mean bitwise BCE over data REs and returns d loss / d LLR.

    loss = mean over (slot, data RE, bit) of max(z,0) - z b + log(1 + e^{-|z|});
    the gradient is (sigmoid(z) - b) / count on data REs and 0 on pilots.
    """
    z = np.asarray(llr, dtype=np.float64)
    b = np.asarray(bits, dtype=np.float64)
    m = np.broadcast_to(np.asarray(data_mask, dtype=bool)[None, :, :, None], z.shape)
    count = float(m.sum())
    per = np.maximum(z, 0.0) - z * b + np.log1p(np.exp(-np.abs(z)))
    loss = float(per[m].sum() / count)
    sig = 1.0 / (1.0 + np.exp(-z))
    g = np.where(m, (sig - b) / count, 0.0)
    return loss, g


# ----------------------------------------------------------------------------- backward

def backward(p: Dict, cache: Dict, dllr: np.ndarray) -> Dict:
    """Reverse-mode gradient of the FP64 forward (quant must have been None).

    Returns a parameter dict with the same structure as unpack(); pack() flattens it.
    The product adjoint is dO[k] = dP * prod_{j != k} O[j], formed without division.
    ReLU derivatives use the strict rule (pre-activation > 0).
    The normalisation adjoint is the same expression for both norms, with the means taken
    over what the statistics were taken over: the C channels of each RE (LayerNorm), or every
    RE of the batch per channel (BatchNorm with batch statistics, where the statistics depend
    on every RE and so does each RE's gradient). Running statistics get zero gradient.
    """
    K, L = p["K"], p["L"]
    mask = cache["mask"]
    variant = cache.get("variant", ("product", False, "ln"))
    if variant not in (("product", False, "ln"), ("product", False, "bn_batch")):
        raise NotImplementedError("the backward covers product fusion without feedback, with LayerNorm or "
                                  "BatchNorm by batch statistics")
    stat_axes = (0, 1, 2) if variant[2] == "bn_batch" else (-1,)
    g = {"branch": [], "gamma": [None] * L, "beta": [None] * L, "norm": p.get("norm", "ln")}
    if g["norm"] == "bn":
        g["bn_mean"] = [np.zeros(p["C"]) for _ in range(L)]
        g["bn_var"] = [np.zeros(p["C"]) for _ in range(L)]
    for _k in range(K):
        g["branch"].append({"W_in": None, "b_in": None, "blocks": [dict() for _ in range(L)]})

    d = np.asarray(dllr, dtype=np.float64)
    aL = cache["aL"]
    g["W_h"] = d.reshape(-1, d.shape[-1]).T @ aL.reshape(-1, aL.shape[-1])
    g["b_h"] = d.reshape(-1, d.shape[-1]).sum(axis=0)
    da = [d @ p["W_h"]] + [np.zeros_like(aL) for _ in range(1, K)]

    for l in range(L, 0, -1):
        lev = cache["levels"][l - 1]
        O = lev["O"]
        if fused_after(mask, l):
            dA = da[0]
            ahat, sig = lev["ahat"], lev["sig"]
            g["gamma"][l - 1] = (dA * ahat).reshape(-1, ahat.shape[-1]).sum(axis=0)
            g["beta"][l - 1] = dA.reshape(-1, dA.shape[-1]).sum(axis=0)
            dh_ = p["gamma"][l - 1] * dA
            dP = (dh_ - dh_.mean(axis=stat_axes, keepdims=True)
                  - ahat * (dh_ * ahat).mean(axis=stat_axes, keepdims=True)) / sig
            dO = []
            for k in range(K):
                others = np.ones_like(O[0])
                for j in range(K):
                    if j != k:
                        others = others * O[j]
                dO.append(dP * others + (da[k] if k >= 1 else 0.0))
        else:
            g["gamma"][l - 1] = np.zeros(p["C"])
            g["beta"][l - 1] = np.zeros(p["C"])
            dO = list(da)
        new_da = []
        for k in range(K):
            blk = p["branch"][k]["blocks"][l - 1]
            gb = g["branch"][k]["blocks"][l - 1]
            x, pre, c1, z1, h = lev["x"][k], lev["pre"][k], lev["c1"][k], lev["z1"][k], lev["h"][k]
            dOk = dO[k]
            gb["b2"] = dOk.reshape(-1, dOk.shape[-1]).sum(axis=0)
            gb["W2"] = conv3x3_weight_grad(h, dOk)
            dh = conv3x3_input_grad(dOk, blk["W2"])
            dz1 = dh * (z1 > 0)
            gb["s1"] = (dz1 * c1).reshape(-1, c1.shape[-1]).sum(axis=0)
            gb["o1"] = dz1.reshape(-1, c1.shape[-1]).sum(axis=0)
            dc1 = dz1 * blk["s1"]
            gb["b1"] = dc1.reshape(-1, c1.shape[-1]).sum(axis=0)
            gb["W1"] = conv3x3_weight_grad(pre, dc1)
            dpre = conv3x3_input_grad(dc1, blk["W1"])
            dx = dOk.copy()
            if lev["mrb"][k]:
                dx += dpre * (x > 0)
                gb["s0"] = np.zeros(p["C"])
                gb["o0"] = np.zeros(p["C"])
            else:
                z0 = blk["s0"] * x + blk["o0"]
                dz0 = dpre * (z0 > 0)
                gb["s0"] = (dz0 * x).reshape(-1, x.shape[-1]).sum(axis=0)
                gb["o0"] = dz0.reshape(-1, x.shape[-1]).sum(axis=0)
                dx += dz0 * blk["s0"]
            new_da.append(dx)
        da = new_da

    X = cache["X"]
    for k in range(K):
        a0 = cache["a0"][k]
        dz = da[k] * (a0 > 0)
        g["branch"][k]["W_in"] = conv3x3_weight_grad(X, dz)
        g["branch"][k]["b_in"] = dz.reshape(-1, dz.shape[-1]).sum(axis=0)
    return g


def grad_blob(p: Dict, X: np.ndarray, dllr: np.ndarray, fuse_mask: Optional[int] = None,
              norm: Optional[str] = None) -> np.ndarray:
    """Gradient of sum(LLR * dllr) with respect to the blob, in blob order (norm: forward()'s)."""
    _, cache = forward(p, X, fuse_mask=fuse_mask, keep=True, norm=norm)
    g = backward(p, cache, dllr)
    return pack(g)


def calibrate(p: Dict, X: np.ndarray, fuse_mask: Optional[int] = None, **variant) -> np.ndarray:
    """Static FP8 activation scales: max |operand| over a calibration batch / 448.
    variant: forward()'s fusion / feedback options of the network being calibrated."""
    K, L = p["K"], p["L"]
    amax = np.zeros(1 + 2 * K * L)
    for b in range(X.shape[0]):
        forward(p, X[b:b + 1], fuse_mask=fuse_mask, calib=amax, **variant)
    return np.where(amax > 0, amax / E4M3_MAX, 1.0)
