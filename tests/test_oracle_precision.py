"""Pins of the oracle's reduced-precision emulation (conet64.Quant) against an independent
construction of the precision contract (CPU).

The contract (BF16 and FP8 paths; written out in the design notes): conv operands are
rounded (BF16: RNE; FP8: saturating RNE onto e4m3 of value / scale, with per-output-channel
filter scales amax/448 and static per-tensor activation scales); a tensor that leaves a
residual block (a block output a support net carries on, the fused activation, the input
layer's output) is stored in BF16 on both paths; everything inside a layer -- accumulation,
bias, affines, ReLU, residual add, fusion, normalisation, head -- is exact (FP64 here).

The construction below uses torch's CPU conv2d and layer_norm in FP64 with torch's own
casts (.to(torch.bfloat16), .to(torch.float8_e4m3fn)) at the contract's points; it shares
no code with conet64. The two agree to FP64 round-off, so a rounding point that moves in
either one fails here, on the CPU, without the GPU.
"""
import numpy as np
import pytest
import torch

from oracle import conet64 as o
from synth import ModelConfig, make_blob

F8MAX = 448.0


def _bf16(t):
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _e4m3(t, s):
    """Saturating e4m3 of t / s (formed in FP32), back to FP64 and rescaled."""
    q = (t / s).to(torch.float32).clamp(-F8MAX, F8MAX)
    return q.to(torch.float8_e4m3fn).to(torch.float64) * s


def _scale_idx(K, L, k, l, which):
    # the activation-scale numbering the C header documents: 0 = input layer, then for
    # branch k, block l (1-based): 1 + 2 (k L + l - 1) + {0: conv 1, 1: conv 2}
    return 1 + 2 * (k * L + l - 1) + which


def _contract_net(p, X, mask, kind, scales=None, fusion="product", feedback=False):
    K, L, C = p["K"], p["L"], p["C"]
    Ls, ds = p.get("Ls", L), p.get("block") == "ds"
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    ch = lambda v: tt(v)[None, :, None, None]

    def weight(W):
        W = tt(W)
        if kind == "bf16":
            return _bf16(W)
        Wf = W.to(torch.float32).to(torch.float64)
        amax = Wf.abs().flatten(1).max(dim=1).values
        s = torch.where(amax > 0, (amax / F8MAX).to(torch.float32).to(torch.float64), torch.ones_like(amax))
        return _e4m3(Wf, s[:, None, None, None])

    def operand(a, idx):
        return _bf16(a) if kind == "bf16" else _e4m3(a, float(scales[idx]))

    def conv(a, idx, W, b):
        return torch.nn.functional.conv2d(operand(a, idx), weight(W), tt(b), padding=1)

    def ds_conv(a, D, P, b):  # depthwise (groups = C), its output rounded as the 1x1 conv's operand
        d = torch.nn.functional.conv2d(operand(a, 0), weight(D[:, None]), padding=1, groups=C)
        return torch.nn.functional.conv2d(operand(d, 0), weight(P[:, :, None, None]), tt(b))

    store = _bf16
    x = tt(X).permute(0, 3, 1, 2)
    a = [store(torch.relu(conv(x, 0, p["branch"][k]["W_in"], p["branch"][k]["b_in"]))) for k in range(K)]
    fused_prev = False
    for l in range(1, L + 1):
        outs = []
        for k in range(K if l <= Ls else 1):
            blk = p["branch"][k]["blocks"][l - 1]
            pre = torch.relu(a[k]) if (k == 0 and fused_prev) else torch.relu(ch(blk["s0"]) * a[k] + ch(blk["o0"]))
            if ds:
                h = torch.relu(ch(blk["s1"]) * ds_conv(pre, blk["D1"], blk["P1"], blk["b1"]) + ch(blk["o1"]))
                outs.append(a[k] + ds_conv(h, blk["D2"], blk["P2"], blk["b2"]))
                continue
            h = torch.relu(ch(blk["s1"]) * conv(pre, _scale_idx(K, L, k, l, 0), blk["W1"], blk["b1"]) + ch(blk["o1"]))
            outs.append(a[k] + conv(h, _scale_idx(K, L, k, l, 1), blk["W2"], blk["b2"]))
        last = l == L
        fused = bool((mask >> (l - 1)) & 1)
        if fused and fusion == "concat":      # a 1x1 conv of the outputs side by side
            cat = torch.cat([operand(outs[0], 0)] + [store(outs[k]) for k in range(1, K)], dim=1)
            P = torch.nn.functional.conv2d(cat, weight(p["Wc"][l - 1][:, :, None, None]), tt(p["bc"][l - 1]))
        elif fused:
            P = outs[0]                       # the main output is consumed inside its block
            for k in range(1, K):             # the supports' outputs left their blocks: BF16
                P = P + store(outs[k]) if fusion == "sum" else P * store(outs[k])
        if fused:
            A = torch.nn.functional.layer_norm(P.permute(0, 2, 3, 1), (C,), tt(p["gamma"][l - 1]),
                                               tt(p["beta"][l - 1]), eps=o.LN_EPS).permute(0, 3, 1, 2)
            sup = [store(store(outs[k]) + A) if feedback else store(outs[k]) for k in range(1, K)]
            a = [A if last else store(A)] + sup
        else:
            a = [outs[0] if last else store(outs[0])] + [store(outs[k]) for k in range(1, len(outs))]
        fused_prev = fused
    return (a[0].permute(0, 2, 3, 1).numpy() @ p["W_h"].T) + p["b_h"]


CASES = [
    # K, L, C, C_in, m, mask, fusion, feedback
    (2, 2, 16, 8, 2, 0b11, "product", False),
    (3, 3, 16, 16, 4, 0b101, "product", False),     # unfused middle block: the main output is stored
    (4, 2, 32, 8, 6, 0b11, "product", False),
    (1, 2, 16, 8, 2, 0b00, "product", False),       # plain ResNet: the last output goes to the head unrounded
    (3, 2, 16, 8, 4, 0b11, "sum", True),            # fusion by addition, Example II feedback
    (2, 3, 16, 8, 4, 0b110, "product", True),
]


@pytest.mark.parametrize("K,L,C,Ci,m,mask,fusion,feedback", CASES)
@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_quant_emulation_follows_the_contract(kind, K, L, C, Ci, m, mask, fusion, feedback):
    mc = ModelConfig(K, L, C, Ci, m)
    p = o.unpack(make_blob(mc, seed=31 + K + L, perturb=True), K, L, C, Ci, m)
    X = np.random.default_rng(5 + K).standard_normal((2, 14, 11, Ci))
    kw = dict(fuse_mask=mask, fusion=fusion, feedback=feedback)
    scales = o.calibrate(p, X, **kw) if kind == "fp8" else None
    got = o.forward(p, X, quant=o.Quant(kind, scales), **kw)
    want = _contract_net(p, X, mask, kind, scales, fusion, feedback)
    exact = o.forward(p, X, **kw)
    # rounding happened (the emulation is not the exact network) ...
    assert np.linalg.norm(got - exact) > 1e-4 * np.linalg.norm(exact)
    # ... at exactly the contract's points: equal to FP64 round-off
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max())


VARIANT_CASES = [
    # K, L, C, C_in, m, mask, support_blocks, fusion, block, feedback
    (2, 3, 16, 8, 2, 0b011, 2, "product", "standard", False),   # shallower support net
    (3, 2, 16, 8, 4, 0b11, 0, "concat", "standard", False),     # fusion by concatenation
    (2, 3, 16, 8, 4, 0b001, 1, "concat", "standard", True),
    (2, 2, 16, 8, 2, 0b11, 0, "product", "ds", False),          # depthwise-separable blocks
    (3, 3, 32, 16, 4, 0b011, 2, "sum", "ds", True),
]


@pytest.mark.parametrize("K,L,C,Ci,m,mask,Ls,fusion,block,feedback", VARIANT_CASES)
def test_quant_emulation_of_block_and_fusion_variants(K, L, C, Ci, m, mask, Ls, fusion, block, feedback):
    """The BF16 contract on the variants: the depthwise output and the concatenated outputs are
    conv operands, rounded as such; shallower supports drop out after their last block."""
    mc = ModelConfig(K, L, C, Ci, m, mask, Ls, fusion, block)
    p = o.unpack(make_blob(mc, seed=41 + K + L, perturb=True), K, L, C, Ci, m, support_blocks=Ls, fusion=fusion,
                 block=block)
    X = np.random.default_rng(6 + K).standard_normal((2, 14, 11, Ci))
    kw = dict(fuse_mask=mask, feedback=feedback)
    got = o.forward(p, X, quant=o.Quant("bf16"), **kw)
    want = _contract_net(p, X, mask, "bf16", None, fusion, feedback)
    exact = o.forward(p, X, **kw)
    assert np.linalg.norm(got - exact) > 1e-4 * np.linalg.norm(exact)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-10 * np.abs(want).max())


def test_contract_construction_detects_a_moved_rounding_point():
    """The construction is sensitive to the contract: dropping the BF16 store of the supports'
    outputs before the product (one of its points) changes the result far beyond round-off."""
    K, L, C, Ci, m = 3, 2, 16, 8, 4
    p = o.unpack(make_blob(ModelConfig(K, L, C, Ci, m), seed=3, perturb=True), K, L, C, Ci, m)
    X = np.random.default_rng(2).standard_normal((1, 14, 9, Ci))
    want = _contract_net(p, X, 0b11, "bf16")

    class NoStore(o.Quant):
        def store(self, a):
            return a

    moved = o.forward(p, X, quant=NoStore("bf16"))
    assert np.abs(moved - want).max() > 1e-6 * np.abs(want).max()
