"""Pins of the oracle's fusion variants (CPU): fusion by addition and Example II's
main -> support feedback (paper Sec. III), against an independent FP64 implementation
built from torch's conv2d and layer_norm, and against special cases that reduce to the
already pinned product fusion."""
import numpy as np
import pytest
import torch

from oracle import conet64 as o
from synth import ModelConfig, make_blob


def _params(K, L, C, Ci, m, seed=0):
    cfg = ModelConfig(K=K, L=L, C=C, C_in=Ci, m=m)
    return o.unpack(make_blob(cfg, seed=seed, perturb=True), K, L, C, Ci, m)


def _x(B=2, T=5, F=7, Ci=4, seed=1):
    return np.random.default_rng(seed).standard_normal((B, T, F, Ci))


def _torch_conet(p, X, mask, fusion, feedback):
    """CoNet from library primitives: NCHW conv2d with padding 1, layer_norm over C."""
    K, L = p["K"], p["L"]
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    ch = lambda v: tt(v)[None, :, None, None]
    conv = lambda x, W, b: torch.nn.functional.conv2d(x, tt(W), tt(b), padding=1)
    x = tt(X).permute(0, 3, 1, 2)
    a = [torch.relu(conv(x, p["branch"][k]["W_in"], p["branch"][k]["b_in"])) for k in range(K)]
    fused_prev = False
    for l in range(L):
        outs = []
        for k in range(K):
            blk = p["branch"][k]["blocks"][l]
            pre = torch.relu(a[k]) if (k == 0 and fused_prev) else torch.relu(ch(blk["s0"]) * a[k] + ch(blk["o0"]))
            h = torch.relu(ch(blk["s1"]) * conv(pre, blk["W1"], blk["b1"]) + ch(blk["o1"]))
            outs.append(a[k] + conv(h, blk["W2"], blk["b2"]))
        fused = bool((mask >> l) & 1)
        if fused:
            P = outs[0]
            for k in range(1, K):
                P = P + outs[k] if fusion == "sum" else P * outs[k]
            C = P.shape[1]
            A = torch.nn.functional.layer_norm(P.permute(0, 2, 3, 1), (C,), tt(p["gamma"][l]), tt(p["beta"][l]),
                                               eps=o.LN_EPS).permute(0, 3, 1, 2)
            a = [A] + [outs[k] + A if feedback else outs[k] for k in range(1, K)]
        else:
            a = outs
        fused_prev = fused
    return (a[0].permute(0, 2, 3, 1).numpy() @ p["W_h"].T) + p["b_h"]


@pytest.mark.parametrize("K,L,mask,fusion,feedback", [
    (2, 3, 0b111, "sum", False),
    (3, 2, 0b11, "sum", False),
    (3, 3, 0b101, "sum", False),
    (2, 3, 0b111, "product", True),
    (3, 3, 0b110, "product", True),
    (3, 2, 0b11, "sum", True),
    (2, 2, 0b11, "product", False),
])
def test_variants_match_torch_reference(K, L, mask, fusion, feedback):
    C, Ci, m = 4, 4, 3
    p = _params(K, L, C, Ci, m, seed=20 + K + L)
    X = _x(seed=K * 10 + L)
    got = o.forward(p, X, fuse_mask=mask, fusion=fusion, feedback=feedback)
    ref = _torch_conet(p, X, mask, fusion, feedback)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def _zero_support(p, k):
    """Branch k outputs exactly 0 everywhere: input conv 0 with bias 0, zero blocks."""
    br = p["branch"][k]
    br["W_in"][:] = 0; br["b_in"][:] = 0.0
    for blk in br["blocks"]:
        blk["W1"][:] = 0; blk["W2"][:] = 0; blk["b2"][:] = 0


def _unit_support(p, k):
    br = p["branch"][k]
    br["W_in"][:] = 0; br["b_in"][:] = 1.0
    for blk in br["blocks"]:
        blk["W1"][:] = 0; blk["W2"][:] = 0; blk["b2"][:] = 0
        blk["s0"][:] = 1.0; blk["o0"][:] = 0.0


@pytest.mark.parametrize("K", [2, 3])
def test_sum_with_zero_supports_equals_product_with_unit_supports(K):
    """Both reduce CoNet to its main net with a LayerNorm after every block."""
    L, C, Ci, m = 2, 4, 4, 2
    ps = _params(K, L, C, Ci, m, seed=31)
    pp = _params(K, L, C, Ci, m, seed=31)
    for k in range(1, K):
        _zero_support(ps, k)
        _unit_support(pp, k)
    X = _x(seed=32)
    np.testing.assert_allclose(o.forward(ps, X, fusion="sum"), o.forward(pp, X, fusion="product"),
                               rtol=1e-12, atol=1e-12)


def test_feedback_without_fusion_changes_nothing():
    """Feedback only acts after a fusion: with an empty fuse_mask it is the plain network."""
    K, L, C, Ci, m = 3, 2, 4, 4, 2
    p = _params(K, L, C, Ci, m, seed=33)
    X = _x(seed=34)
    np.testing.assert_array_equal(o.forward(p, X, fuse_mask=0, feedback=True), o.forward(p, X, fuse_mask=0))


def test_backward_refuses_variants():
    K, L, C, Ci, m = 2, 1, 4, 4, 2
    p = _params(K, L, C, Ci, m, seed=35)
    llr, cache = o.forward(p, _x(seed=36), fusion="sum", keep=True)
    with pytest.raises(NotImplementedError):
        o.backward(p, cache, np.ones_like(llr))
