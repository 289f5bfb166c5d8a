"""Pins of the oracle's network structure: special cases, invariants, closed forms (CPU)."""
import numpy as np
import pytest
import torch

from oracle import conet64 as o
from synth import ModelConfig, make_blob


def _params(K, L, C, Ci, m, seed=0, perturb=True):
    cfg = ModelConfig(K=K, L=L, C=C, C_in=Ci, m=m)
    return o.unpack(make_blob(cfg, seed=seed, perturb=perturb), K, L, C, Ci, m)


def _x(B=2, T=5, F=7, Ci=4, seed=1):
    return np.random.default_rng(seed).standard_normal((B, T, F, Ci))


def test_unpack_pack_roundtrip():
    cfg = ModelConfig(K=3, L=2, C=4, C_in=8, m=2)
    blob = make_blob(cfg, seed=3, perturb=True)
    p = o.unpack(blob, 3, 2, 4, 8, 2)
    np.testing.assert_array_equal(o.pack(p), blob.astype(np.float64))


def test_unpack_rejects_wrong_size():
    with pytest.raises(ValueError):
        o.unpack(np.zeros(10), 1, 1, 2, 2, 2)


def test_zero_weight_blocks_are_identity():
    """W1 = W2 = 0 and b2 = 0 make every RB and MRB return its input exactly."""
    K, L, C, Ci, m = 1, 3, 4, 4, 2
    p = _params(K, L, C, Ci, m)
    for blk in p["branch"][0]["blocks"]:
        blk["W1"][:] = 0; blk["W2"][:] = 0; blk["b2"][:] = 0
    X = _x()
    a0 = np.maximum(o.conv3x3(X, p["branch"][0]["W_in"], p["branch"][0]["b_in"]), 0)
    llr = o.forward(p, X, fuse_mask=0)
    np.testing.assert_array_equal(llr, a0 @ p["W_h"].T + p["b_h"])


def test_plain_preact_resnet_special_case():
    """K = 1 without fusion is a pre-activation ResNet; checked with torch's fp64 conv2d."""
    K, L, C, Ci, m = 1, 2, 3, 4, 2
    p = _params(K, L, C, Ci, m, seed=4)
    X = _x(seed=5)
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    conv = lambda x, W, b: torch.nn.functional.conv2d(x, tt(W), tt(b), padding=1)
    x = tt(X).permute(0, 3, 1, 2)
    br = p["branch"][0]
    a = torch.relu(conv(x, br["W_in"], br["b_in"]))
    ch = lambda v: tt(v)[None, :, None, None]
    for blk in br["blocks"]:
        h = torch.relu(ch(blk["s0"]) * a + ch(blk["o0"]))
        h = torch.relu(ch(blk["s1"]) * conv(h, blk["W1"], blk["b1"]) + ch(blk["o1"]))
        a = a + conv(h, blk["W2"], blk["b2"])
    ref = (a.permute(0, 2, 3, 1).numpy() @ p["W_h"].T) + p["b_h"]
    np.testing.assert_allclose(o.forward(p, X, fuse_mask=0), ref, atol=1e-11, rtol=1e-11)


def _unit_support(p, k):
    """Branch k outputs exactly 1 everywhere: input conv 0 + bias 1, zero blocks."""
    br = p["branch"][k]
    br["W_in"][:] = 0; br["b_in"][:] = 1.0
    for blk in br["blocks"]:
        blk["W1"][:] = 0; blk["W2"][:] = 0; blk["b2"][:] = 0
        blk["s0"][:] = 1.0; blk["o0"][:] = 0.0


@pytest.mark.parametrize("K", [2, 3, 4])
def test_unit_support_nets_make_product_the_identity(K):
    """Support nets that output 1 reduce CoNet to its main net with LN after each block."""
    L, C, Ci, m = 2, 4, 4, 3
    p = _params(K, L, C, Ci, m, seed=6)
    for k in range(1, K):
        _unit_support(p, k)
    p1 = dict(p)
    p1["K"] = 1
    p1["branch"] = p["branch"][:1]
    X = _x(seed=7)
    np.testing.assert_allclose(o.forward(p, X), o.forward(p1, X), atol=1e-12, rtol=1e-12)


def test_support_nets_matter():
    """Control for the pin above: random support nets change the LLRs."""
    p = _params(2, 2, 4, 4, 2, seed=8)
    p1 = dict(p); p1["K"] = 1; p1["branch"] = p["branch"][:1]
    X = _x(seed=9)
    assert np.abs(o.forward(p, X) - o.forward(p1, X)).max() > 1e-3


def test_product_is_over_all_branches():
    """Two unit supports, one rescaled to output 3: the product is exactly 3 * O_main."""
    K, L, C, Ci, m = 3, 1, 5, 4, 2
    p = _params(K, L, C, Ci, m, seed=10)
    for k in (1, 2):
        _unit_support(p, k)
    p["branch"][2]["b_in"][:] = 3.0         # branch 2 now outputs 3
    X = _x(seed=11)
    _, cache = o.forward(p, X, keep=True)
    lev = cache["levels"][0]
    np.testing.assert_allclose(lev["P"], 3.0 * lev["O"][0], rtol=1e-14, atol=0)


def test_mrb_ignores_leading_affine_only_after_fusion():
    K, L, C, Ci, m = 2, 2, 4, 4, 2
    p = _params(K, L, C, Ci, m, seed=12)
    X = _x(seed=13)
    base_f = o.forward(p, X, fuse_mask=0b11)
    base_n = o.forward(p, X, fuse_mask=0b10)
    blk = p["branch"][0]["blocks"][1]           # main net, block 2
    blk["s0"][:] *= 1.7; blk["o0"][:] += 0.3
    np.testing.assert_array_equal(o.forward(p, X, fuse_mask=0b11), base_f)   # MRB: unchanged
    assert np.abs(o.forward(p, X, fuse_mask=0b10) - base_n).max() > 1e-3    # RB: changed


def test_support_blocks_are_never_mrb():
    K, L, C, Ci, m = 2, 2, 4, 4, 2
    p = _params(K, L, C, Ci, m, seed=14)
    X = _x(seed=15)
    base = o.forward(p, X)
    p["branch"][1]["blocks"][1]["s0"][:] *= 1.5
    assert np.abs(o.forward(p, X) - base).max() > 1e-3


def test_layernorm_invariant():
    """With gamma = 1, beta = 0 the fused activation has per-RE mean 0 and variance v/(v+eps)."""
    K, L, C, Ci, m = 3, 2, 6, 4, 2
    p = _params(K, L, C, Ci, m, seed=16)
    for l in range(L):
        p["gamma"][l][:] = 1.0; p["beta"][l][:] = 0.0
    X = _x(seed=17)
    _, cache = o.forward(p, X, keep=True)
    for lev in cache["levels"]:
        A = lev["ahat"]
        P = lev["P"]
        v = P.var(axis=-1)
        np.testing.assert_allclose(A.mean(axis=-1), 0.0, atol=1e-12)
        np.testing.assert_allclose(A.var(axis=-1), v / (v + o.LN_EPS), rtol=1e-12, atol=1e-14)


def test_head_closed_form_and_fusion_mask():
    K, L, C, Ci, m = 2, 2, 4, 4, 3
    p = _params(K, L, C, Ci, m, seed=18)
    X = _x(seed=19)
    llr, cache = o.forward(p, X, keep=True)
    np.testing.assert_allclose(llr, np.einsum("btfc,mc->btfm", cache["aL"], p["W_h"]) + p["b_h"], atol=1e-13)
    # fusion only after block 2 ("selectively, the deeper ones") differs from fusion everywhere
    assert np.abs(o.forward(p, X, fuse_mask=0b10) - llr).max() > 1e-3


def test_forward_slots_equals_batched():
    p = _params(2, 1, 4, 4, 2, seed=20)
    X = _x(B=3, seed=21)
    np.testing.assert_allclose(o.forward_slots(p, X), o.forward(p, X), atol=1e-12)


def test_bce_matches_torch_and_fd():
    rng = np.random.default_rng(22)
    z = rng.standard_normal((2, 4, 6, 2)) * 3
    b = rng.integers(0, 2, z.shape)
    dm = np.ones((4, 6), bool); dm[1, ::2] = False
    loss, g = o.bce_with_logits(z, b, dm)
    m = np.broadcast_to(dm[None, :, :, None], z.shape)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(torch.from_numpy(z[m]), torch.from_numpy(b[m].astype(float)))
    assert abs(loss - float(ref)) < 1e-12
    assert np.all(g[~m] == 0)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 3, 5, 1), (0, 2, 3, 1)]:
        zp = z.copy(); zp[idx] += h
        zm = z.copy(); zm[idx] -= h
        fd = (o.bce_with_logits(zp, b, dm)[0] - o.bce_with_logits(zm, b, dm)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-8
