"""Pins of the oracle's fusion variants (CPU): fusion by addition, Example II's
main -> support feedback and BatchNorm after the fusion (paper Sec. III), against an
independent FP64 implementation built from torch's conv2d, layer_norm and batch_norm, and
against special cases that reduce to the already pinned product fusion."""
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


def _torch_conet(p, X, mask, fusion, feedback, norm="ln"):
    """CoNet from library primitives: NCHW conv2d with padding 1, layer_norm over C, or
    batch_norm over (N, H, W) with running statistics ("bn") or the batch's ("bn_batch").
    Depthwise-separable blocks: conv2d with groups = C, then a 1x1 conv2d; fusion by
    concatenation: torch.cat over channels, then a 1x1 conv2d; shallower supports stop."""
    K, L, C = p["K"], p["L"], p["C"]
    Ls, ds = p.get("Ls", L), p.get("block") == "ds"
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    ch = lambda v: tt(v)[None, :, None, None]
    conv = lambda x, W, b: torch.nn.functional.conv2d(x, tt(W), tt(b), padding=1)

    def dsconv(x, D, P, b):
        d = torch.nn.functional.conv2d(x, tt(D[:, None]), padding=1, groups=C)
        return torch.nn.functional.conv2d(d, tt(P[:, :, None, None]), tt(b))

    x = tt(X).permute(0, 3, 1, 2)
    a = [torch.relu(conv(x, p["branch"][k]["W_in"], p["branch"][k]["b_in"])) for k in range(K)]
    fused_prev = False
    for l in range(L):
        outs = []
        for k in range(K if l < Ls else 1):
            blk = p["branch"][k]["blocks"][l]
            pre = torch.relu(a[k]) if (k == 0 and fused_prev) else torch.relu(ch(blk["s0"]) * a[k] + ch(blk["o0"]))
            if ds:
                h = torch.relu(ch(blk["s1"]) * dsconv(pre, blk["D1"], blk["P1"], blk["b1"]) + ch(blk["o1"]))
                outs.append(a[k] + dsconv(h, blk["D2"], blk["P2"], blk["b2"]))
                continue
            h = torch.relu(ch(blk["s1"]) * conv(pre, blk["W1"], blk["b1"]) + ch(blk["o1"]))
            outs.append(a[k] + conv(h, blk["W2"], blk["b2"]))
        fused = bool((mask >> l) & 1)
        if fused and fusion == "concat":
            P = torch.nn.functional.conv2d(torch.cat(outs, dim=1), tt(p["Wc"][l][:, :, None, None]), tt(p["bc"][l]))
        elif fused:
            P = outs[0]
            for k in range(1, K):
                P = P + outs[k] if fusion == "sum" else P * outs[k]
        if fused:
            C = P.shape[1]
            if norm == "ln":
                A = torch.nn.functional.layer_norm(P.permute(0, 2, 3, 1), (C,), tt(p["gamma"][l]), tt(p["beta"][l]),
                                                   eps=o.LN_EPS).permute(0, 3, 1, 2)
            else:
                rm, rv = (tt(p["bn_mean"][l]), tt(p["bn_var"][l])) if norm == "bn" else (None, None)
                A = torch.nn.functional.batch_norm(P, rm, rv, tt(p["gamma"][l]), tt(p["beta"][l]),
                                                   training=norm == "bn_batch", eps=o.LN_EPS)
            a = [A] + [outs[k] + A if feedback else outs[k] for k in range(1, len(outs))]
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


def _bn_params(K, L, C, Ci, m, seed):
    """Parameters with BatchNorm running statistics appended to the blob (mean ~ N(0, 0.3^2),
    variance ~ U(0.5, 2))."""
    cfg = ModelConfig(K=K, L=L, C=C, C_in=Ci, m=m)
    rng = np.random.default_rng(seed + 1000)
    tail = np.concatenate([np.concatenate([0.3 * rng.standard_normal(C), rng.uniform(0.5, 2.0, C)]) for _ in range(L)])
    blob = np.concatenate([make_blob(cfg, seed=seed, perturb=True), tail.astype(np.float32)])
    return o.unpack(blob, K, L, C, Ci, m, norm="bn"), blob


@pytest.mark.parametrize("K,L,mask,norm", [(2, 3, 0b111, "bn"), (3, 2, 0b10, "bn"), (3, 3, 0b101, "bn_batch"),
                                           (2, 2, 0b11, "bn_batch")])
def test_batchnorm_matches_torch_reference(K, L, mask, norm):
    C, Ci, m = 4, 4, 3
    p, _ = _bn_params(K, L, C, Ci, m, seed=40 + K + L)
    X = _x(seed=41)
    got = o.forward(p, X, fuse_mask=mask, norm=norm)
    ref = _torch_conet(p, X, mask, "product", False, norm=norm)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_batch_statistics_as_running_statistics_reproduce_batch_mode():
    """Running statistics recorded from a batch, stored in the blob and applied in inference
    mode give exactly the batch-statistics forward on that batch; pack() round-trips them."""
    K, L, C, Ci, m = 3, 3, 4, 4, 2
    p, blob = _bn_params(K, L, C, Ci, m, seed=42)
    np.testing.assert_array_equal(o.pack(p), blob.astype(np.float64))
    X = _x(B=3, seed=43)
    stats = {}
    batch = o.forward(p, X, norm="bn_batch", bn_stats=stats)
    assert sorted(stats) == [0, 1, 2]
    for l, (mu, var) in stats.items():
        p["bn_mean"][l], p["bn_var"][l] = mu, var
    np.testing.assert_allclose(o.forward(p, X, norm="bn"), batch, rtol=1e-12, atol=1e-12)


def test_batchnorm_with_unit_statistics_is_the_affine():
    """mean 0, var 1 - eps: BN reduces to gamma P + beta, which a LayerNorm network cannot
    produce; checked against the fusion written out by hand for one block."""
    K, L, C, Ci, m = 2, 1, 4, 4, 2
    p, _ = _bn_params(K, L, C, Ci, m, seed=44)
    p["bn_mean"][0] = np.zeros(C)
    p["bn_var"][0] = np.full(C, 1.0 - o.LN_EPS)
    X = _x(seed=45)
    got = o.forward(p, X, norm="bn")
    a = [o.relu(o.conv3x3(X, p["branch"][k]["W_in"], p["branch"][k]["b_in"])) for k in range(K)]
    outs = []
    for k in range(K):
        blk = p["branch"][k]["blocks"][0]
        h = o.relu(blk["s1"] * o.conv3x3(o.relu(blk["s0"] * a[k] + blk["o0"]), blk["W1"], blk["b1"]) + blk["o1"])
        outs.append(a[k] + o.conv3x3(h, blk["W2"], blk["b2"]))
    A = p["gamma"][0] * (outs[0] * outs[1]) + p["beta"][0]
    np.testing.assert_allclose(got, A @ p["W_h"].T + p["b_h"], rtol=1e-12, atol=1e-12)


def test_backward_refuses_batchnorm():
    p, _ = _bn_params(2, 1, 4, 4, 2, seed=46)
    llr, cache = o.forward(p, _x(seed=47), keep=True)
    with pytest.raises(NotImplementedError):
        o.backward(p, cache, np.ones_like(llr))


# ----------------------------------------------------------------------------- block and fusion variants

def _vparams(K, L, C, Ci, m, Ls=0, fusion="product", block="standard", seed=0):
    cfg = ModelConfig(K, L, C, Ci, m, -1, Ls, fusion, block)
    return o.unpack(make_blob(cfg, seed=seed, perturb=True), K, L, C, Ci, m, support_blocks=Ls, fusion=fusion,
                    block=block)


def test_depthwise_conv_is_a_diagonal_conv3x3_and_a_grouped_conv():
    """The depthwise filter is the 3x3 conv whose filter is zero off the channel diagonal, and
    torch's grouped conv2d with one group per channel."""
    rng = np.random.default_rng(61)
    x = rng.standard_normal((2, 5, 7, 6))
    D = rng.standard_normal((6, 3, 3))
    W = np.zeros((6, 6, 3, 3))
    for c in range(6):
        W[c, c] = D[c]
    got = o.dwconv3x3(x, D)
    np.testing.assert_allclose(got, o.conv3x3_bruteforce(x, W), rtol=1e-12, atol=1e-12)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(D[:, None]),
                                     padding=1, groups=6).permute(0, 2, 3, 1).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("K,L,mask,Ls,fusion,block,feedback", [
    (2, 3, 0b011, 2, "product", "standard", False),
    (3, 3, 0b001, 1, "sum", "standard", True),
    (2, 2, 0b11, 0, "concat", "standard", False),
    (3, 3, 0b101, 0, "concat", "standard", True),
    (2, 2, 0b11, 0, "product", "ds", False),
    (3, 3, 0b011, 2, "concat", "ds", True),
    (1, 3, 0b000, 0, "product", "ds", False),
])
def test_block_and_fusion_variants_match_torch_reference(K, L, mask, Ls, fusion, block, feedback):
    C, Ci, m = 4, 4, 3
    p = _vparams(K, L, C, Ci, m, Ls, fusion, block, seed=50 + K + L)
    X = _x(seed=K * 7 + L)
    got = o.forward(p, X, fuse_mask=mask, feedback=feedback)
    ref = _torch_conet(p, X, mask, fusion, feedback)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_depthwise_with_centre_tap_filters_is_the_standard_net_with_1x1_filters():
    """D = the identity filter (centre tap 1) makes each separable conv the 1x1 conv P; the
    standard network whose 3x3 filters hold P at the centre tap computes the same."""
    K, L, C, Ci, m = 2, 2, 4, 4, 2
    pd = _vparams(K, L, C, Ci, m, block="ds", seed=62)
    ps = _vparams(K, L, C, Ci, m, seed=62)
    for k in range(K):
        ps["branch"][k]["W_in"] = pd["branch"][k]["W_in"]
        ps["branch"][k]["b_in"] = pd["branch"][k]["b_in"]
        for bs, bd in zip(ps["branch"][k]["blocks"], pd["branch"][k]["blocks"]):
            for key in ("s0", "o0", "b1", "s1", "o1", "b2"):
                bs[key] = bd[key]
            for i in (1, 2):
                bd[f"D{i}"] = np.zeros((C, 3, 3)); bd[f"D{i}"][:, 1, 1] = 1.0
                W = np.zeros((C, C, 3, 3)); W[:, :, 1, 1] = bd[f"P{i}"]
                bs[f"W{i}"] = W
    for key in ("gamma", "beta", "W_h", "b_h"):
        ps[key] = pd[key]
    X = _x(seed=63)
    np.testing.assert_allclose(o.forward(pd, X), o.forward(ps, X), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("K", [2, 3])
def test_concat_with_stacked_identities_is_sum_fusion(K):
    """Wc = [I I ... I], bc = 0 projects the concatenated outputs onto their sum."""
    L, C, Ci, m = 2, 4, 4, 2
    pc = _vparams(K, L, C, Ci, m, fusion="concat", seed=64)
    for l in range(L):
        pc["Wc"][l] = np.tile(np.eye(C), (1, K)); pc["bc"][l] = np.zeros(C)
    X = _x(seed=65)
    np.testing.assert_allclose(o.forward(pc, X), o.forward(pc, X, fusion="sum"), rtol=1e-12, atol=1e-12)


def test_concat_selecting_the_main_output_ignores_the_supports():
    """Wc = [I 0], bc = 0: the fused activation is LN(O[0]); without feedback the supports then
    cannot touch the result, so the network equals its main branch alone (K = 1, same norms)."""
    K, L, C, Ci, m = 2, 3, 4, 4, 2
    pc = _vparams(K, L, C, Ci, m, fusion="concat", seed=66)
    for l in range(L):
        pc["Wc"][l] = np.concatenate([np.eye(C), np.zeros((C, C))], axis=1); pc["bc"][l] = np.zeros(C)
    p1 = dict(pc, K=1, branch=pc["branch"][:1], fusion="product")
    X = _x(seed=67)
    np.testing.assert_allclose(o.forward(pc, X), o.forward(p1, X), rtol=1e-12, atol=1e-12)


def test_support_blocks_after_the_last_fusion_do_not_matter():
    """A support net of Ls blocks equals a full-depth one whose blocks after Ls are arbitrary,
    when the fusions stop at Ls: those blocks feed nothing."""
    K, L, C, Ci, m, Ls = 3, 4, 4, 4, 2, 2
    ps = _vparams(K, L, C, Ci, m, Ls=Ls, seed=68)
    pf = _vparams(K, L, C, Ci, m, seed=69)
    for k in range(K):
        for key in ("W_in", "b_in"):
            pf["branch"][k][key] = ps["branch"][k][key]
        n = L if k == 0 else Ls
        pf["branch"][k]["blocks"][:n] = ps["branch"][k]["blocks"]
    for key in ("gamma", "beta", "W_h", "b_h"):
        pf[key] = ps[key]
    X = _x(seed=70)
    for mask, fb in ((0b11, False), (0b01, True), (0b10, True)):
        np.testing.assert_allclose(o.forward(ps, X, fuse_mask=mask, feedback=fb),
                                   o.forward(pf, X, fuse_mask=mask, feedback=fb), rtol=1e-12, atol=1e-12)


def test_variant_errors():
    p = _vparams(2, 3, 4, 4, 2, Ls=2, seed=71)
    with pytest.raises(ValueError):
        o.forward(p, _x(), fuse_mask=0b100)           # the supports have no block 3
    with pytest.raises(ValueError):
        o.forward(p, _x(), fusion="concat")           # no projection weights in this blob
    pd = _vparams(2, 2, 16, 4, 2, block="ds", seed=72)
    with pytest.raises(ValueError):
        o.forward(pd, _x(), quant=o.Quant("fp8", np.ones(9)))
    llr, cache = o.forward(p, _x(), fuse_mask=0b11, keep=True)
    with pytest.raises(NotImplementedError):
        o.backward(p, cache, np.ones_like(llr))
