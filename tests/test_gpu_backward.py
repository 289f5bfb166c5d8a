"""GPU backward / training through the C ABI against the FP64 oracle's gradient (which is
itself pinned by finite differences), plus finite differences of the GPU forward, the
BCE and Adam closed forms, repacking after an update, determinism and the autograd
integration.

Tolerances: FP32 kernels vs the FP64 gradient: rel-L2 <= 1e-4 per parameter tensor
(FP32 accumulation over up to 64*14*2 REs x 576 terms; measured ~4e-6). BF16: the gradient
of these networks is ill-conditioned (K-way products feeding a per-RE LayerNorm): the
FP64 gradient itself moves by 0.09 rel-L2 when the weights are perturbed by 2^-9
relative, and the exact FP64 backward evaluated at the BF16-rounded forward state is 0.15
from it. The BF16 kernels are therefore checked against that oracle backward at the
BF16-emulated forward state (cosine >= 0.999, rel-L2 <= 3e-2 per parameter group, which
leaves the backward's own BF16 rounding), and against the plain FP64 gradient with the
stated bound rel-L2 <= 0.25.
"""
import numpy as np
import pytest

from helpers import features, rel_l2, say
from oracle import conet64 as o
from synth import ModelConfig, SimConfig, blob_layout, make_blob, workload
from synth.ofdm import data_mask

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _model(mc, blob, dtype, mask=-1, max_res=1 << 16):
    from paper_2510_12739_amd import Conet
    return Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, dtype=dtype, fuse_mask=mask, max_res=max_res, train=True)


def _gpu_grad(model, X, d):
    x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    dl = torch.from_numpy(np.ascontiguousarray(d, np.float32)).cuda()
    llr = model.forward(x, save=True)
    g = model.backward(dl)
    torch.cuda.synchronize()
    return llr.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)


def _split(mc, v):
    out, off = {}, 0
    for name, shape in blob_layout(mc):
        n = int(np.prod(shape))
        out[name] = v[off:off + n]
        off += n
    return out


def _groups(mc, v):
    """Parameter groups: every W*, every s*/o*/b*, gamma/beta, head."""
    parts = _split(mc, v)
    grp = {}
    for name, a in parts.items():
        leaf = name.split(".")[-1]
        key = "W" if leaf in ("W_in", "W1", "W2") else ("head" if leaf in ("W_h", "b_h") else
                                                        ("norm" if leaf in ("gamma", "beta") else "vec"))
        grp.setdefault(key, []).append(a)
    return {k: np.concatenate(v) for k, v in grp.items()}


@pytest.mark.parametrize("K,L,C,mask", [(3, 2, 16, -1), (2, 2, 32, 0b10), (3, 2, 16, 0b01), (1, 2, 16, 0),
                                       (4, 1, 16, 0b1), (2, 3, 32, 0b101), (3, 4, 64, -1)])
def test_fp32_gradient_matches_oracle_24x14(K, L, C, mask):
    """The 24 x 14 gradient-check grid, FP32 kernels vs the FP64 oracle gradient, per tensor."""
    mc = ModelConfig(K, L, C, 16, 4)
    blob = make_blob(mc, seed=40 + K + L, perturb=True)
    X = features(SimConfig(F=24, n_rx=4, bits_per_symbol=4, seed=8), 2)
    d = np.random.default_rng(K * 7 + L).standard_normal((2, 14, 24, 4))
    say(f"fp32 backward K={K} L={L} C={C} mask={mask}")
    model = _model(mc, blob, "f32", mask)
    llr, g = _gpu_grad(model, X, d)
    p = o.unpack(blob, K, L, C, 16, 4)
    ref = o.grad_blob(p, X.astype(np.float64), d, fuse_mask=None if mask < 0 else mask)
    assert rel_l2(llr, o.forward(p, X.astype(np.float64), fuse_mask=None if mask < 0 else mask)) < 1e-5
    gp, rp = _split(mc, g), _split(mc, ref)
    bad = []
    for name in rp:
        if np.linalg.norm(rp[name]) == 0:
            if np.abs(gp[name]).max() > 1e-6:
                bad.append((name, "should be 0", float(np.abs(gp[name]).max())))
            continue
        e = rel_l2(gp[name], rp[name])
        if e > 1e-4:
            bad.append((name, e))
    assert not bad, bad


def test_bf16_gradient_training_model():
    """The training workload's model (K=3, L=4, C=64, C_in=16) on a 64 x 14 grid, BF16."""
    w = workload("train_b128_f1024")
    mc = w.model
    blob = make_blob(mc, seed=3, perturb=True)
    X = features(SimConfig(F=64, n_rx=4, bits_per_symbol=4, seed=4), 2)
    d = np.random.default_rng(5).standard_normal((2, 14, 64, 4))
    say("bf16 backward K=3 L=4 C=64 F=64")
    model = _model(mc, blob, "bf16")
    _, g = _gpu_grad(model, X, d)
    p = o.unpack(blob, mc.K, mc.L, mc.C, mc.C_in, mc.m)
    ref = o.grad_blob(p, X.astype(np.float64), d)
    _, cache = o.forward(p, X.astype(np.float64), quant=o.Quant("bf16"), keep=True)
    emu = o.pack(o.backward(p, cache, d))
    gg, rg, eg = _groups(mc, g), _groups(mc, ref), _groups(mc, emu)
    for k in rg:
        cos = float(gg[k] @ eg[k] / (np.linalg.norm(gg[k]) * np.linalg.norm(eg[k])))
        say(f"  {k}: vs backward at the BF16 forward: cosine {cos:.5f}, rel-L2 {rel_l2(gg[k], eg[k]):.2e}; "
            f"vs FP64: rel-L2 {rel_l2(gg[k], rg[k]):.2e}")
        assert cos >= 0.999 and rel_l2(gg[k], eg[k]) <= 3e-2, (k, cos, rel_l2(gg[k], eg[k]))
        assert rel_l2(gg[k], rg[k]) <= 0.25


@pytest.mark.parametrize("K,L,C,mask,F", [(3, 2, 32, -1, 50), (2, 3, 64, 0b101, 62), (3, 2, 64, 0b10, 34)])
def test_bf16_gradient_block_input_gradient_in_one_launch(K, L, C, mask, F):
    """BF16 models at 32 and 64 channels, whose two input-gradient convs per block run as one
    launch: ragged last tiles (F not a multiple of the 44- or 30-subcarrier tile), partial fusion
    masks (blocks with and without the plain-ReLU pre-activation of a main branch after a fusion,
    the input layer's mask at block 0), against the oracle backward at the BF16-emulated forward
    state with the training-model test's bounds."""
    mc = ModelConfig(K, L, C, 16, 4)
    blob = make_blob(mc, seed=60 + K + L, perturb=True)
    X = features(SimConfig(F=F, n_rx=4, bits_per_symbol=4, seed=12), 2)
    d = np.random.default_rng(K + 3 * L).standard_normal((2, 14, F, 4))
    fm = None if mask < 0 else mask
    say(f"bf16 backward, one-launch input gradient: K={K} L={L} C={C} mask={mask} F={F}")
    model = _model(mc, blob, "bf16", mask)
    _, g = _gpu_grad(model, X, d)
    p = o.unpack(blob, K, L, C, 16, 4)
    _, cache = o.forward(p, X.astype(np.float64), fuse_mask=fm, quant=o.Quant("bf16"), keep=True)
    emu = o.pack(o.backward(p, cache, d))
    gg, eg = _groups(mc, g), _groups(mc, emu)
    for k in eg:
        cos = float(gg[k] @ eg[k] / (np.linalg.norm(gg[k]) * np.linalg.norm(eg[k])))
        say(f"  {k}: cosine {cos:.5f}, rel-L2 {rel_l2(gg[k], eg[k]):.2e}")
        assert cos >= 0.999 and rel_l2(gg[k], eg[k]) <= 3e-2, (k, cos, rel_l2(gg[k], eg[k]))


def test_fp32_gradient_vs_finite_differences_of_gpu_forward():
    """Directional derivative of the GPU FP32 forward vs the GPU backward, along a random direction
    over the parameters that follow the last ReLU (last block's second conv of every branch, its
    norm, the head): the LLRs are smooth in them, so central differences converge as h^2 (h = 1e-3)
    without crossing ReLU kinks, which FP32 round-off would otherwise force. Checks the product /
    LayerNorm adjoint and the filter gradient against the forward kernels themselves."""
    from paper_2510_12739_amd import Conet
    mc = ModelConfig(2, 2, 16, 16, 2)
    blob = make_blob(mc, seed=61, perturb=True).astype(np.float64)
    X = features(SimConfig(F=24, n_rx=4, bits_per_symbol=2, seed=9), 1)
    d = np.random.default_rng(62).standard_normal((1, 14, 24, 2))
    rng = np.random.default_rng(63)
    v = np.zeros(blob.size)
    off = 0
    for name, shape in blob_layout(mc):
        n = int(np.prod(shape))
        if name.endswith(f"l{mc.L}.W2") or name.endswith(f"l{mc.L}.b2") or name.startswith(f"l{mc.L}.") \
                or name in ("W_h", "b_h"):
            v[off:off + n] = rng.standard_normal(n)
        off += n
    say("fp32 finite differences")
    _, g = _gpu_grad(_model(mc, blob.astype(np.float32), "f32"), X, d)
    xt = torch.from_numpy(X).cuda()

    def f(bl):
        m = Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, bl.astype(np.float32), dtype="f32", max_res=1 << 12)
        y = m(xt)
        torch.cuda.synchronize()
        return float(np.sum(y.cpu().numpy().astype(np.float64) * d))
    h = 1e-3
    fd = (f(blob + h * v) - f(blob - h * v)) / (2 * h)
    an = float(g @ v)
    say(f"  central difference {fd:.5f}, backward {an:.5f}")
    assert abs(fd - an) <= 2e-3 * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("group", ["input_layer", "block1_conv1", "block1_affines", "block1_conv2", "norm1", "head"])
def test_fp32_gradient_vs_fp64_finite_differences_every_parameter_group(group):
    """The GPU backward against central differences of the network itself, along a random
    direction over one parameter group at a time (every branch's input layer, the first
    block's convs and affines, the first fusion's norm, the head; K=2, L=2, C=16 on a 24 x 14
    grid). The differences are taken on the FP64 forward (the oracle's forward only, not its
    backward) at h = 1e-6 of the group's scale, where no ReLU kink is crossed in practice and FP64
    round-off is ~1e-10 of the result, so they stand for the exact directional derivative; the
    FP32 GPU gradient must match it within 1e-4 relative (its own accumulation error). The
    FP32 forward cannot be differenced this finely: its round-off swamps h, and a larger h
    crosses kinks."""
    mc = ModelConfig(2, 2, 16, 16, 2)
    blob = make_blob(mc, seed=64, perturb=True).astype(np.float32).astype(np.float64)
    X = features(SimConfig(F=24, n_rx=4, bits_per_symbol=2, seed=10), 1)
    d = np.random.default_rng(65).standard_normal((1, 14, 24, 2))
    rng = np.random.default_rng(66)
    sel = {
        "input_layer": lambda n: n.endswith(".W_in") or n.endswith(".b_in"),
        "block1_conv1": lambda n: ".l1.W1" in n or ".l1.b1" in n,
        "block1_affines": lambda n: any(f".l1.{a}" in n for a in ("s0", "o0", "s1", "o1")),
        "block1_conv2": lambda n: ".l1.W2" in n or ".l1.b2" in n,
        "norm1": lambda n: n in ("l1.gamma", "l1.beta"),
        "head": lambda n: n in ("W_h", "b_h"),
    }[group]
    v = np.zeros(blob.size)
    off = 0
    for name, shape in blob_layout(mc):
        n = int(np.prod(shape))
        if sel(name):
            v[off:off + n] = rng.standard_normal(n) * max(1e-2, float(np.abs(blob[off:off + n]).mean()))
        off += n
    assert np.any(v != 0)
    say(f"fp32 gradient vs fp64 finite differences, group {group}")
    _, g = _gpu_grad(_model(mc, blob.astype(np.float32), "f32"), X, d)
    X64 = X.astype(np.float64)

    def f(bl):
        return float(np.sum(o.forward(o.unpack(bl, mc.K, mc.L, mc.C, mc.C_in, mc.m), X64) * d))
    h = 1e-6
    fd = (f(blob + h * v) - f(blob - h * v)) / (2 * h)
    an = float(g @ v)
    say(f"  central difference (FP64) {fd:.7f}, GPU backward {an:.7f}")
    assert abs(fd - an) <= 1e-4 * abs(an) + 1e-6, (group, fd, an)


def test_bce_matches_oracle():
    mc = ModelConfig(1, 1, 16, 16, 4)
    model = _model(mc, make_blob(mc, seed=1), "f32")
    rng = np.random.default_rng(70)
    z = (rng.standard_normal((2, 14, 24, 4)) * 3).astype(np.float32)
    b = rng.integers(0, 2, z.shape).astype(np.uint8)
    dm = data_mask(14, 24)
    say("bce")
    loss, dl = model.bce(torch.from_numpy(z).cuda(), torch.from_numpy(b).cuda(),
                         torch.from_numpy(dm.astype(np.uint8)).cuda(), int(dm.sum()))
    torch.cuda.synchronize()
    rl, rg = o.bce_with_logits(z.astype(np.float64), b, dm)
    assert abs(float(loss.cpu()) - rl) <= 1e-5 * abs(rl)
    np.testing.assert_allclose(dl.cpu().numpy(), rg, rtol=1e-4, atol=1e-9)


def test_adam_first_step_closed_form_and_repack():
    """Step 1 of Adam moves every weight by -lr g/(|g| + eps) (bias-corrected moments); the next
    forward runs with the updated weights (packs regenerated from the master)."""
    mc = ModelConfig(2, 2, 16, 16, 4)
    blob = make_blob(mc, seed=80, perturb=True)
    X = features(SimConfig(F=24, n_rx=4, bits_per_symbol=4, seed=10), 2)
    d = np.random.default_rng(81).standard_normal((2, 14, 24, 4))
    say("adam + repack")
    model = _model(mc, blob, "f32")
    _, g = _gpu_grad(model, X, d)
    lr = 1e-2
    model.adam_step(lr=lr, beta1=0.9, beta2=0.999, eps=1e-8)
    w1 = model.get_weights().astype(np.float64)
    exp = blob.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(w1, exp, rtol=0, atol=2e-6)
    y = model(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    ref = o.forward(o.unpack(w1, mc.K, mc.L, mc.C, mc.C_in, mc.m), X.astype(np.float64))
    assert rel_l2(y.cpu().numpy(), ref) <= 1e-5


def test_backward_is_deterministic_and_needs_a_saved_forward():
    from paper_2510_12739_amd import ConetError
    mc = ModelConfig(3, 2, 32, 16, 4)
    blob = make_blob(mc, seed=90, perturb=True)
    X = features(SimConfig(F=40, n_rx=4, bits_per_symbol=4, seed=11), 2)
    d = np.random.default_rng(91).standard_normal((2, 14, 40, 4))
    say("determinism")
    model = _model(mc, blob, "bf16")
    _, g1 = _gpu_grad(model, X, d)
    _, g2 = _gpu_grad(model, X, d)
    np.testing.assert_array_equal(g1, g2)
    model.adam_step()
    with pytest.raises(ConetError, match="ESTATE"):
        model.backward(torch.zeros((2, 14, 40, 4), device="cuda"))


def test_autograd_function_and_training_reduces_loss():
    from paper_2510_12739_amd import conet_function
    w = workload("train_b128_f1024", F=96, batch=8)
    mc = w.model
    model = _model(mc, make_blob(mc, seed=0), "bf16", max_res=8 * 14 * 96)
    Fn = conet_function()
    dm = torch.from_numpy(data_mask(14, 96).astype(np.uint8)).cuda()
    n_data = int(dm.sum())
    say("autograd + 20 Adam steps")
    params = model.master()
    params.requires_grad_(True)
    losses = []
    for step in range(20):
        Xs = features(w.sim, 8, first=100 + (step % 4) * 8)
        from synth.ofdm import simulate_slot
        bits = np.stack([simulate_slot(w.sim, 100 + (step % 4) * 8 + s).bits for s in range(8)])
        x = torch.from_numpy(Xs).cuda()
        llr = Fn.apply(x, params, model)
        loss, dllr = model.bce(llr.detach(), torch.from_numpy(bits).cuda(), dm, n_data)
        if step == 0:
            # autograd path: d(sum(llr * dllr))/dparams equals the library's gradient
            llr.backward(dllr)
            g_auto = params.grad.clone()
            g_lib = model.grads().clone()
            assert torch.equal(g_auto, g_lib)
            params.grad = None
        else:
            model.backward(dllr)
        model.adam_step(lr=2e-3)
        losses.append(float(loss.cpu()))
    say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.mean(losses[-4:]) < np.mean(losses[:4])


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_checkpoint_resume_continues_bitwise(dtype):
    """A training run checkpointed after 3 Adam steps (master weights, both moments, step
    count) and resumed in a fresh model continues exactly: after 2 more steps on the same
    batches, the resumed model's weights, moments and losses equal the uninterrupted run's."""
    w = workload("train_b128_f1024", F=48, batch=4)
    mc = w.model
    blob = make_blob(mc, seed=0)
    dm = torch.from_numpy(data_mask(14, 48).astype(np.uint8)).cuda()
    n_data = int(dm.sum())
    from synth.ofdm import simulate_slot
    batches = []
    for step in range(5):
        first = 200 + step * 4
        X = features(w.sim, 4, first=first)
        bits = np.stack([simulate_slot(w.sim, first + s).bits for s in range(4)])
        batches.append((torch.from_numpy(X).cuda(), torch.from_numpy(bits).cuda()))

    def run(model, steps):
        losses = []
        for x, bt in steps:
            llr = model.forward(x, save=True)
            loss, dllr = model.bce(llr, bt, dm, n_data)
            model.backward(dllr)
            model.adam_step(lr=2e-3)
            losses.append(float(loss.cpu()))
        return losses

    say(f"checkpoint / resume ({dtype})")
    a = _model(mc, blob, dtype, max_res=4 * 14 * 48)
    run(a, batches[:3])
    ckpt = a.save_train_state()
    assert ckpt[3] == 3
    la = run(a, batches[3:])
    wa, ma, va, na = a.save_train_state()
    b = _model(mc, make_blob(mc, seed=1), dtype, max_res=4 * 14 * 48)  # other weights: all overwritten
    b.load_train_state(*ckpt)
    lb = run(b, batches[3:])
    wb, mb, vb, nb = b.save_train_state()
    assert la == lb and na == nb == 5
    for x, y in ((wa, wb), (ma, mb), (va, vb)):
        np.testing.assert_array_equal(x, y)
