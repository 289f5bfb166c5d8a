"""BatchNorm by batch statistics while training (Sec. III allows BN instead of LN after each
fusion) through the C ABI: the forward, the gradient and the running statistics against the
FP64 oracle (whose backward through the batch statistics is pinned by central differences on
the CPU), a short training run, the inference model made from the trained weights, and the
calls that refuse a BatchNorm model in training.

Tolerances: FP32 as the LayerNorm training tests: LLRs rel-L2 <= 1e-5 and max |error| <=
1e-4 RMS, gradients rel-L2 <= 1e-4 per parameter tensor (FP32 sums over 672 REs x 576 terms),
running statistics to 1e-5 relative. BF16: the LayerNorm training model's bounds against the
plain FP64 oracle (LLRs rel-L2 <= 3e-2, gradients rel-L2 <= 0.25 per parameter group; the
forward state itself carries BF16 rounding, see test_gpu_backward.py).
"""
import numpy as np
import pytest

from helpers import features, max_over_rms, rel_l2, say
from oracle import conet64 as o
from synth import ModelConfig, SimConfig, blob_layout, make_blob, workload
from synth.ofdm import data_mask, simulate_slot

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MOMENTUM = 0.1  # CONET_BN_MOMENTUM


def _bn_blob(mc, seed):
    """He-normal weights with perturbed affines, then running statistics for every block."""
    rng = np.random.default_rng(seed + 1000)
    tail = np.concatenate([np.concatenate([0.3 * rng.standard_normal(mc.C), rng.uniform(0.5, 2.0, mc.C)])
                           for _ in range(mc.L)])
    return np.concatenate([make_blob(mc, seed=seed, perturb=True), tail.astype(np.float32)])


def _model(mc, blob, dtype, mask=-1, max_res=1 << 16, train=True):
    from paper_2510_12739_amd import Conet
    return Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, dtype=dtype, fuse_mask=mask, max_res=max_res,
                 train=train, norm="bn")


def _split(mc, v):
    names = [(n, int(np.prod(s))) for n, s in blob_layout(mc)]
    for l in range(mc.L):
        names += [(f"bn{l + 1}.mean", mc.C), (f"bn{l + 1}.var", mc.C)]
    out, off = {}, 0
    for name, n in names:
        out[name] = v[off:off + n]
        off += n
    assert off == v.size
    return out


def _run(model, X, d):
    x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    dl = torch.from_numpy(np.ascontiguousarray(d, np.float32)).cuda()
    llr = model.forward(x, save=True)
    g = model.backward(dl)
    torch.cuda.synchronize()
    return llr.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)


def _oracle(mc, blob, X, d, mask):
    p = o.unpack(blob.astype(np.float64), mc.K, mc.L, mc.C, mc.C_in, mc.m, norm="bn")
    fm = None if mask < 0 else mask
    stats = {}
    llr = o.forward(p, X.astype(np.float64), fuse_mask=fm, norm="bn_batch", bn_stats=stats)
    g = o.grad_blob(p, X.astype(np.float64), d, fuse_mask=fm, norm="bn_batch")
    return p, llr, g, stats


@pytest.mark.parametrize("K,L,C,mask", [(3, 2, 32, -1), (2, 3, 32, 0b101), (3, 4, 64, -1), (4, 1, 32, 0b1),
                                       (2, 2, 64, 0b10)])
def test_fp32_forward_gradient_and_running_statistics(K, L, C, mask):
    mc = ModelConfig(K, L, C, 16, 4)
    blob = _bn_blob(mc, seed=60 + K + L)
    X = features(SimConfig(F=24, n_rx=4, bits_per_symbol=4, seed=9), 2)
    d = np.random.default_rng(K * 5 + L).standard_normal((2, 14, 24, 4))
    say(f"fp32 BatchNorm training K={K} L={L} C={C} mask={mask}")
    model = _model(mc, blob, "f32", mask)
    llr, g = _run(model, X, d)
    p, ref_llr, ref_g, stats = _oracle(mc, blob, X, d, mask)
    assert rel_l2(llr, ref_llr) < 1e-5
    assert max_over_rms(llr, ref_llr) < 1e-4
    gp, rp = _split(mc, g), _split(mc, ref_g)
    bad = []
    for name in rp:
        if np.linalg.norm(rp[name]) == 0:  # unfused levels' gamma/beta, every running statistic
            if np.abs(gp[name]).max() > 1e-6:
                bad.append((name, "should be 0", float(np.abs(gp[name]).max())))
            continue
        e = rel_l2(gp[name], rp[name])
        if e > 1e-4:
            bad.append((name, e))
    assert not bad, bad
    # the forward moved the running statistics of every fused level towards the batch's
    n = X.shape[0] * 14 * 24
    w = _split(mc, model.get_weights().astype(np.float64))
    w0 = _split(mc, blob.astype(np.float64))
    fm = (1 << L) - 1 if mask < 0 else mask
    for l in range(L):
        mean, var = w[f"bn{l + 1}.mean"], w[f"bn{l + 1}.var"]
        if not (fm >> l) & 1:
            np.testing.assert_array_equal(mean, w0[f"bn{l + 1}.mean"])
            np.testing.assert_array_equal(var, w0[f"bn{l + 1}.var"])
            continue
        mu_b, var_b = stats[l]
        ref_mean = (1 - MOMENTUM) * w0[f"bn{l + 1}.mean"] + MOMENTUM * mu_b
        ref_var = (1 - MOMENTUM) * w0[f"bn{l + 1}.var"] + MOMENTUM * var_b * n / (n - 1)
        np.testing.assert_allclose(mean, ref_mean, rtol=1e-5, atol=1e-6 * np.abs(ref_mean).max())
        np.testing.assert_allclose(var, ref_var, rtol=1e-5)


def test_fp32_deterministic_and_eval_free_of_side_effects():
    """Two backward calls give the same bits; a forward without save_for_backward normalises
    by the same batch statistics (same LLRs, bitwise) and leaves the running statistics alone."""
    mc = ModelConfig(3, 2, 32, 16, 4)
    blob = _bn_blob(mc, seed=5)
    X = features(SimConfig(F=40, n_rx=4, bits_per_symbol=4, seed=11), 2)
    d = np.random.default_rng(3).standard_normal((2, 14, 40, 4))
    say("fp32 BatchNorm training determinism")
    model = _model(mc, blob, "f32")
    x = torch.from_numpy(X).cuda()
    w_before = model.get_weights()
    llr_plain = model.forward(x).cpu().numpy()
    np.testing.assert_array_equal(model.get_weights(), w_before)
    llr1, g1 = _run(model, X, d)
    llr2, g2 = _run(model, X, d)
    np.testing.assert_array_equal(llr_plain.astype(np.float64), llr1)
    np.testing.assert_array_equal(llr1, llr2)
    np.testing.assert_array_equal(g1, g2)


def test_bf16_training_model_against_fp64():
    """The training workload's network (K=3, L=4, C=64, C_in=16) with BatchNorm, BF16, 64 x 14."""
    mc = workload("train_b128_f1024").model
    blob = _bn_blob(mc, seed=7)
    X = features(SimConfig(F=64, n_rx=4, bits_per_symbol=4, seed=4), 2)
    d = np.random.default_rng(8).standard_normal((2, 14, 64, 4))
    say("bf16 BatchNorm training K=3 L=4 C=64 F=64")
    model = _model(mc, blob, "bf16")
    llr, g = _run(model, X, d)
    _, ref_llr, ref_g, _ = _oracle(mc, blob, X, d, -1)
    e_llr = rel_l2(llr, ref_llr)
    gp, rp = _split(mc, g), _split(mc, ref_g)
    groups = {}
    for name in rp:
        leaf = name.split(".")[-1]
        key = ("W" if leaf in ("W_in", "W1", "W2") else "head" if leaf in ("W_h", "b_h") else
               "norm" if leaf in ("gamma", "beta") else "stats" if leaf in ("mean", "var") else "vec")
        groups.setdefault(key, ([], []))
        groups[key][0].append(gp[name])
        groups[key][1].append(rp[name])
    errs = {k: rel_l2(np.concatenate(a), np.concatenate(b)) for k, (a, b) in groups.items() if k != "stats"}
    say(f"  llr rel-L2 {e_llr:.3e}, gradient rel-L2 per group {errs}")
    assert e_llr < 3e-2
    assert all(e < 0.25 for e in errs.values()), errs
    assert np.abs(np.concatenate(groups["stats"][0])).max() == 0.0


def test_training_run_and_inference_model_from_its_weights():
    """30 Adam steps of a BatchNorm model on simulator batches lower the loss; the weights it
    returns (running statistics included) make an inference model (train = 0) that matches the
    oracle's running-statistics forward."""
    w = workload("train_b128_f1024", F=48, batch=4)
    mc = w.model
    blob = _bn_blob(mc, seed=0)
    dm = torch.from_numpy(data_mask(14, 48).astype(np.uint8)).cuda()
    n_data = int(dm.sum())
    say("BatchNorm training run, 30 steps, F=48")
    model = _model(mc, blob, "f32", max_res=4 * 14 * 48)
    losses = []
    for step in range(30):
        first = 300 + (step % 6) * 4
        X = features(w.sim, 4, first=first)
        bits = np.stack([simulate_slot(w.sim, first + s).bits for s in range(4)])
        llr = model.forward(torch.from_numpy(X).cuda(), save=True)
        loss, dllr = model.bce(llr, torch.from_numpy(bits).cuda(), dm, n_data)
        model.backward(dllr)
        model.adam_step(lr=2e-3)
        losses.append(float(loss.cpu()))
    say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.mean(losses[-5:]) < 0.9 * np.mean(losses[:5])
    trained = model.get_weights()
    say("  inference model from the trained weights")
    inf = _model(mc, trained, "f32", max_res=4 * 14 * 48, train=False)
    X = features(w.sim, 2, first=900)
    got = inf.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    p = o.unpack(trained.astype(np.float64), mc.K, mc.L, mc.C, mc.C_in, mc.m, norm="bn")
    ref = o.forward(p, X.astype(np.float64), norm="bn")
    assert rel_l2(got, ref) < 1e-5


def test_serving_and_static_scratch_refuse_a_training_batchnorm_model():
    from paper_2510_12739_amd import ConetError, Server
    mc = ModelConfig(2, 2, 32, 16, 4)
    model = _model(mc, _bn_blob(mc, seed=1), "bf16", max_res=4096)
    say("BatchNorm training model: refused by the server and the static-scratch forward")
    with pytest.raises(ConetError, match="BatchNorm"):
        Server(model, mem_budget=1 << 28, n_streams=1, max_batch_res=4096)
    x = torch.zeros((1, 14, 16, 16), dtype=torch.float32, device="cuda")
    out = torch.empty((1, 14, 16, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(ConetError, match="BatchNorm"):
        model.forward_noalloc(x, out)
