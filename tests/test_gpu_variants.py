"""GPU parity of the block and fusion variants (through the C ABI) against the FP64 oracle:
support nets shallower than the main net and fusion by concatenation (Sec. III), and
depthwise-separable residual blocks (Sec. II-A).

Bounds as for the standard network: FP32 vs FP64 rel-L2 <= 1e-5 and max|d|/RMS <= 1e-4;
BF16 and FP8 against the oracle's emulation of the same contract within the bound of its
model of the GPU arithmetic (helpers.check_vs_emulation: element-wise, rel-L2, tile seams),
and BF16 against FP64 within rel-L2 3e-2 and 99 % sign agreement."""
import numpy as np
import pytest

from helpers import check_vs_emulation, features, max_over_rms, rel_l2, say, sign_agree
from oracle import conet64 as o
from synth import ModelConfig, SimConfig, make_blob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DS_TW = 16


def _setup(K, L, C, Ci, m, mask, Ls, fusion, block, seed):
    mc = ModelConfig(K, L, C, Ci, m, mask, Ls, fusion, block)
    blob = make_blob(mc, seed=seed, perturb=True)
    p = o.unpack(blob, K, L, C, Ci, m, support_blocks=Ls, fusion=fusion, block=block)
    return mc, blob, p


def _model(mc, blob, dtype, fusion, block, feedback=False, max_res=1 << 20):
    from paper_2510_12739_amd import Conet
    return Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, dtype=dtype, fuse_mask=mc.mask, fusion=fusion,
                 feedback=feedback, support_blocks=mc.support_blocks, block=block, max_res=max_res)


def _run(model, X):
    y = model(torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda())
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def _check(dtype, got, p, X, mc, feedback, tw, label, scales=None):
    kw = dict(fuse_mask=mc.mask, feedback=feedback)
    ref = o.forward_slots(p, X.astype(np.float64), **kw)
    if dtype == "f32":
        assert rel_l2(got, ref) <= 1e-5 and max_over_rms(got, ref) <= 1e-4, (label, rel_l2(got, ref),
                                                                              max_over_rms(got, ref))
        return
    check_vs_emulation(got, p, X.astype(np.float64), o.Quant(dtype, scales), tw, label, **kw)
    if dtype == "bf16":
        assert rel_l2(got, ref) <= 3e-2 and sign_agree(got, ref) >= 0.99, (label, rel_l2(got, ref),
                                                                            sign_agree(got, ref))


CASES = [
    # dtype, K, L, C, C_in, mask, support_blocks, fusion, block, feedback, F
    ("bf16", 3, 4, 64, 16, 0b0011, 2, "product", "standard", False, 70),   # fused 16x16 kernels
    ("f32", 2, 3, 32, 16, 0b001, 1, "sum", "standard", True, 45),
    ("bf16", 2, 3, 96, 16, 0b011, 2, "product", "standard", False, 40),     # fused 32x32 kernels
    ("bf16", 3, 3, 64, 16, 0b111, 0, "concat", "standard", False, 70),
    ("bf16", 2, 3, 32, 16, 0b101, 0, "concat", "standard", True, 53),
    ("f32", 4, 2, 32, 16, 0b11, 0, "concat", "standard", False, 33),
    ("bf16", 2, 4, 64, 16, 0b0011, 2, "concat", "standard", True, 70),
    ("bf16", 2, 2, 64, 16, 0b11, 0, "product", "ds", False, 70),
    ("f32", 3, 2, 32, 16, 0b11, 0, "sum", "ds", True, 37),
    ("bf16", 3, 3, 64, 16, 0b011, 2, "concat", "ds", True, 70),
    ("bf16", 1, 3, 64, 16, 0b000, 0, "product", "ds", False, 17),          # separable ResNet
    ("f32", 2, 3, 64, 16, 0b010, 0, "product", "ds", False, 16),
    ("bf16", 3, 2, 32, 8, 0b01, 0, "sum", "ds", False, 100),
]


@pytest.mark.parametrize("dtype,K,L,C,Ci,mask,Ls,fusion,block,feedback,F", CASES)
def test_variant_vs_oracle(dtype, K, L, C, Ci, mask, Ls, fusion, block, feedback, F):
    m = 4
    mc, blob, p = _setup(K, L, C, Ci, m, mask, Ls, fusion, block, seed=K * 100 + L * 10 + C)
    X = features(SimConfig(F=F, n_rx=Ci // 4, bits_per_symbol=m, seed=71), 2)
    label = f"{dtype} K={K} L={L} C={C} mask={mask:b} Ls={Ls or L} {fusion} {block} feedback={feedback} F={F}"
    say("variant", label)
    model = _model(mc, blob, dtype, fusion, block, feedback)
    got = _run(model, X)
    tw = DS_TW if block == "ds" else (model.block_tile_width or 32)
    _check(dtype, got, p, X, mc, feedback, tw, label)
    model.close()


def test_fp8_with_shallower_supports():
    """FP8 (32x32x64 fused kernels) with support nets of 2 of 3 blocks, scales calibrated by
    the oracle on the same slots."""
    K, L, C, Ci, m, mask, Ls = 4, 3, 96, 32, 8, 0b011, 2
    mc, blob, p = _setup(K, L, C, Ci, m, mask, Ls, "product", "standard", seed=81)
    X = features(SimConfig(F=48, n_rx=8, bits_per_symbol=m, seed=82), 2)
    scales = o.calibrate(p, X.astype(np.float64), fuse_mask=mask)
    say("fp8 shallower supports")
    model = _model(mc, blob, "fp8", "product", "standard")
    model.set_act_scales(scales)
    got = _run(model, X)
    _check("fp8", got, p, X, mc, False, model.block_tile_width, "fp8 Ls=2", scales=scales)
    model.close()


@pytest.mark.parametrize("block,fusion", [("ds", "product"), ("standard", "concat")])
def test_variant_ragged_equals_slots_alone_bitwise(block, fusion):
    K, L, C, Ci, m = 3, 2, 64, 16, 4
    mc, blob, _ = _setup(K, L, C, Ci, m, -1, 0, fusion, block, seed=83)
    model = _model(mc, blob, "bf16", fusion, block)
    rng = np.random.default_rng(84)
    Fs = [48, 7, 100, 33, 1, 16, 17]
    slots = [rng.standard_normal((14, F, Ci)).astype(np.float32) for F in Fs]
    packed = torch.from_numpy(np.concatenate([s.reshape(-1, Ci) for s in slots])).cuda()
    say(f"variant ragged vs alone ({block}, {fusion}), F =", Fs)
    mix = model.forward_ragged(packed, 14, Fs).cpu().numpy()
    off = 0
    for s in slots:
        alone = _run(model, s[None]).reshape(-1, m)
        n = s.shape[0] * s.shape[1]
        np.testing.assert_array_equal(mix[off:off + n], alone.astype(np.float32))
        off += n
    model.close()


def test_separable_full_size_sampled_slot():
    """A separable CoNet (K=3, L=4, C=64, BF16) on the throughput batch: 64 slots of 3276 x 14;
    slot 63 against the emulating oracle, and two runs bitwise equal."""
    K, L, C, Ci, m = 3, 4, 64, 16, 4
    mc, blob, p = _setup(K, L, C, Ci, m, -1, 0, "product", "ds", seed=85)
    sim = SimConfig(F=3276, n_rx=4, bits_per_symbol=m, n_taps=8, max_doppler_hz=400.0, seed=2)
    X = np.concatenate([features(sim, 8)] * 8, axis=0)
    X[63] = features(sim, 1, first=63)[0]
    say("separable full size 64 x 14 x 3276")
    model = _model(mc, blob, "bf16", "product", "ds", max_res=64 * 14 * 3276)
    got = _run(model, X)
    np.testing.assert_array_equal(got, _run(model, X))
    check_vs_emulation(got[63:], p, X[63:].astype(np.float64), o.Quant("bf16"), DS_TW, "separable full size slot 63",
                       fuse_mask=mc.mask)
    model.close()


def test_variant_configurations_refused():
    from paper_2510_12739_amd import Conet, ConetError
    say("variant configurations refused")
    for kw, dims in (
        (dict(dtype="fp8", block="ds"), (2, 2, 64, 16, 4)),               # separable: FP32 / BF16 only
        (dict(dtype="fp8", fusion="concat"), (2, 2, 64, 16, 4)),
        (dict(dtype="bf16", block="ds"), (2, 2, 96, 16, 4)),              # separable: C = 32 / 64
        (dict(dtype="bf16", fusion="concat"), (5, 2, 32, 16, 4)),         # concatenation: K <= 4
        (dict(dtype="bf16", support_blocks=2, fuse_mask=0b111), (2, 3, 64, 16, 4)),  # fusion after block 3
        (dict(dtype="bf16", support_blocks=4), (2, 3, 64, 16, 4)),
        (dict(dtype="bf16", block="ds", train=True), (2, 2, 64, 16, 4)),
        (dict(dtype="bf16", support_blocks=1, train=True), (2, 2, 64, 16, 4)),
    ):
        K, L, C, Ci, m = dims
        with pytest.raises(ConetError):
            Conet(K, L, C, Ci, m, np.zeros(10, np.float32), **kw)


@pytest.mark.parametrize("kw", [{"block": "ds"}, {"fusion": "concat", "support_blocks": 2}])
def test_variant_models_serve_and_run_without_allocation(kw):
    """A separable model and a concatenation model with shallower supports behind the
    continuous-batching server (ragged batches of uneven requests) and the allocation-free
    forward: each request's LLRs equal the model's own forward of that slot bit for bit."""
    from paper_2510_12739_amd import Conet, Server
    from synth.requests import make_requests
    K, L, C, Ci, m = 3, 3, 64, 16, 6
    mc = ModelConfig(K, L, C, Ci, m, -1, kw.get("support_blocks", 0), kw.get("fusion", "product"),
                     kw.get("block", "standard"))
    model = Conet(K, L, C, Ci, m, make_blob(mc, seed=95), dtype="bf16", max_res=14 * 3276, **kw)
    reqs = make_requests(12, seed=96)
    say(f"serving a variant model {kw}")
    srv = Server(model, mem_budget=2 << 30, n_streams=2, max_batch_res=200_000)
    tickets = [srv.submit(r.x, r.n_prb, r.n_rx, r.m) for r in reqs]
    for t, _ in tickets:
        srv.wait(t)
    srv.close()
    for r, (_, llr) in zip(reqs, tickets):
        x = np.zeros((1, 14, r.x.shape[1], Ci), np.float32)
        x[0, ..., :r.x.shape[2]] = r.x
        xt = torch.from_numpy(x).cuda()
        alone = model(xt)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(llr, alone.cpu().numpy()[0, ..., :r.m])
        if 14 * r.x.shape[1] <= model.noalloc_capacity:  # the static array's capacity
            out = torch.empty_like(alone)
            model.forward_noalloc(xt, out)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), alone.cpu().numpy())
    model.close()
