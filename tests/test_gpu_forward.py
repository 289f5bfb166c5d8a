"""GPU parity of the forward pass (through the C ABI) against the FP64 oracle.

Tolerances:
  * FP32 kernels vs FP64: rel-L2 <= 1e-5 and max|d|/RMS <= 1e-4 (FP32 accumulation over
    at most 9*96 terms per conv and 2L+2 layers).
  * BF16 / FP8 kernels vs the oracle emulating the same roundings (the precision contract of
    the oracle's Quant): tolerances from the oracle's own model of the GPU's arithmetic
    (tests/helpers.emulation_with_bound). Each conv sum carries FP32 rounding error, the FP8
    matrix instructions also truncate each product to 13 fractional bits of the largest
    product of its group of 8 (measured property of the instructions), and every value rounded
    to BF16 or e4m3 carries the FP32 error of the operations forming it. Such errors decide
    roundings next to a rounding boundary, and the K-way products amplify those flips; the
    model's own spread over two draws, times 4 element-wise and times 2 in rel-L2, is the
    bound. Tile seams must also look like the interior (mean |d| at most 3x).
  * vs plain FP64 (the stated LLR tolerances): BF16 rel-L2 <= 3e-2 and sign agreement >= 99 %;
    FP8 rel-L2 <= 0.25 and sign agreement >= 93 % on the small grids.
"""
import os

import numpy as np
import pytest

from helpers import check_vs_emulation as _elementwise
from helpers import elementwise_report, emulation_with_bound, features, max_over_rms, rel_l2, say, sign_agree
from oracle import conet64 as o
from synth import ModelConfig, SimConfig, make_blob, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _model(K, L, C, Ci, m, dtype, blob, mask=-1, max_res=1 << 20):
    from paper_2510_12739_amd import Conet
    return Conet(K, L, C, Ci, m, blob, dtype=dtype, fuse_mask=mask, max_res=max_res)


def _run(model, X):
    x = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    y = model(x)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def _oracle(K, L, C, Ci, m, blob, X, mask=-1, quant=None):
    p = o.unpack(blob, K, L, C, Ci, m)
    return o.forward_slots(p, X.astype(np.float64), fuse_mask=None if mask < 0 else mask, quant=quant)


# ----------------------------------------------------------------------------- FP32

def test_fp32_single_slot_72x14():
    """The plain FP32 workload: 1 slot, 72 x 14 grid, 2 rx, QPSK, K=2, L=2, C=32, He init."""
    w = workload("fp32_b1_f72")
    mc = w.model
    blob = make_blob(mc, seed=w.weight_seed)
    X = features(w.sim, w.batch)
    say("fp32 72x14 single slot")
    got = _run(_model(mc.K, mc.L, mc.C, mc.C_in, mc.m, "f32", blob), X)
    ref = _oracle(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, X)
    assert got.shape == (1, 14, 72, 2)
    assert rel_l2(got, ref) <= 1e-5 and max_over_rms(got, ref) <= 1e-4, (rel_l2(got, ref), max_over_rms(got, ref))


@pytest.mark.parametrize("K,L,C,Ci,m,mask,B,T,F", [
    (2, 2, 32, 8, 2, -1, 1, 14, 72),
    (3, 2, 32, 8, 4, 0b10, 2, 14, 40),     # fusion only after the deeper block
    (1, 2, 32, 8, 2, 0, 2, 14, 33),        # plain pre-activation ResNet (K=1, no fusion)
    (4, 1, 16, 8, 6, 0b1, 1, 14, 17),      # four branches, ragged tile tail
    (2, 3, 32, 8, 3, 0b101, 3, 7, 5),      # T < 14, F narrower than a tile
    (2, 2, 64, 16, 4, -1, 2, 14, 65),      # C = 64 at FP32
    (1, 1, 16, 8, 1, 0b1, 2, 1, 1),        # one RE per slot
])
def test_fp32_variants_perturbed(K, L, C, Ci, m, mask, B, T, F):
    mc = ModelConfig(K, L, C, Ci, m)
    blob = make_blob(mc, seed=K * 100 + L, perturb=True)
    rng = np.random.default_rng(K + 10 * L + F)
    X = rng.standard_normal((B, T, F, Ci)).astype(np.float32)
    say(f"fp32 variant K={K} L={L} C={C} mask={mask} B={B} T={T} F={F}")
    got = _run(_model(K, L, C, Ci, m, "f32", blob, mask), X)
    ref = _oracle(K, L, C, Ci, m, blob, X, mask)
    assert rel_l2(got, ref) <= 1e-5 and max_over_rms(got, ref) <= 1e-4, (rel_l2(got, ref), max_over_rms(got, ref))


def test_fp32_narrow_and_default_tiles_agree_bitwise():
    """FP32 convs run on 16-subcarrier tiles when a batch cannot give every CU a work-group and on
    their default 32-subcarrier tiles otherwise; the arithmetic per RE is the same, so a slot
    gives the same LLRs bit for bit alone (narrow) and in a 4-slot batch (default), and both
    match the oracle."""
    K, L, C, Ci, m = 2, 2, 32, 8, 2
    blob = make_blob(ModelConfig(K, L, C, Ci, m), seed=12, perturb=True)
    X = features(SimConfig(F=1040, n_rx=2, bits_per_symbol=2, seed=13), 4)
    model = _model(K, L, C, Ci, m, "f32", blob, max_res=4 * 14 * 1040)
    say("fp32 narrow vs default tiles, 4 x 14 x 1040")
    big = _run(model, X)
    alone = _run(model, X[:1])
    np.testing.assert_array_equal(big[:1], alone)
    ref = _oracle(K, L, C, Ci, m, blob, X[:1])
    assert rel_l2(alone, ref) <= 1e-5 and max_over_rms(alone, ref) <= 1e-4, (rel_l2(alone, ref), max_over_rms(alone, ref))
    model.close()


@pytest.mark.parametrize("dtype,K,L,C,Ci,m", [
    ("bf16", 2, 2, 32, 8, 2),     # 16x16 fused kernel, 44-subcarrier tiles
    ("bf16", 3, 2, 96, 16, 4),    # 32x32x16 fused kernel, 18-subcarrier tiles
    ("fp8", 4, 2, 96, 32, 8),     # 32x32x64 fused kernel, 22-subcarrier tiles
    ("f32", 2, 1, 96, 16, 4),     # two-conv path, 16-subcarrier tiles
])
def test_ragged_equals_uniform_slots_bitwise(dtype, K, L, C, Ci, m):
    """Each slot of a ragged batch gives exactly what it gives alone (tiles never span slots),
    for every fused tile width: slot widths below, at and across tile boundaries."""
    blob = make_blob(ModelConfig(K, L, C, Ci, m), seed=5, perturb=True)
    model = _model(K, L, C, Ci, m, dtype, blob)
    if dtype == "fp8":
        model.set_act_scales(np.full(1 + 2 * K * L, 0.05))
    rng = np.random.default_rng(3)
    Fs = [48, 7, 100, 33, 1, 22, 18, 44]
    slots = [rng.standard_normal((14, F, Ci)).astype(np.float32) for F in Fs]
    packed = torch.from_numpy(np.concatenate([s.reshape(-1, Ci) for s in slots])).cuda()
    say(f"ragged vs alone ({dtype}, C={C}), F =", Fs)
    mix = model.forward_ragged(packed, 14, Fs).cpu().numpy()
    off = 0
    for s in slots:
        alone = _run(model, s[None]).reshape(-1, m)
        n = s.shape[0] * s.shape[1]
        np.testing.assert_array_equal(mix[off:off + n], alone.astype(np.float32))
        off += n


def test_edge_cases_and_errors():
    from paper_2510_12739_amd import ConetError
    K, L, C, Ci, m = 2, 1, 32, 8, 2
    blob = make_blob(ModelConfig(K, L, C, Ci, m), seed=1)
    model = _model(K, L, C, Ci, m, "f32", blob, max_res=14 * 40)
    say("edge cases")
    x0 = torch.zeros((0, 14, 8, Ci), device="cuda")
    assert model(x0).shape == (0, 14, 8, m)
    with pytest.raises(ConetError, match="ESHAPE"):
        model(torch.zeros((1, 14, 41, Ci), device="cuda"))      # beyond max_res
    with pytest.raises(ConetError, match="ESHAPE"):
        model(torch.zeros((1, 15, 8, Ci), device="cuda"))       # more than 14 symbols
    with pytest.raises(ValueError):
        model(torch.zeros((1, 14, 8, Ci + 1), device="cuda"))
    # zero input -> every RE sees only biases; with zero biases the LLR is exactly b_h = 0
    y = model(torch.zeros((1, 14, 40, Ci), device="cuda"))
    torch.cuda.synchronize()
    assert torch.all(y == 0)


# ----------------------------------------------------------------------------- BF16

def test_bf16_small_grid_vs_emulated_and_fp64():
    K, L, C, Ci, m = 3, 2, 64, 16, 4
    blob = make_blob(ModelConfig(K, L, C, Ci, m), seed=7, perturb=True)
    sim = SimConfig(F=72, n_rx=4, bits_per_symbol=4, seed=2)
    X = features(sim, 2)
    say("bf16 K=3 L=2 C=64 F=72 B=2")
    model = _model(K, L, C, Ci, m, "bf16", blob)
    got = _run(model, X)
    p = o.unpack(blob, K, L, C, Ci, m)
    emu = _elementwise(got, p, X.astype(np.float64), o.Quant("bf16"), model.block_tile_width, "bf16 small grid")
    ref = _oracle(K, L, C, Ci, m, blob, X)
    say(f'  rel-L2 vs emulated {rel_l2(got, emu):.2e}, vs fp64 {rel_l2(got, ref):.2e}, sign {sign_agree(got, ref):.4f}')
    assert rel_l2(got, ref) <= 3e-2 and sign_agree(got, ref) >= 0.99, (rel_l2(got, ref), sign_agree(got, ref))


def test_bf16_full_size_64x3276_sampled_slots():
    """The BF16 throughput workload at full size (64 slots of 3276 x 14), in the launch
    configuration the benchmark times; the oracle checks three sampled slots."""
    w = workload("bf16_b64_f3276")
    mc = w.model
    blob = make_blob(mc, seed=w.weight_seed)
    sampled = [0, 37, 63]
    X = features(w.sim, 8)
    X = np.concatenate([X] * 8, axis=0)                       # 64 slots
    X[37] = features(w.sim, 1, first=37)[0]
    X[63] = features(w.sim, 1, first=63)[0]
    say("bf16 full size 64 x 14 x 3276")
    model = _model(mc.K, mc.L, mc.C, mc.C_in, mc.m, "bf16", blob, max_res=64 * 14 * 3276)
    got = _run(model, X)
    got2 = _run(model, X)
    np.testing.assert_array_equal(got, got2)                  # deterministic
    p = o.unpack(blob, mc.K, mc.L, mc.C, mc.C_in, mc.m)
    for s in sampled:
        ref = _oracle(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, X[s:s + 1])
        emu = _elementwise(got[s:s + 1], p, X[s:s + 1].astype(np.float64), o.Quant("bf16"), model.block_tile_width,
                           f"bf16 full size, slot {s}")
        say(f"  slot {s}: rel-L2 vs emulated {rel_l2(got[s:s + 1], emu):.2e}, vs fp64 {rel_l2(got[s:s + 1], ref):.2e}, "
            f"sign {sign_agree(got[s:s + 1], ref):.4f}")
        assert rel_l2(got[s:s + 1], ref) <= 3e-2 and sign_agree(got[s:s + 1], ref) >= 0.99


# ----------------------------------------------------------------------------- FP8

def test_fp8_small_grid_vs_emulated_and_fp64():
    K, L, C, Ci, m = 4, 2, 96, 32, 8
    mc = ModelConfig(K, L, C, Ci, m)
    blob = make_blob(mc, seed=11, perturb=True)
    sim = SimConfig(F=48, n_rx=8, bits_per_symbol=8, seed=3)
    X = features(sim, 2)
    p = o.unpack(blob, K, L, C, Ci, m)
    scales = o.calibrate(p, X.astype(np.float64))
    say("fp8 K=4 L=2 C=96 F=48 B=2")
    model = _model(K, L, C, Ci, m, "fp8", blob)
    model.set_act_scales(scales)
    got = _run(model, X)
    emu = _elementwise(got, p, X.astype(np.float64), o.Quant("fp8", scales), model.block_tile_width, "fp8 small grid")
    ref = o.forward_slots(p, X.astype(np.float64))
    say(f'  rel-L2 vs emulated {rel_l2(got, emu):.2e}, vs fp64 {rel_l2(got, ref):.2e}, sign {sign_agree(got, ref):.4f}')
    assert rel_l2(got, ref) <= 0.25 and sign_agree(got, ref) >= 0.93, (rel_l2(got, ref), sign_agree(got, ref))


@pytest.mark.parametrize("K,L,mask,fusion,feedback,T,F", [
    (1, 1, 0, "product", False, 14, 75),      # plain block with the head
    (4, 1, -1, "product", False, 14, 75),     # fused main branch with the head, three supports
    (2, 2, 0b01, "product", False, 14, 75),   # fused main branch (no head), then a plain head block
    (3, 3, -1, "sum", True, 14, 40),          # feedback: every main branch launched alone
    (4, 3, 0b101, "product", False, 14, 75),  # main + next supports paired in one launch
    (4, 2, -1, "product", False, 7, 29),      # short slot
])
def test_bf16_96_channel_fused_block_kernel(K, L, mask, fusion, feedback, T, F):
    """BF16 at 96 channels runs each block as one fused kernel on the 32x32x16 MFMA (its own
    filter packing and chunk order), for every launch kind, both fusion operators, feedback
    and a short slot, on two slots with a ragged tile tail: against the BF16-emulating
    oracle (model-derived tolerances) and plain FP64 at the stated BF16 LLR tolerance."""
    from paper_2510_12739_amd import Conet
    C, Ci, m = 96, 16, 4
    mc = ModelConfig(K, L, C, Ci, m, mask)
    blob = make_blob(mc, seed=80 + K + L, perturb=True)
    X = features(SimConfig(F=F, n_rx=4, bits_per_symbol=m, seed=81), 2)[:, :T]
    p = o.unpack(blob, K, L, C, Ci, m)
    X64 = X.astype(np.float64)
    kw = dict(fuse_mask=mc.mask, fusion=fusion, feedback=feedback)
    say(f"bf16 96-channel fused block K={K} L={L} mask={mc.mask:b} {fusion} feedback={feedback} T={T} F={F}")
    model = Conet(K, L, C, Ci, m, blob, dtype="bf16", fuse_mask=mc.mask, fusion=fusion, feedback=feedback)
    assert 0 < model.block_tile_width < F
    got = _run(model, X)
    tw = model.block_tile_width
    model.close()
    emu = _elementwise(got, p, X64, o.Quant("bf16"), tw, "bf16 96 channels", **kw)
    ref = o.forward_slots(p, X64, **kw)
    say(f'  rel-L2 vs emulated {rel_l2(got, emu):.2e}, vs fp64 {rel_l2(got, ref):.2e}, sign {sign_agree(got, ref):.4f}')
    assert got.shape == (2, T, F, m)
    assert rel_l2(got, ref) <= 3e-2 and sign_agree(got, ref) >= 0.99, (rel_l2(got, ref), sign_agree(got, ref))


def test_fp8_full_size_128x3276_sampled_windows():
    """The FP8 throughput workload at full size (128 slots of 3276 x 14, K=4 L=6 C=96), in
    the launch configuration the benchmark times. A whole slot costs the FP64 oracle about
    a minute, but an output depends only on inputs within 2L+1 = 13 subcarriers (13 stacked
    3x3 convs), so the oracle computes sampled 64-subcarrier windows exactly from the window
    plus a 13-subcarrier margin (none at a slot edge, where the zero padding is the slot's).
    Checks: two full-size runs are bitwise equal; each window run alone on the GPU gives
    bitwise the full-size run's outputs there (per-RE arithmetic does not depend on tiling);
    against the FP8-emulating oracle, the model-derived element-wise and rel-L2 tolerances;
    against FP64, sign agreement >= 0.85. Weights: the trained network when its blob is in
    tests/golden (the workload the BER comparison uses), else He-normal random weights (with
    which FP8 at this depth is ill-conditioned: the emulation itself is ~0.4 rel-L2 from FP64)."""
    w = workload("fp8_b128_f3276")
    mc = w.model
    trained = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trained_fp8_b128_f3276.npy")
    blob = np.load(trained).astype(np.float32) if os.path.exists(trained) else make_blob(mc, seed=w.weight_seed)
    R = 2 * mc.L + 1
    X = np.concatenate([features(w.sim, 8)] * 16, axis=0)     # 128 slots
    windows = [(0, 0, 64), (77, 1600, 1664), (127, 3212, 3276)]
    for s, _, _ in windows[1:]:
        X[s] = features(w.sim, 1, first=s)[0]
    def win(s, f0, f1):
        a, b = max(f0 - R, 0), min(f1 + R, X.shape[2])
        return X[s:s + 1, :, a:b], f0 - a
    p = o.unpack(blob, mc.K, mc.L, mc.C, mc.C_in, mc.m)
    scales = np.max([o.calibrate(p, win(*wd)[0].astype(np.float64)) for wd in windows], axis=0)
    say("fp8 full size 128 x 14 x 3276")
    model = _model(mc.K, mc.L, mc.C, mc.C_in, mc.m, "fp8", blob, max_res=128 * 14 * 3276)
    model.set_act_scales(scales)
    got = _run(model, X)
    np.testing.assert_array_equal(got, _run(model, X))       # deterministic
    for s, f0, f1 in windows:
        Xw, off = win(s, f0, f1)
        alone = _run(model, Xw)[:, :, off:off + (f1 - f0)]
        np.testing.assert_array_equal(alone, got[s:s + 1, :, f0:f1])
        Xw64 = Xw.astype(np.float64)
        own = lambda a: a[:, :, off:off + (f1 - f0)]
        g = got[s:s + 1, :, f0:f1]
        emu, bound, rel_bound = emulation_with_bound(p, Xw64, o.Quant("fp8", scales), sel=own)
        ref = own(o.forward(p, Xw64))
        rep = elementwise_report(g, emu, model.block_tile_width, f"fp8 full size slot {s} [{f0}, {f1}) "
                                 f"(bound {bound:.2e})")
        say(f"  slot {s} [{f0}, {f1}): vs emulated {rel_l2(g, emu):.3f} (bound {rel_bound:.3f}), vs fp64 "
            f"{rel_l2(g, ref):.3f} (emulated {rel_l2(emu, ref):.3f}), sign {sign_agree(g, ref):.4f}")
        assert rep["all"][0] <= bound and rel_l2(g, emu) <= rel_bound, (rep["all"][0], bound, rel_l2(g, emu), rel_bound)
        assert sign_agree(g, ref) >= 0.85
    model.close()


def test_fp8_calibration_matches_oracle_scales():
    K, L, C, Ci, m = 2, 2, 64, 16, 4
    mc = ModelConfig(K, L, C, Ci, m)
    blob = make_blob(mc, seed=12, perturb=True)
    X = features(SimConfig(F=64, n_rx=4, bits_per_symbol=4, seed=9), 2)
    say("fp8 calibration")
    model = _model(K, L, C, Ci, m, "fp8", blob)
    model.calibrate(torch.from_numpy(X).cuda())
    got = model.get_act_scales()
    ref = o.calibrate(o.unpack(blob, K, L, C, Ci, m), X.astype(np.float64))
    # the GPU calibrates on its own quantised forward, the oracle on exact values
    np.testing.assert_allclose(got, ref, rtol=0.1)
    y = _run(model, X)
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("K,L,mask,fusion,feedback,T,F", [
    (1, 1, 0, "product", False, 14, 75),      # plain block with the head
    (4, 1, -1, "product", False, 14, 75),     # fused main branch with the head, three supports
    (2, 2, 0b01, "product", False, 14, 75),   # fused main branch (no head), then a plain head block
    (3, 3, -1, "sum", True, 14, 40),          # feedback: every main branch launched alone
    (4, 3, 0b101, "product", False, 14, 75),  # main + next supports paired in one launch
    (4, 2, -1, "product", False, 7, 29),      # short slot: symbols 7..13 are conv padding
])
def test_fp8_fused_block_kernel_vs_emulated(K, L, mask, fusion, feedback, T, F):
    """FP8 at 96 channels runs each block as one fused kernel on the 32x32x64 MFMA (its own
    filter packing and chunk order). Every launch kind (plain, main with and without the
    head, paired main + supports), both fusion operators, feedback and a short slot, on two
    slots with a ragged tile tail, against the FP8-emulating oracle (model-derived
    tolerances, see the module notes) and plain FP64 at the FP8 bounds."""
    from paper_2510_12739_amd import Conet
    C, Ci, m = 96, 32, 8
    mc = ModelConfig(K, L, C, Ci, m, mask)
    blob = make_blob(mc, seed=70 + K + L, perturb=True)
    X = features(SimConfig(F=F, n_rx=8, bits_per_symbol=8, seed=71), 2)[:, :T]
    p = o.unpack(blob, K, L, C, Ci, m)
    X64 = X.astype(np.float64)
    kw = dict(fuse_mask=mc.mask, fusion=fusion, feedback=feedback)
    scales = o.calibrate(p, X64, **kw)
    say(f"fp8 fused block K={K} L={L} mask={mc.mask:b} {fusion} feedback={feedback} T={T} F={F}")
    model = Conet(K, L, C, Ci, m, blob, dtype="fp8", fuse_mask=mc.mask, fusion=fusion, feedback=feedback)
    assert 0 < model.block_tile_width < F  # fused kernel, several tiles per slot
    model.set_act_scales(scales)
    got = _run(model, X)
    emu = _elementwise(got, p, X64, o.Quant("fp8", scales), model.block_tile_width, "fp8 fused block", **kw)
    ref = o.forward_slots(p, X64, **kw)
    say(f'  rel-L2 vs emulated {rel_l2(got, emu):.2e}, vs fp64 {rel_l2(got, ref):.2e}, sign {sign_agree(got, ref):.4f}')
    assert got.shape == (2, T, F, m)
    assert rel_l2(got, ref) <= 0.25 and sign_agree(got, ref) >= 0.93, (rel_l2(got, ref), sign_agree(got, ref))
    model.close()


# ----------------------------------------------------------------------------- fusion variants

@pytest.mark.parametrize("dtype,K,L,C,mask,fusion,feedback", [
    ("f32", 2, 3, 32, -1, "sum", False),
    ("f32", 3, 2, 32, 0b11, "product", True),
    ("f32", 3, 3, 32, 0b101, "sum", True),
    ("bf16", 3, 3, 64, -1, "sum", False),       # fused block kernel
    ("bf16", 3, 3, 64, 0b011, "product", True),
    ("bf16", 2, 2, 32, -1, "sum", True),
])
def test_fusion_variants_vs_oracle(dtype, K, L, C, mask, fusion, feedback):
    """Fusion by addition and Example II feedback (Sec. III), through both the fused block
    kernel (BF16, C = 32/64) and the two-conv path (FP32), on a 2-slot grid with a ragged
    tile tail (F = 70): FP32 vs FP64 at the FP32 bounds, BF16 vs the BF16-emulating oracle
    (model-derived tolerances) and vs FP64 at the stated LLR tolerance."""
    from paper_2510_12739_amd import Conet
    Ci, m = 16, 4
    sim = SimConfig(F=70, n_rx=4, bits_per_symbol=m, seed=41)
    mc = ModelConfig(K, L, C, Ci, m, mask)
    blob = make_blob(mc, seed=42, perturb=True)
    X = features(sim, 2)
    say(f"fusion variant {dtype} K={K} L={L} C={C} mask={mc.mask:b} {fusion} feedback={feedback}")
    model = Conet(K, L, C, Ci, m, blob, dtype=dtype, fuse_mask=mc.mask, fusion=fusion, feedback=feedback)
    got = _run(model, X)
    p = o.unpack(blob, K, L, C, Ci, m)
    ref = o.forward_slots(p, X.astype(np.float64), fuse_mask=mc.mask, fusion=fusion, feedback=feedback)
    if dtype == "f32":
        assert rel_l2(got, ref) <= 1e-5, rel_l2(got, ref)
        assert max_over_rms(got, ref) <= 1e-4
    else:
        emu = _elementwise(got, p, X.astype(np.float64), o.Quant("bf16"), model.block_tile_width or 32,
                           f"bf16 {fusion} feedback={feedback}", fuse_mask=mc.mask, fusion=fusion, feedback=feedback)
        assert rel_l2(got, ref) <= 3e-2 and sign_agree(got, ref) >= 0.99
    model.close()


@pytest.mark.parametrize("K,L,C,mask", [
    (2, 6, 96, -1),     # CoNet of the depth-latency comparison: 14 sequential layers
    (1, 11, 96, 0),     # the 24-layer pre-activation ResNet it is compared with
    (1, 12, 64, 0),     # the equal-parameter 26-layer ResNet, at C = 64
])
def test_depth_latency_models_bf16(K, L, C, mask):
    """The networks the benchmark's depth-vs-latency experiment times (Sec. IV's comparison of
    a 14-layer CoNet with a 24-layer ResNet), at BF16 on a 2-slot grid with a ragged tail:
    against the emulating oracle with model-derived tolerances and against FP64."""
    Ci, m = 16, 4
    sim = SimConfig(F=70, n_rx=4, bits_per_symbol=m, seed=43)
    mc = ModelConfig(K, L, C, Ci, m, mask)
    blob = make_blob(mc, seed=44, perturb=True)
    X = features(sim, 2)
    say(f"depth-latency model bf16 K={K} L={L} C={C}")
    model = _model(K, L, C, Ci, m, "bf16", blob, mc.mask)
    got = _run(model, X)
    p = o.unpack(blob, K, L, C, Ci, m)
    _elementwise(got, p, X.astype(np.float64), o.Quant("bf16"), model.block_tile_width, f"bf16 K={K} L={L} C={C}",
                 fuse_mask=mc.mask)
    ref = _oracle(K, L, C, Ci, m, blob, X, mc.mask)
    assert rel_l2(got, ref) <= 3e-2 and sign_agree(got, ref) >= 0.99, (rel_l2(got, ref), sign_agree(got, ref))
    model.close()


@pytest.mark.parametrize("dtype,K,L,C,Ci,mask", [
    ("f32", 2, 2, 32, 16, -1),       # two-conv path (fusion epilogue of the second conv)
    ("bf16", 3, 3, 64, 16, -1),      # fused 16x16 kernels: paired launches, main branch with the head
    ("bf16", 3, 2, 96, 16, 0b01),    # fused 32x32x16 kernel, fused main without the head
    ("fp8", 4, 2, 96, 32, -1),       # fused 32x32x64 kernel
])
def test_batchnorm_fusion_vs_oracle(dtype, K, L, C, Ci, mask):
    """BatchNorm after the fusion (Sec. III allows BN or LN) with running statistics: the
    library folds them into a per-channel affine. The statistics are the oracle's own batch
    statistics of the same slots (BN's training-time estimate), appended to the blob.
    Bounds as for the LayerNorm network of the same dtype."""
    from paper_2510_12739_amd import Conet
    m = 4
    sim = SimConfig(F=70, n_rx=Ci // 4, bits_per_symbol=m, seed=51)
    mc = ModelConfig(K, L, C, Ci, m, mask)
    base = make_blob(mc, seed=52, perturb=True)
    X = features(sim, 2)
    X64 = X.astype(np.float64)
    p = o.unpack(np.concatenate([base, np.tile(np.concatenate([np.zeros(C), np.ones(C)]), L).astype(np.float32)]),
                 K, L, C, Ci, m, norm="bn")
    stats = {}
    o.forward(p, X64, fuse_mask=mc.mask, norm="bn_batch", bn_stats=stats)
    for l, (mu, var) in stats.items():
        p["bn_mean"][l], p["bn_var"][l] = mu, var
    blob = o.pack(p).astype(np.float32)
    p = o.unpack(blob, K, L, C, Ci, m, norm="bn")          # the FP32 statistics both sides see
    say(f"batchnorm fusion {dtype} K={K} L={L} C={C} mask={mc.mask:b}")
    model = Conet(K, L, C, Ci, m, blob, dtype=dtype, fuse_mask=mc.mask, norm="bn")
    quant = None
    if dtype == "fp8":
        scales = o.calibrate(p, X64, fuse_mask=mc.mask)
        model.set_act_scales(scales)
        quant = o.Quant("fp8", scales)
    elif dtype == "bf16":
        quant = o.Quant("bf16")
    got = _run(model, X)
    tw = model.block_tile_width or 32
    model.close()
    ref = o.forward_slots(p, X64, fuse_mask=mc.mask)
    if dtype == "f32":
        assert rel_l2(got, ref) <= 1e-5, rel_l2(got, ref)
        assert max_over_rms(got, ref) <= 1e-4
        return
    emu = _elementwise(got, p, X64, quant, tw, f"batchnorm {dtype}", fuse_mask=mc.mask)
    say(f'  rel-L2 vs emulated {rel_l2(got, emu):.2e}, vs fp64 {rel_l2(got, ref):.2e}, sign {sign_agree(got, ref):.4f}')
    if dtype == "bf16":
        assert rel_l2(got, ref) <= 3e-2 and sign_agree(got, ref) >= 0.99
    else:
        assert rel_l2(got, ref) <= 0.25 and sign_agree(got, ref) >= 0.93


def test_batchnorm_training_and_bad_variance_are_refused():
    from paper_2510_12739_amd import Conet, ConetError
    K, L, C, Ci, m = 2, 1, 16, 16, 2
    base = make_blob(ModelConfig(K, L, C, Ci, m), seed=1)
    ok = np.concatenate([base, np.zeros(C, np.float32), np.ones(C, np.float32)])
    with pytest.raises(ConetError, match="EINVAL"):
        Conet(K, L, C, Ci, m, ok, dtype="bf16", train=True, norm="bn")
    bad = ok.copy()
    bad[-1] = -1.0
    with pytest.raises(ConetError, match="EINVAL"):
        Conet(K, L, C, Ci, m, bad, dtype="bf16", norm="bn")


def test_fusion_variant_training_is_refused():
    from paper_2510_12739_amd import Conet, ConetError
    mc = ModelConfig(2, 1, 16, 16, 2)
    blob = make_blob(mc, seed=1)
    with pytest.raises(ConetError, match="EINVAL"):
        Conet(2, 1, 16, 16, 2, blob, dtype="bf16", train=True, fusion="sum")


@pytest.mark.parametrize("F", [3276, 1656])
def test_narrow_and_wide_fused_tiles_agree_bitwise(F):
    """A batch too small to fill the GPU runs on narrow fused tiles; the per-RE arithmetic is
    the same at every width, so a slot's LLRs must be bit-identical alone (narrow) and inside
    a batch large enough for wide tiles. One 1656-subcarrier slot runs on 14-subcarrier tiles
    (3 x 119 work-groups per paired launch); one 3276-subcarrier slot has too many of those for
    two work-groups per CU and runs on the 13-subcarrier build for three per CU."""
    from paper_2510_12739_amd import Conet
    K, L, C, Ci, m = 3, 2, 64, 16, 4
    blob = make_blob(ModelConfig(K, L, C, Ci, m), seed=61, perturb=True)
    sim = SimConfig(F=F, n_rx=4, bits_per_symbol=4, seed=62)
    X = features(sim, 2)
    Xb = np.concatenate([X] * 4, axis=0)  # 8 slots: 8 x (F / 30) wide tiles x 3 branches fill the GPU
    model = Conet(K, L, C, Ci, m, blob, dtype="bf16", max_res=8 * 14 * F)
    say(f"narrow (1 slot) vs wide (8 slots) fused tiles, F={F}")
    alone = _run(model, X[1:2])
    batch = _run(model, Xb)
    np.testing.assert_array_equal(alone[0], batch[5])
    model.close()
