"""GPU parity on the interference-limited workload (Eq. (1) with g z, the variance input
channels of Sec. II-A): the featuriser with the variances (conet_featurise_var) and the
forward with C_in = 16 + 8 input channels, against the FP64 oracle.

Tolerances are those of the plain featuriser and forward tests: features within a few FP32
ulps (received samples and variances exact); FP32 forward rel-L2 <= 1e-5 and max|d|/RMS <=
1e-4 against FP64; BF16 against the oracle's emulation within the bound of its model of the
GPU arithmetic, and rel-L2 <= 3e-2, sign agreement >= 99 % against FP64."""
import numpy as np
import pytest

from helpers import check_vs_emulation, max_over_rms, rel_l2, say, sign_agree
from oracle import conet64 as o
from oracle import featurise as fz
from synth import SimConfig, make_blob, simulate_slot, workload

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WL = "interf_bf16_b64_f3276"


def _sim(F):
    return SimConfig(**{**workload(WL).sim.__dict__, "F": F})


def _slots(sim, B, first=0):
    sl = [simulate_slot(sim, first + s) for s in range(B)]
    y = np.stack([s.y for s in sl])
    v = np.array([[s.noise_var - s.interf_var, s.interf_var] for s in sl])
    return y, v, np.stack([s.features for s in sl])


@pytest.mark.parametrize("F,B", [(70, 2), (71, 3), (3276, 2)])
def test_featurise_with_variances_matches_oracle(F, B):
    from paper_2510_12739_amd import featurise
    y, v, _ = _slots(_sim(F), B)
    y32 = np.stack([y.real, y.imag], axis=-1).astype(np.float32)
    v32 = v.astype(np.float32)
    say(f"featurise with variances F={F} B={B}")
    out = featurise(torch.from_numpy(np.ascontiguousarray(y32)).cuda(), 24,
                    variances=torch.from_numpy(v32).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    yq = y32[..., 0].astype(np.float64) + 1j * y32[..., 1].astype(np.float64)
    ref = fz.features(yq, 24, variances=v32.astype(np.float64))
    for n in range(4):
        np.testing.assert_array_equal(got[..., 4 * n], ref[..., 4 * n])
        np.testing.assert_array_equal(got[..., 4 * n + 1], ref[..., 4 * n + 1])
    np.testing.assert_array_equal(got[..., 16:], ref[..., 16:])
    tol = 1e-6 * np.abs(ref).max() + 1e-7
    assert np.abs(got - ref).max() <= tol, (np.abs(got - ref).max(), tol)


def test_featurise_with_variances_errors():
    from paper_2510_12739_amd import ConetError, featurise
    v = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
    say("featurise with variances: errors")
    with pytest.raises(ConetError, match="ESHAPE"):   # 4 antennas leave no room for the variances
        featurise(torch.zeros((1, 14, 8, 4, 2), dtype=torch.float32, device="cuda"), 16, variances=v)
    with pytest.raises(ValueError):
        featurise(torch.zeros((1, 14, 8, 4, 2), dtype=torch.float32, device="cuda"), 24,
                  variances=torch.zeros((2, 2), dtype=torch.float32, device="cuda"))
    # fewer antennas than the layout holds: zero groups between the antennas and the variances
    y = torch.randn((1, 14, 8, 2, 2), dtype=torch.float32, device="cuda")
    v = torch.tensor([[0.5, 0.25]], dtype=torch.float32, device="cuda")
    x = featurise(y, 24, variances=v).cpu().numpy()
    assert np.all(x[..., 8:16] == 0) and np.all(x[..., 16] == 0.5) and np.all(x[..., 17] == 0.25)
    assert np.all(x[..., 18:] == 0)


def _model(dtype, blob, max_res=1 << 20):
    from paper_2510_12739_amd import Conet
    mc = workload(WL).model
    return Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, dtype=dtype, max_res=max_res)


def _run(model, X):
    y = model(torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda())
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def test_forward_24_input_channels_fp32_and_bf16():
    """K=3 L=4 C=64, C_in=24 on two slots of 100 x 14: FP32 against FP64, BF16 against the
    emulation (the input conv runs 27 16-byte channel chunks per RE, one K step padded)."""
    mc = workload(WL).model
    blob = make_blob(mc, seed=61, perturb=True)
    _, _, X = _slots(_sim(100), 2)
    p = o.unpack(blob, mc.K, mc.L, mc.C, mc.C_in, mc.m)
    ref = o.forward_slots(p, X.astype(np.float64))
    say("forward C_in=24 fp32 F=100 B=2")
    got = _run(_model("f32", blob), X)
    assert rel_l2(got, ref) <= 1e-5 and max_over_rms(got, ref) <= 1e-4, (rel_l2(got, ref), max_over_rms(got, ref))
    say("forward C_in=24 bf16 F=100 B=2")
    model = _model("bf16", blob)
    got = _run(model, X)
    check_vs_emulation(got, p, X.astype(np.float64), o.Quant("bf16"), model.block_tile_width, "bf16 C_in=24")
    assert rel_l2(got, ref) <= 3e-2 and sign_agree(got, ref) >= 0.99, (rel_l2(got, ref), sign_agree(got, ref))


def test_forward_24_input_channels_full_size_sampled_slots():
    """The interference workload at full size (64 slots of 3276 x 14) in BF16; slots 0 and 63
    against the emulating oracle."""
    w = workload(WL)
    mc = w.model
    blob = make_blob(mc, seed=w.weight_seed)
    _, _, X8 = _slots(w.sim, 8)
    X = np.concatenate([X8] * 8, axis=0)
    X[63] = _slots(w.sim, 1, first=63)[2][0]
    say("forward C_in=24 bf16 full size 64 x 14 x 3276")
    model = _model("bf16", blob, max_res=64 * 14 * 3276)
    got = _run(model, X)
    p = o.unpack(blob, mc.K, mc.L, mc.C, mc.C_in, mc.m)
    for s in (0, 63):
        check_vs_emulation(got[s:s + 1], p, X[s:s + 1].astype(np.float64), o.Quant("bf16"), model.block_tile_width,
                           f"bf16 C_in=24 full size, slot {s}")


def test_fp8_with_24_input_channels_is_refused():
    from paper_2510_12739_amd import ConetError
    mc = workload(WL).model
    say("fp8 C_in=24 refused")
    with pytest.raises(ConetError):
        _model("fp8", make_blob(mc, seed=1))
