"""GPU featuriser (conet_featurise) against the FP64 oracle featuriser.

Bound: the kernel forms each estimate with a handful of FP32 operations (one complex
division by the pilot as a scaled add, one mean, one interpolation step), so every
feature is within a few FP32 ulps of the FP64 value: max |d| <= 1e-6 * max |X| + 1e-7;
the received-sample channels are copies and must match the float32 input exactly."""
import numpy as np
import pytest

from helpers import say
from oracle import featurise as fz
from synth import SimConfig, simulate_slot

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _y(sim, n):
    return np.stack([simulate_slot(sim, s).y for s in range(n)])  # (B, T, F, N) complex128


def _gpu(y, C_in):
    from paper_2510_12739_amd import featurise
    y32 = np.stack([y.real, y.imag], axis=-1).astype(np.float32)
    out = featurise(torch.from_numpy(np.ascontiguousarray(y32)).cuda(), C_in)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), y32


def _check(got, y32, C_in):
    yq = y32[..., 0].astype(np.float64) + 1j * y32[..., 1].astype(np.float64)
    ref = fz.features(yq, C_in)  # oracle on the same (float32) received samples
    N = y32.shape[3]
    for n in range(N):
        np.testing.assert_array_equal(got[..., 4 * n], ref[..., 4 * n])
        np.testing.assert_array_equal(got[..., 4 * n + 1], ref[..., 4 * n + 1])
    tol = 1e-6 * np.abs(ref).max() + 1e-7
    assert np.abs(got - ref).max() <= tol, (np.abs(got - ref).max(), tol)
    assert np.all(got[..., 4 * N:] == 0)


@pytest.mark.parametrize("F,n_rx,C_in,B", [(70, 4, 16, 2), (71, 4, 16, 2), (48, 2, 16, 3), (72, 8, 32, 1)])
def test_featurise_matches_oracle(F, n_rx, C_in, B):
    sim = SimConfig(F=F, n_rx=n_rx, bits_per_symbol=4, seed=51)
    say(f"featurise F={F} n_rx={n_rx} C_in={C_in} B={B}")
    got, y32 = _gpu(_y(sim, B), C_in)
    _check(got, y32, C_in)


def test_featurise_full_size_sampled_slots():
    """64 slots x 3276 x 14, 4 rx (the throughput workload's input); slots 0 and 63 checked."""
    sim = SimConfig(F=3276, n_rx=4, bits_per_symbol=4, seed=52)
    y = np.stack([simulate_slot(sim, s % 4).y for s in range(64)])
    say("featurise 64 x 3276 x 14")
    got, y32 = _gpu(y, 16)
    for s in (0, 63):
        _check(got[s:s + 1], y32[s:s + 1], 16)


def test_featurise_errors():
    from paper_2510_12739_amd import ConetError, featurise
    y = torch.zeros((1, 10, 8, 2, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(ConetError, match="ESHAPE"):
        featurise(y, 16)  # T = 10 has no symbol 11
    y = torch.zeros((1, 14, 8, 5, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(ConetError, match="ESHAPE"):
        featurise(y, 16)  # 5 antennas need 20 channels


# ----------------------------------------------------------------------------- forward from the grid

@pytest.mark.parametrize("dtype,K,L,C,n_rx,C_in,T,F,B", [
    ("f32", 2, 2, 32, 4, 16, 14, 71, 2),
    ("bf16", 3, 3, 64, 4, 16, 14, 3276, 2),   # the throughput workload's grid
    ("bf16", 2, 2, 96, 2, 16, 12, 45, 3),     # 2 antennas into a 4-antenna input layer, T = 12
    ("fp8", 4, 2, 96, 8, 32, 14, 48, 2),
])
def test_forward_from_grid_equals_featurise_then_forward(dtype, K, L, C, n_rx, C_in, T, F, B):
    """conet_forward_grid forms the features inside the input layer's staging with the
    featuriser's own steps, so its LLRs equal conet_featurise + conet_forward bit for bit;
    and both match the oracle's features + forward (FP32 at the FP32 forward bound)."""
    from paper_2510_12739_amd import Conet, featurise
    from oracle import conet64 as o
    from synth import ModelConfig, make_blob
    m = 4
    sim = SimConfig(F=F, n_rx=n_rx, bits_per_symbol=m, seed=53, T=T)
    y = _y(sim, B)
    y32 = np.ascontiguousarray(np.stack([y.real, y.imag], axis=-1).astype(np.float32))
    blob = make_blob(ModelConfig(K, L, C, C_in, m), seed=54, perturb=True)
    say(f"forward from grid {dtype} K={K} L={L} C={C} n_rx={n_rx} T={T} F={F} B={B}")
    model = Conet(K, L, C, C_in, m, blob, dtype=dtype, max_res=B * T * F)
    yd = torch.from_numpy(y32).cuda()
    x = featurise(yd, C_in)
    if dtype == "fp8":
        model.calibrate(x)
    a = model(x).cpu().numpy()
    b = model.forward_grid(yd).cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a, b)
    if dtype == "f32":
        yq = y32[..., 0].astype(np.float64) + 1j * y32[..., 1].astype(np.float64)
        p = o.unpack(blob, K, L, C, C_in, m)
        ref = o.forward_slots(p, fz.features(yq, C_in))
        rel = np.linalg.norm(b - ref) / np.linalg.norm(ref)
        assert rel <= 1e-5 and np.abs(b - ref).max() <= 1e-4 * np.sqrt(np.mean(ref ** 2)), rel
    model.close()


def test_forward_from_grid_errors():
    from paper_2510_12739_amd import Conet, ConetError
    from synth import ModelConfig, make_blob
    model = Conet(2, 1, 32, 16, 2, make_blob(ModelConfig(2, 1, 32, 16, 2), seed=1), dtype="f32", max_res=14 * 64)
    say("forward from grid: errors")
    with pytest.raises(ConetError, match="ESHAPE"):
        model.forward_grid(torch.zeros((1, 11, 8, 4, 2), dtype=torch.float32, device="cuda"))  # no symbol 11
    with pytest.raises(ConetError, match="ESHAPE"):
        model.forward_grid(torch.zeros((1, 14, 8, 5, 2), dtype=torch.float32, device="cuda"))  # 20 > C_in
    with pytest.raises(ConetError, match="ESHAPE"):
        model.forward_grid(torch.zeros((1, 14, 65, 4, 2), dtype=torch.float32, device="cuda"))  # > max_res
    assert model.forward_grid(torch.zeros((0, 14, 8, 4, 2), dtype=torch.float32, device="cuda")).shape[0] == 0
    model.close()
