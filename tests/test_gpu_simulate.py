"""The on-device slot generator (conet_simulate) against its host reference (synth.devsim),
and a training loop fed by it (GPU).

Bound: bits bit-exact; received samples within 2e-6 of max |y| (the GPU keeps the channel
taps in FP32 and rounds y to FP32; the reference runs in FP64); noise variances within FP32
rounding."""
import numpy as np
import pytest

from helpers import say
from synth import devsim as d
from synth.ofdm import data_mask

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("F,n_rx,m,L,T,first,B", [
    (72, 4, 4, 8, 14, 5, 3),
    (37, 2, 6, 4, 12, 0, 2),
    (3276, 8, 8, 8, 14, 1000, 2),
    (24, 1, 2, 16, 13, 7, 1),
])
def test_simulate_matches_host_reference(F, n_rx, m, L, T, first, B):
    from paper_2510_12739_amd import simulate
    cfg = d.DevSimConfig(F=F, n_rx=n_rx, bits_per_symbol=m, n_taps=L, seed=0x1234567890, T=T)
    say(f"simulate F={F} n_rx={n_rx} m={m} L={L} T={T} slots {first}..{first + B - 1}")
    y, bits, nv = simulate(F, n_rx, m, first, B, n_taps=L, seed=cfg.seed, T=T)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    bits, nv = bits.cpu().numpy(), nv.cpu().numpy()
    for b in range(B):
        yr, br, _, nvr = d.simulate(cfg, first + b)
        np.testing.assert_array_equal(bits[b], br)
        got = y[b, ..., 0] + 1j * y[b, ..., 1]
        assert np.abs(got - yr).max() <= 2e-6 * np.abs(yr).max(), np.abs(got - yr).max()
        assert abs(nv[b] - nvr) <= 1e-6 * nvr


def test_slot_does_not_depend_on_its_batch():
    from paper_2510_12739_amd import simulate
    say("simulate: batch split")
    a = simulate(64, 2, 4, 10, 4, seed=9)
    b = simulate(64, 2, 4, 12, 2, seed=9)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u[2:].cpu().numpy(), v.cpu().numpy())


def test_simulate_errors():
    from paper_2510_12739_amd import ConetError, simulate
    say("simulate: errors")
    with pytest.raises(ConetError, match="EINVAL"):
        simulate(16, 2, 3, 0, 1)            # odd bits per symbol
    with pytest.raises(ConetError, match="EINVAL"):
        simulate(16, 9, 4, 0, 1)            # too many antennas
    with pytest.raises(ConetError, match="ESHAPE"):
        simulate(16, 2, 4, 0, 1, T=11)      # no second pilot symbol
    with pytest.raises(ConetError, match="EINVAL"):
        simulate(16, 2, 4, 0, 1, snr_db=(10.0, 5.0))


def test_training_on_device_generated_batches():
    """Every step draws a fresh batch on the GPU (conet_simulate), featurises it, and runs
    forward + BCE + backward + Adam; the host never touches the data. The loss falls."""
    from paper_2510_12739_amd import Conet, featurise, simulate
    from synth import ModelConfig, make_blob
    K, L, C, Ci, m, B, F = 2, 2, 32, 16, 4, 8, 96
    mc = ModelConfig(K, L, C, Ci, m)
    model = Conet(K, L, C, Ci, m, make_blob(mc, seed=3), dtype="f32", max_res=B * 14 * F, train=True)
    dm = torch.from_numpy(data_mask(14, F).astype(np.uint8)).cuda()
    n_data = int(dm.sum())
    x = torch.empty((B, 14, F, Ci), dtype=torch.float32, device="cuda")
    llr = torch.empty((B, 14, F, m), dtype=torch.float32, device="cuda")
    bufs = None
    losses = []
    say("training on device-generated batches")
    for step in range(100):
        bufs = simulate(F, 4, m, step * B, B, seed=77, snr_db=(5.0, 20.0), out=bufs)
        featurise(bufs[0], Ci, out=x)
        model.forward(x, out=llr, save=True)
        loss, dllr = model.bce(llr, bufs[1], dm, n_data)
        model.backward(dllr)
        model.adam_step(lr=3e-3)
        losses.append(float(loss.cpu()))
    model.close()
    first, last = np.mean(losses[:5]), np.mean(losses[-5:])
    say(f"  loss {first:.4f} -> {last:.4f}")
    assert np.all(np.isfinite(losses)) and last < 0.85 * first, (first, last)
