"""A forward recorded as a HIP graph (conet_graph_*) replays exactly the eager forward (GPU):
every replay, with eager work and synchronisations between replays and new inputs written
into the recorded buffer, equals conet_forward bit for bit."""
import numpy as np
import pytest

from helpers import features, say
from synth import ModelConfig, SimConfig, make_blob

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("dtype,K,L,C,Ci,m,B,F,kw", [
    ("f32", 2, 2, 32, 8, 2, 1, 72, {}),                      # the single-slot FP32 workload
    ("bf16", 3, 4, 64, 16, 4, 2, 300, {}),
    ("fp8", 4, 2, 96, 32, 8, 1, 96, {}),
    ("bf16", 3, 2, 64, 16, 4, 2, 70, {"block": "ds"}),
    ("bf16", 3, 3, 32, 16, 4, 1, 53, {"fusion": "concat", "support_blocks": 2}),
])
def test_graph_replays_equal_eager_forward(dtype, K, L, C, Ci, m, B, F, kw):
    from paper_2510_12739_amd import Conet
    mc = ModelConfig(K, L, C, Ci, m, -1, kw.get("support_blocks", 0), kw.get("fusion", "product"),
                     kw.get("block", "standard"))
    model = Conet(K, L, C, Ci, m, make_blob(mc, seed=91, perturb=True), dtype=dtype, max_res=B * 14 * F, **kw)
    sims = [SimConfig(F=F, n_rx=Ci // 4, bits_per_symbol=m, seed=s) for s in (92, 93, 94)]
    xs = [torch.from_numpy(features(sm, B)).cuda() for sm in sims]
    if dtype == "fp8":
        model.calibrate(xs[0])
    x = xs[0].clone()
    out = torch.empty((B, 14, F, m), dtype=torch.float32, device="cuda")
    say(f"graph replay {dtype} K={K} L={L} C={C} B={B} F={F} {kw}")
    g = model.record(x, out)
    for rep in range(6):
        x.copy_(xs[rep % 3])
        want = model(xs[rep % 3]).clone()              # eager forward between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want.cpu().numpy())
    g.close()
    model.close()


def test_graph_errors():
    from paper_2510_12739_amd import Conet, ConetError
    model = Conet(2, 1, 32, 16, 2, make_blob(ModelConfig(2, 1, 32, 16, 2), seed=1), dtype="fp8", max_res=14 * 64)
    x = torch.zeros((1, 14, 64, 16), device="cuda")
    out = torch.empty((1, 14, 64, 2), device="cuda")
    say("graph errors")
    with pytest.raises(ConetError, match="ESTATE"):
        model.record(x, out)                           # FP8 without activation scales
    model.close()
