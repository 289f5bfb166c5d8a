"""The allocation-free forward (conet_forward_noalloc, activation buffers in the library's
static device array) gives bitwise the results of conet_forward on the same model and input,
on two calls in a row (the second smaller, so stale contents of the shared array from the
first call would show), and rejects a batch beyond its capacity with ESHAPE."""
import numpy as np
import pytest

from helpers import features, say
from synth import ModelConfig, SimConfig, make_blob

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("dtype,K,L,C,Ci,m,F1,F2", [
    ("bf16", 3, 4, 64, 16, 4, 3276, 600),    # fused block kernels; one full-band slot, then a narrower one
    ("f32", 2, 2, 32, 8, 2, 1000, 72),       # two-conv path
])
def test_noalloc_forward_equals_forward(dtype, K, L, C, Ci, m, F1, F2):
    from paper_2510_12739_amd import Conet, ConetError
    mc = ModelConfig(K, L, C, Ci, m)
    blob = make_blob(mc, seed=91, perturb=True)
    model = Conet(K, L, C, Ci, m, blob, dtype=dtype, max_res=2 * 14 * F1)
    cap = model.noalloc_capacity
    say(f"noalloc forward {dtype} K={K} L={L} C={C}: capacity {cap} REs")
    assert cap >= 14 * F1
    for F in (F1, F2):
        X = features(SimConfig(F=F, n_rx=Ci // 4, bits_per_symbol=m, seed=92), 1)
        x = torch.from_numpy(X).cuda()
        want = model.forward(x)
        got = torch.full_like(want, float("nan"))
        model.forward_noalloc(x, got)
        torch.cuda.synchronize()
        say(f"  F={F}: compared {got.numel()} LLRs")
        np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy())
    B_over = cap // (14 * 72) + 1                 # one slot more than the array holds
    xo = torch.zeros((B_over, 14, 72, Ci), device="cuda")
    with pytest.raises(ConetError, match="ESHAPE"):
        model.forward_noalloc(xo, torch.empty((B_over, 14, 72, m), device="cuda"))
    model.close()
