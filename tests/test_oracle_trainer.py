"""Pins of the weight trainer's network (oracle/trainer.py) against the FP64 oracle (CPU):
in FP64 its forward equals conet64.forward and its autograd gradient equals the hand-written
conet64.backward, so the weights it trains belong to the network the oracle computes."""
import numpy as np
import torch

from oracle import conet64 as o
from oracle import trainer
from synth import ModelConfig, make_blob


def _setup(K=3, L=2, C=16, Ci=8, m=4, mask=None, seed=4):
    p = o.unpack(make_blob(ModelConfig(K, L, C, Ci, m), seed=seed, perturb=True), K, L, C, Ci, m)
    X = np.random.default_rng(seed).standard_normal((2, 14, 10, Ci))
    return p, X


def test_trainer_forward_equals_oracle_fp64():
    for mask in (None, 0b01, 0b10, 0):
        p, X = _setup()
        net = trainer.TorchConet(p, fuse_mask=mask, dtype=torch.float64)
        got = net(torch.from_numpy(X)).detach().numpy()
        ref = o.forward(p, X, fuse_mask=mask)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_trainer_gradient_equals_oracle_backward_fp64():
    p, X = _setup(K=2, L=2)
    net = trainer.TorchConet(p, dtype=torch.float64)
    dllr = np.random.default_rng(9).standard_normal((2, 14, 10, 4))
    (net(torch.from_numpy(X)) * torch.from_numpy(dllr)).sum().backward()
    # write the autograd gradients into the blob order through the same parameter walk
    # (parameters the network never reads, the main net's s0/o0 after a fusion, get 0)
    for prm in net.parameters():
        prm.data.copy_(prm.grad if prm.grad is not None else torch.zeros_like(prm))
    got = net.to_blob().astype(np.float64)      # FP32 view of the gradient in blob order
    ref = o.grad_blob(p, X, dllr)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-6 * np.abs(ref).max())


def test_trainer_blob_round_trip():
    p, _ = _setup()
    blob = make_blob(ModelConfig(3, 2, 16, 8, 4), seed=4, perturb=True)
    np.testing.assert_array_equal(trainer.TorchConet(p).to_blob(), blob)


def test_bce_loss_matches_oracle():
    rng = np.random.default_rng(1)
    z = rng.standard_normal((2, 14, 6, 4)) * 3
    b = rng.integers(0, 2, z.shape).astype(np.float64)
    from synth.ofdm import data_mask
    dm = data_mask(14, 6)
    want, _ = o.bce_with_logits(z, b, dm)
    got = trainer.bce_loss(torch.from_numpy(z), torch.from_numpy(b), torch.from_numpy(dm)).item()
    assert abs(got - want) <= 1e-12 * abs(want)
