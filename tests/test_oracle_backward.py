"""Pins of the oracle's hand-written backward: central finite differences in FP64 (CPU)."""
import numpy as np
import pytest

from oracle import conet64 as o
from synth import ModelConfig, make_blob


def _setup(K, L, C, Ci, m, mask, seed):
    cfg = ModelConfig(K=K, L=L, C=C, C_in=Ci, m=m)
    blob = make_blob(cfg, seed=seed, perturb=True).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    X = rng.standard_normal((2, 4, 5, Ci))
    d = rng.standard_normal((2, 4, 5, m))
    f = lambda bl: float(np.sum(o.forward(o.unpack(bl, K, L, C, Ci, m), X, fuse_mask=mask) * d))
    g = o.grad_blob(o.unpack(blob, K, L, C, Ci, m), X, d, fuse_mask=mask)
    return blob, f, g


@pytest.mark.parametrize("K,L,mask", [(1, 1, 0), (1, 2, 0b11), (2, 2, 0b11), (3, 2, 0b10), (4, 1, 0b1), (2, 3, 0b101)])
def test_directional_derivative(K, L, mask):
    C, Ci, m = 3, 4, 2
    seed = 30 + K * 7 + L
    blob, f, g = _setup(K, L, C, Ci, m, mask, seed)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(blob.size)
    h = 1e-6
    fd = (f(blob + h * v) - f(blob - h * v)) / (2 * h)
    an = float(g @ v)
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_per_coordinate(K):
    """Central differences on random coordinates of every parameter kind (product adjoint, K = 2..4)."""
    L, C, Ci, m, mask = 2, 3, 4, 2, 0b11
    seed = 50 + K
    blob, f, g = _setup(K, L, C, Ci, m, mask, seed)
    rng = np.random.default_rng(seed)
    idx = rng.choice(blob.size, size=min(200, blob.size), replace=False)
    h = 1e-6
    bad = []
    for i in idx:
        e = np.zeros_like(blob); e[i] = h
        fd = (f(blob + e) - f(blob - e)) / (2 * h)
        if abs(fd - g[i]) > 1e-6 * max(1.0, abs(g[i])):
            bad.append((int(i), fd, g[i]))
    # a coordinate sitting on a ReLU kink can legitimately disagree; none is expected here
    assert len(bad) == 0, bad[:5]


def test_input_layer_gradient_of_zero_output():
    """A branch whose input conv output is negative everywhere gets no W_in gradient (ReLU mask)."""
    K, L, C, Ci, m = 1, 1, 3, 4, 2
    cfg = ModelConfig(K=K, L=L, C=C, C_in=Ci, m=m)
    blob = make_blob(cfg, seed=3, perturb=True).astype(np.float64)
    p = o.unpack(blob, K, L, C, Ci, m)
    p["branch"][0]["W_in"][:] = 0.0
    p["branch"][0]["b_in"][:] = -1.0
    X = np.random.default_rng(1).standard_normal((1, 4, 5, Ci))
    d = np.random.default_rng(2).standard_normal((1, 4, 5, m))
    _, cache = o.forward(p, X, keep=True)
    g = o.backward(p, cache, d)
    assert np.all(g["branch"][0]["W_in"] == 0) and np.all(g["branch"][0]["b_in"] == 0)


def _bn_setup(K, L, C, Ci, m, mask, seed):
    """A BatchNorm model (running statistics at the blob's end) trained by batch statistics:
    f(blob) = sum(LLR * d) of the forward that normalises by the batch's own statistics."""
    cfg = ModelConfig(K=K, L=L, C=C, C_in=Ci, m=m)
    rng = np.random.default_rng(seed + 1000)
    tail = np.concatenate([np.concatenate([0.3 * rng.standard_normal(C), rng.uniform(0.5, 2.0, C)])
                           for _ in range(L)])
    blob = np.concatenate([make_blob(cfg, seed=seed, perturb=True).astype(np.float64), tail])
    X = rng.standard_normal((3, 4, 5, Ci))
    d = rng.standard_normal((3, 4, 5, m))
    up = lambda bl: o.unpack(bl, K, L, C, Ci, m, norm="bn")
    f = lambda bl: float(np.sum(o.forward(up(bl), X, fuse_mask=mask, norm="bn_batch") * d))
    g = o.grad_blob(up(blob), X, d, fuse_mask=mask, norm="bn_batch")
    return blob, f, g


@pytest.mark.parametrize("K,L,mask", [(2, 2, 0b11), (3, 2, 0b10), (4, 1, 0b1), (2, 3, 0b101)])
def test_batchnorm_batch_statistics_directional(K, L, mask):
    C, Ci, m = 3, 4, 2
    seed = 70 + K * 7 + L
    blob, f, g = _bn_setup(K, L, C, Ci, m, mask, seed)
    assert g.size == blob.size
    v = np.random.default_rng(seed).standard_normal(blob.size)
    h = 1e-6
    fd = (f(blob + h * v) - f(blob - h * v)) / (2 * h)
    an = float(g @ v)
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_batchnorm_batch_statistics_per_coordinate():
    """Every coordinate of a K = 3 model: the statistics couple all REs of the batch, so an
    adjoint that averaged over the channels (LayerNorm's) or dropped either mean term fails
    on gamma, beta and everything below the fusion. The running statistics are not read by
    a batch-statistics forward: their gradient is exactly zero."""
    K, L, C, Ci, m, mask = 3, 2, 3, 4, 2, 0b11
    blob, f, g = _bn_setup(K, L, C, Ci, m, mask, 91)
    h = 1e-6
    bad = []
    for i in range(blob.size):
        e = np.zeros_like(blob); e[i] = h
        fd = (f(blob + e) - f(blob - e)) / (2 * h)
        if abs(fd - g[i]) > 1e-6 * max(1.0, abs(g[i])):
            bad.append((int(i), fd, g[i]))
    assert len(bad) == 0, bad[:5]
    np.testing.assert_array_equal(g[-2 * L * C:], 0.0)
