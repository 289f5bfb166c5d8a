"""Pins of the oracle's 3x3 convolution and its two adjoints (CPU)."""
import numpy as np
import pytest
import torch

from oracle import conet64 as o


def _rand(rng, *shape):
    return rng.standard_normal(shape)


@pytest.mark.parametrize("B,T,F,Ci,Co", [(1, 3, 4, 2, 3), (2, 4, 6, 3, 2), (1, 1, 1, 1, 1), (1, 2, 5, 3, 3)])
def test_conv_matches_bruteforce(B, T, F, Ci, Co):
    rng = np.random.default_rng(10)
    x, W, b = _rand(rng, B, T, F, Ci), _rand(rng, Co, Ci, 3, 3), _rand(rng, Co)
    np.testing.assert_allclose(o.conv3x3(x, W, b), o.conv3x3_bruteforce(x, W, b), atol=1e-12, rtol=0)


def test_conv_matches_torch_conv2d_fp64():
    rng = np.random.default_rng(11)
    x, W, b = _rand(rng, 2, 14, 9, 5), _rand(rng, 4, 5, 3, 3), _rand(rng, 4)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(W),
                                     torch.from_numpy(b), padding=1).permute(0, 2, 3, 1).numpy()
    np.testing.assert_allclose(o.conv3x3(x, W, b), ref, atol=1e-12, rtol=0)


@pytest.mark.parametrize("dt,df", [(-1, -1), (-1, 1), (0, 1), (1, 0), (1, -1)])
def test_single_tap_is_a_shift(dt, df):
    """A filter with one tap at offset (dt, df) reads x[t+dt, f+df] (cross-correlation), zero outside."""
    rng = np.random.default_rng(12)
    x = _rand(rng, 1, 5, 7, 2)
    W = np.zeros((2, 2, 3, 3))
    W[0, 0, dt + 1, df + 1] = 1.0
    W[1, 1, dt + 1, df + 1] = 1.0
    out = o.conv3x3(x, W)
    exp = np.zeros_like(x)
    for t in range(5):
        for f in range(7):
            if 0 <= t + dt < 5 and 0 <= f + df < 7:
                exp[0, t, f] = x[0, t + dt, f + df]
    np.testing.assert_array_equal(out, exp)


def test_padding_does_not_cross_slots():
    rng = np.random.default_rng(13)
    x, W = _rand(rng, 3, 4, 5, 2), _rand(rng, 3, 2, 3, 3)
    full = o.conv3x3(x, W)
    for b in range(3):
        np.testing.assert_allclose(full[b:b + 1], o.conv3x3(x[b:b + 1], W), atol=1e-13, rtol=0)


def test_input_grad_is_adjoint():
    """<conv(x), d> = <x, dconv(d)> for random x, d (dot-product test of the adjoint)."""
    rng = np.random.default_rng(14)
    x, W, d = _rand(rng, 2, 6, 8, 3), _rand(rng, 4, 3, 3, 3), _rand(rng, 2, 6, 8, 4)
    lhs = np.sum(o.conv3x3(x, W) * d)
    rhs = np.sum(x * o.conv3x3_input_grad(d, W))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_weight_grad_is_adjoint():
    """conv is linear in W: <conv(x; W), d> = <W, dW(x, d)>."""
    rng = np.random.default_rng(15)
    x, W, d = _rand(rng, 2, 6, 8, 3), _rand(rng, 4, 3, 3, 3), _rand(rng, 2, 6, 8, 4)
    lhs = np.sum(o.conv3x3(x, W) * d)
    rhs = np.sum(W * o.conv3x3_weight_grad(x, d))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_weight_grad_bruteforce():
    rng = np.random.default_rng(16)
    x, d = _rand(rng, 1, 3, 4, 2), _rand(rng, 1, 3, 4, 2)
    dW = o.conv3x3_weight_grad(x, d)
    exp = np.zeros((2, 2, 3, 3))
    for t in range(3):
        for f in range(4):
            for a in range(3):
                for c in range(3):
                    tt, ff = t + a - 1, f + c - 1
                    if 0 <= tt < 3 and 0 <= ff < 4:
                        exp[:, :, a, c] += np.outer(d[0, t, f], x[0, tt, ff])
    np.testing.assert_allclose(dW, exp, atol=1e-12, rtol=0)
