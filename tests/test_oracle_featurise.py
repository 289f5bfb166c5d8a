"""Pins of the oracle featuriser (CPU): closed forms and special cases of LS estimation
with linear interpolation."""
import numpy as np
import pytest

from oracle import featurise as fz


def _grid_from_channel(H, x=None):
    """Noiseless received grid y = H x with pilots (symbols 2, 11, even f) and data x."""
    T, F, N = H.shape
    rng = np.random.default_rng(0)
    sym = x if x is not None else (rng.choice([-1, 1], (T, F)) + 1j * rng.choice([-1, 1], (T, F))) / np.sqrt(2)
    for t in (2, 11):
        sym[t, 0::2] = fz.PILOT
    return H * sym[..., None]


@pytest.mark.parametrize("F", [7, 8])
def test_flat_static_channel_is_recovered_exactly(F):
    """One constant channel over the grid: every estimate equals it, odd edge included."""
    h = np.array([0.3 - 1.1j, -0.7 + 0.2j])
    H = np.broadcast_to(h, (14, F, 2)).copy()
    est = fz.channel_estimate(_grid_from_channel(H))
    np.testing.assert_allclose(est, H, atol=1e-14)


def test_channel_linear_in_time_is_recovered_exactly():
    """A channel on a straight line in t (constant in f) is reproduced at every symbol,
    including extrapolated symbols 0, 1, 12, 13."""
    t = np.arange(14)[:, None, None]
    H = (0.5 + 0.1j) + (0.05 - 0.02j) * t + np.zeros((14, 6, 1))
    est = fz.channel_estimate(_grid_from_channel(H))
    np.testing.assert_allclose(est, H, atol=1e-14)


def test_channel_linear_in_frequency_interior_exact_last_odd_copies():
    """A channel linear in f: interior odd subcarriers are interpolated exactly; the last
    odd subcarrier (F even) takes its left neighbour's estimate."""
    F = 10
    f = np.arange(F)[None, :, None]
    H = (1.0 - 0.5j) + (0.1 + 0.03j) * f + np.zeros((14, 1, 1))
    est = fz.channel_estimate(_grid_from_channel(H))
    np.testing.assert_allclose(est[:, :F - 1], H[:, :F - 1], atol=1e-14)
    np.testing.assert_allclose(est[:, F - 1], H[:, F - 2], atol=1e-14)


def test_pilot_division_closed_form():
    """y / p with p = (1+j)/sqrt(2) is ((a+b) + j(b-a))/sqrt(2)."""
    row = np.array([[3.0 + 4.0j], [0.0 + 0.0j]])
    h = fz.pilot_estimate(row)
    np.testing.assert_allclose(h[0, 0], (7.0 + 1.0j) / np.sqrt(2.0), atol=1e-15)


def test_feature_layout_and_zero_padding():
    """Channels 4n..4n+3 = Re y, Im y, Re H, Im H; antennas beyond N are zero."""
    rng = np.random.default_rng(3)
    y = rng.standard_normal((1, 14, 5, 2)) + 1j * rng.standard_normal((1, 14, 5, 2))
    X = fz.features(y, 16)
    H = fz.channel_estimate(y[0])
    np.testing.assert_array_equal(X[0, :, :, 4], y[0, :, :, 1].real)
    np.testing.assert_array_equal(X[0, :, :, 5], y[0, :, :, 1].imag)
    np.testing.assert_array_equal(X[0, :, :, 6], H[:, :, 1].real)
    assert np.all(X[..., 8:] == 0)
