"""Pins of the interference term g z of Eq. (1) and of the variance input channels (CPU).

The simulator splits the total noise-plus-interference variance 1/SINR of a slot into
Gaussian noise and an interferer (QAM symbols z through its own Rayleigh channel g), with
the interferer's share drawn per slot (Sec. IV trains with 10-90 %). The pins: a zero share
reproduces the interferer-free grid bit for bit; a flat, static interferer channel makes the
disturbance rank one across antennas with QAM-valued ratios; Monte Carlo powers match the
configured split; and the variance channels (Sec. II-A) sit where both featurisers put them.
"""
import numpy as np
import pytest

from oracle import featurise as fz
from synth import ofdm as s

BASE = dict(F=48, n_rx=4, bits_per_symbol=4, n_taps=8, max_doppler_hz=300.0, snr_db=6.0, seed=21)


def test_zero_share_reproduces_the_interference_free_grid():
    """Noise is drawn before every interferer draw, so a 0 % share leaves y unchanged."""
    a = s.simulate_slot(s.SimConfig(**BASE), 5)
    b = s.simulate_slot(s.SimConfig(**BASE, interference_share=(0.0, 0.0)), 5)
    np.testing.assert_array_equal(a.y, b.y)
    np.testing.assert_array_equal(a.bits, b.bits)
    assert b.interf_var == 0.0 and b.noise_var == a.noise_var


def test_flat_static_interferer_is_rank_one_with_qam_ratios():
    """All-interference share, one tap, no Doppler: y - h x = g z with g constant over the grid,
    so the disturbance on antenna n over antenna 0 is one constant, and two REs' disturbances on
    one antenna differ by a ratio of two 16-QAM points."""
    cfg = s.SimConfig(F=24, n_rx=3, bits_per_symbol=4, n_taps=1, max_doppler_hz=0.0, snr_db=0.0, seed=22,
                      interference_share=(1.0, 1.0))
    sl = s.simulate_slot(cfg, 0)
    d = sl.y - sl.H * sl.x[..., None]
    r = d[..., 1:] / d[..., :1]
    np.testing.assert_allclose(r, np.broadcast_to(r[0, 0], r.shape), rtol=1e-9, atol=1e-12)
    pts, _ = s.constellation(4)
    ratios = (pts[:, None] / pts[None, :]).ravel()
    q = (d[..., 0] / d[0, 0, 0]).ravel()
    assert np.min(np.abs(q[:, None] - ratios[None, :]), axis=1).max() < 1e-9
    # the interferer's power is g's times the unit-energy constellation's: total = 1 here
    assert sl.interf_var == pytest.approx(1.0) and sl.noise_var == pytest.approx(1.0)


def test_noise_and_interference_powers_follow_the_split():
    """Over many slots: E|y - h x|^2 = 1/SINR, and its interference part has the drawn share."""
    cfg = s.SimConfig(**BASE, interference_share=(0.1, 0.9))
    tot, sh = [], []
    for k in range(160):
        sl = s.simulate_slot(cfg, k)
        tot.append(np.mean(np.abs(sl.y - sl.H * sl.x[..., None]) ** 2) / sl.noise_var)
        sh.append(sl.interf_var / sl.noise_var)
        assert 0.1 <= sh[-1] <= 0.9
    tot, sh = np.array(tot), np.array(sh)
    for arr, target in ((tot, 1.0), (sh, 0.5)):
        se = arr.std(ddof=1) / np.sqrt(len(arr))
        assert abs(arr.mean() - target) < 4 * se, (arr.mean(), target, se)
    # share uniform on [0.1, 0.9]: variance 0.8^2 / 12
    assert abs(sh.var(ddof=1) - 0.64 / 12) < 0.3 * 0.64 / 12


def test_interference_is_not_white_across_antennas():
    """Noise is independent across antennas; a strong interferer through one channel per
    antenna correlates them: the sample covariance of y - h x over one slot is far from
    diagonal at a 90 % share and close to diagonal at 0 %."""
    def offdiag_ratio(share):
        cfg = s.SimConfig(**{**BASE, "n_taps": 1, "max_doppler_hz": 0.0, "F": 96},
                          interference_share=(share, share))
        sl = s.simulate_slot(cfg, 3)
        d = (sl.y - sl.H * sl.x[..., None]).reshape(-1, cfg.n_rx)
        R = d.conj().T @ d / d.shape[0]
        off = np.abs(R - np.diag(np.diag(R))).max()
        return off / np.abs(np.diag(R)).mean()
    assert offdiag_ratio(0.9) > 0.3
    assert offdiag_ratio(0.0) < 0.1


def test_variance_channels_layout_in_both_featurisers():
    cfg = s.SimConfig(**BASE, interference_share=(0.1, 0.9), variance_channels=True)
    sl = s.simulate_slot(cfg, 4)
    N = cfg.n_rx
    X = sl.features
    assert X.shape == (14, cfg.F, 4 * N + s.VARIANCE_CHANNELS)
    sig_n, sig_i = sl.noise_var - sl.interf_var, sl.interf_var
    assert np.all(X[..., 4 * N] == np.float32(sig_n)) and np.all(X[..., 4 * N + 1] == np.float32(sig_i))
    assert np.all(X[..., 4 * N + 2:] == 0)
    # the antenna channels are those of the same slot without variance channels
    plain = s.simulate_slot(s.SimConfig(**BASE, interference_share=(0.1, 0.9)), 4)
    np.testing.assert_array_equal(X[..., :4 * N], plain.features)
    # the oracle featuriser places the variances identically (independent implementation)
    ref = fz.features(sl.y[None], 4 * N + 8, variances=np.array([[sig_n, sig_i]]))
    np.testing.assert_allclose(ref[0], X.astype(np.float64), rtol=2e-7, atol=1e-6 * np.abs(ref).max())
    np.testing.assert_array_equal(ref[0, ..., 4 * N:],
                                  np.broadcast_to([sig_n, sig_i, 0, 0, 0, 0, 0, 0], ref.shape[1:3] + (8,)))


def test_oracle_features_with_variances_zero_pad_between():
    """Fewer antennas than the layout holds: antenna groups, then zeros, then the variances."""
    rng = np.random.default_rng(8)
    y = rng.standard_normal((2, 14, 6, 2)) + 1j * rng.standard_normal((2, 14, 6, 2))
    v = np.array([[0.25, 0.5], [1.5, 0.125]])
    X = fz.features(y, 24, variances=v)
    assert np.all(X[..., 8:16] == 0)
    for b in range(2):
        np.testing.assert_array_equal(X[b, ..., 16], np.full((14, 6), v[b, 0]))
        np.testing.assert_array_equal(X[b, ..., 17], np.full((14, 6), v[b, 1]))
    assert np.all(X[..., 18:] == 0)
    np.testing.assert_array_equal(X[..., :8], fz.features(y, 8))
