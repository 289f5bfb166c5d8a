"""Pins of the OFDM simulator and the classical receiver (CPU).

Closed forms (QAM energy, Gray labelling, exact QPSK LLRs, MRC over Rayleigh),
special cases (noiseless recovery, exact LS at pilots, linear channels) and
Monte Carlo statistics of the channel and noise.
"""
import numpy as np
import pytest

from oracle import classical as c
from synth import ofdm as s


@pytest.mark.parametrize("m", [2, 4, 6, 8])
def test_qam_unit_energy_and_gray(m):
    pts, labels = s.constellation(m)
    assert abs(np.mean(np.abs(pts) ** 2) - 1.0) < 1e-15
    assert len(np.unique(np.round(pts, 12))) == (1 << m)
    d = np.abs(pts[:, None] - pts[None, :])
    dmin = d[d > 1e-12].min()
    for i in range(len(pts)):
        for j in range(len(pts)):
            if i != j and abs(d[i, j] - dmin) < 1e-9:
                assert int(np.sum(labels[i] != labels[j])) == 1     # nearest neighbours: 1 bit


def test_qpsk_closed_form():
    bits = np.array([[0, 0], [1, 0], [0, 1], [1, 1]])
    exp = ((1 - 2 * bits[:, 0]) + 1j * (1 - 2 * bits[:, 1])) / np.sqrt(2)
    np.testing.assert_allclose(s.qam_map(bits), exp, atol=1e-15)


def test_16qam_levels_follow_nr_table():
    """16-QAM: I = (1-2b0)(2-(1-2b2))/sqrt(10), Q = (1-2b1)(2-(1-2b3))/sqrt(10)."""
    rng = np.random.default_rng(0)
    b = rng.integers(0, 2, (64, 4))
    exp = ((1 - 2 * b[:, 0]) * (2 - (1 - 2 * b[:, 2])) + 1j * (1 - 2 * b[:, 1]) * (2 - (1 - 2 * b[:, 3]))) / np.sqrt(10)
    np.testing.assert_allclose(s.qam_map(b), exp, atol=1e-15)


def test_oracle_and_synth_constellations_agree():
    for m in (2, 4, 6, 8):
        p1, l1 = s.constellation(m)
        p2, l2 = c.constellation(m)
        np.testing.assert_array_equal(l1, l2)
        np.testing.assert_allclose(p1, p2, atol=1e-15)


def test_pilot_pattern():
    pm = s.pilot_mask(14, 72)
    assert pm.sum() == 2 * 36
    assert pm[2, 0] and pm[11, 70] and not pm[2, 1] and not pm[3, 0]
    assert s.data_mask(14, 72).sum() == 13 * 72


def test_noiseless_ls_exact_at_pilots_and_perfect_csi_recovers_bits():
    cfg = s.SimConfig(F=72, n_rx=2, bits_per_symbol=4, n_taps=4, max_doppler_hz=0, snr_db=10, seed=3)
    sl = s.simulate_slot(cfg, 0, noise_var_override=0.0)
    pm = s.pilot_mask(14, 72)
    np.testing.assert_allclose(sl.H_ls[pm], sl.H[pm], atol=1e-12)
    llr = c.classical_rx(sl.y, sl.H, 1e-12, 4)
    dm = s.data_mask(14, 72)
    assert np.array_equal(c.hard_bits(llr)[dm], sl.bits[dm])


def test_flat_static_channel_interpolates_exactly():
    cfg = s.SimConfig(F=24, n_rx=2, bits_per_symbol=2, n_taps=1, max_doppler_hz=0, snr_db=10, seed=4)
    sl = s.simulate_slot(cfg, 0, noise_var_override=0.0)
    np.testing.assert_allclose(sl.H_ls, sl.H, atol=1e-12)


def test_channel_linear_in_time_is_reproduced():
    T, F, N = 14, 20, 2
    t = np.arange(T)[:, None, None]
    H = (0.3 + 0.2j) + (0.05 - 0.01j) * t + np.zeros((T, F, N))
    H[..., 1] *= -1.3
    cfg = s.SimConfig(F=F, n_rx=N, bits_per_symbol=2, n_taps=1, max_doppler_hz=0, snr_db=10, seed=5)
    sl = s.simulate_slot(cfg, 0, noise_var_override=0.0, channel_override=H)
    np.testing.assert_allclose(sl.H_ls, H, atol=1e-12)


def test_features_layout():
    cfg = s.SimConfig(F=12, n_rx=3, bits_per_symbol=2, n_taps=2, max_doppler_hz=100, snr_db=5, seed=6)
    sl = s.simulate_slot(cfg, 2)
    X = sl.features
    assert X.shape == (14, 12, 12) and X.dtype == np.float32
    np.testing.assert_array_equal(X[..., 4 * 1 + 1], sl.y[..., 1].imag.astype(np.float32))
    np.testing.assert_array_equal(X[..., 4 * 2 + 2], sl.H_ls[..., 2].real.astype(np.float32))


def test_slot_regenerates_alone():
    cfg = s.SimConfig(F=24, n_rx=2, bits_per_symbol=4, seed=7)
    X, bits, _, _ = s.simulate_batch(cfg, 3)
    sl = s.simulate_slot(cfg, 2)
    np.testing.assert_array_equal(X[2], sl.features)
    np.testing.assert_array_equal(bits[2], sl.bits)


@pytest.mark.parametrize("m", [2, 4, 6])
def test_maxlog_equals_bruteforce_definition_and_qpsk_closed_form(m):
    rng = np.random.default_rng(8)
    h = (rng.standard_normal((50, 3)) + 1j * rng.standard_normal((50, 3))) / np.sqrt(2)
    y = (rng.standard_normal((50, 3)) + 1j * rng.standard_normal((50, 3)))
    nv = 0.3
    llr = c.classical_rx(y, h, nv, m)
    if m == 2:
        hy = np.sum(np.conj(h) * y, axis=-1)
        exp = np.stack([-2 * np.sqrt(2) * hy.real / nv, -2 * np.sqrt(2) * hy.imag / nv], axis=-1)
        np.testing.assert_allclose(llr, exp, rtol=1e-10, atol=1e-12)
    pts, labels = s.constellation(m)
    for r in range(0, 50, 7):   # loop form of the max-log definition on a few REs
        z = np.sum(np.conj(h[r]) * y[r]) / np.sum(np.abs(h[r]) ** 2)
        ne = nv / np.sum(np.abs(h[r]) ** 2)
        for i in range(m):
            d0 = min(abs(z - p) ** 2 for p, l in zip(pts, labels) if l[i] == 0)
            d1 = min(abs(z - p) ** 2 for p, l in zip(pts, labels) if l[i] == 1)
            assert abs(llr[r, i] - (d0 - d1) / ne) < 1e-9 * max(1, abs(llr[r, i]))


def test_channel_power_and_noise_variance():
    cfg = s.SimConfig(F=96, n_rx=2, bits_per_symbol=2, n_taps=8, max_doppler_hz=400, snr_db=3.0, seed=9)
    Hs, ns = [], []
    for k in range(200):
        sl = s.simulate_slot(cfg, k)
        Hs.append(np.mean(np.abs(sl.H) ** 2))
        ns.append(np.mean(np.abs(sl.y - sl.H * sl.x[..., None]) ** 2))
    Hs, ns = np.array(Hs), np.array(ns)
    for arr, target in ((Hs, 1.0), (ns, 10 ** (-0.3))):
        se = arr.std(ddof=1) / np.sqrt(len(arr))
        assert abs(arr.mean() - target) < 4 * se, (arr.mean(), target, se)


def test_jakes_time_correlation():
    fd = 300.0
    R = s.jakes_covariance(14, fd)
    rng = np.random.default_rng(10)
    n = 40000
    w = (rng.standard_normal((n, 14)) + 1j * rng.standard_normal((n, 14))) / np.sqrt(2)
    g = s.correlated_gains(w, R)
    emp = (g.conj().T @ g / n).real
    # MC error of a CN(0,1) correlation estimate is about 1/sqrt(n)
    assert np.abs(emp - R).max() < 4 * np.sqrt(1.0 / n) * 1.5
    from scipy.special import j0
    assert abs(R[0, 5] - j0(2 * np.pi * fd * 5 * s.SYMBOL_PERIOD_S)) < 1e-15


@pytest.mark.parametrize("N,snr_db", [(1, 6.0), (2, 4.0)])
def test_qpsk_mrc_rayleigh_ber_matches_textbook(N, snr_db):
    """Whole simulator + classical receiver (perfect CSI) vs Proakis' MRC closed form."""
    cfg = s.SimConfig(F=48, n_rx=N, bits_per_symbol=2, n_taps=8, max_doppler_hz=400, snr_db=snr_db, seed=11)
    dm = s.data_mask(14, 48)
    per_slot = []
    for k in range(800):
        sl = s.simulate_slot(cfg, k)
        llr = c.classical_rx(sl.y, sl.H, sl.noise_var, 2)
        per_slot.append(np.mean((c.hard_bits(llr) != sl.bits)[dm]))
    per_slot = np.array(per_slot)
    est, se = per_slot.mean(), per_slot.std(ddof=1) / np.sqrt(len(per_slot))
    theory = c.mrc_rayleigh_ber(10 ** (snr_db / 10) / 2, N)
    assert abs(est - theory) < 3.0 * se, (est, theory, se)   # 99.7 % MC interval


def test_snr_gap():
    snr = np.arange(0, 11.0)
    ber_a = 10 ** (-(snr - 2.0) / 3.0)
    ber_b = 10 ** (-snr / 3.0)
    assert abs(c.snr_gap_db(snr, ber_a, ber_b, 1e-2) - 2.0) < 1e-9
