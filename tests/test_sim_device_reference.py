"""Pins of the counter-based slot generator (synth.devsim), the host reference of the GPU's
on-device simulator (CPU).

Philox4x32-10 against the known-answer vectors published with the generator (Salmon et al.,
SC 2011); the uniform and Box-Muller maps against their moments; the slot model against what
it must satisfy: unit channel power, the drawn noise variance, Clarke's time correlation
J0(2 pi f_D T_sym dt) for each slot's Doppler, QAM symbols and pilots where synth.ofdm puts them."""
import numpy as np
import pytest
from scipy.special import j0

from synth import devsim as d
from synth import ofdm as s


@pytest.mark.parametrize("ctr,key,want", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, want):
    got = d.philox4x32_10(np.array([ctr], dtype=np.uint32), key)[0]
    assert tuple(int(v) for v in got) == want


def test_uniform_and_normal_maps():
    w = d.draws(7, 0, 9, 200000)
    u = d.uniform(w[:, 0])
    assert u.min() > 0 and u.max() < 1
    assert np.all(u.astype(np.float32).astype(np.float64) == u)      # exact in FP32
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / u.size) and abs(u.var() - 1 / 12) < 2e-3
    z = d.cnormal(w[:, 0], w[:, 1])
    n = z.size
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 4 * np.sqrt(1.0 / n)
    assert abs(np.mean(z)) < 4 * np.sqrt(1.0 / n) and abs(np.mean(z * z)) < 4 * np.sqrt(2.0 / n)


def test_counters_separate_slots_and_streams():
    a, b = d.draws(1, 5, 2, 64), d.draws(1, 6, 2, 64)
    c = d.draws(1, 5, 3, 64)
    assert not np.any(np.all(a == b, axis=1)) and not np.any(np.all(a == c, axis=1))
    np.testing.assert_array_equal(a[10:20], d.draws(1, 5, 2, 20)[10:20])   # a draw depends on its counter only


def test_symbols_bits_and_pilots():
    cfg = d.DevSimConfig(F=30, n_rx=2, bits_per_symbol=6, seed=3, snr_lo_db=200.0, snr_hi_db=200.0)
    y, bits, H, nv = d.simulate(cfg, 4)
    x = y[..., 0] / H[..., 0]                      # noiseless at 200 dB
    pm = s.pilot_mask(14, 30)
    np.testing.assert_allclose(x[pm], s.PILOT_VALUE, atol=1e-9)
    np.testing.assert_allclose(x[~pm], s.qam_map(bits)[~pm], atol=1e-9)
    assert abs(bits.mean() - 0.5) < 0.05


def test_channel_power_noise_variance_and_time_correlation():
    cfg = d.DevSimConfig(F=48, n_rx=2, bits_per_symbol=2, seed=11, max_doppler_hz=400.0)
    pw, nz, acc, ref = [], [], np.zeros(14), np.zeros(14)
    for k in range(120):
        y, bits, H, nv = d.simulate(cfg, k)
        pw.append(np.mean(np.abs(H) ** 2))
        x = np.where(s.pilot_mask(14, 48), s.PILOT_VALUE, s.qam_map(bits))
        nz.append(np.mean(np.abs(y - H * x[..., None]) ** 2) / nv)
        # time correlation of the channel at lag dt, against J0 at this slot's Doppler
        fd, _ = d.slot_params(cfg, k)
        acc += np.array([np.mean((H[dt:] * np.conj(H[:14 - dt])).real) for dt in range(14)])
        ref += j0(2 * np.pi * fd * s.SYMBOL_PERIOD_S * np.arange(14))
    pw, nz = np.array(pw), np.array(nz)
    assert abs(pw.mean() - 1.0) < 4 * pw.std(ddof=1) / np.sqrt(len(pw))
    assert abs(nz.mean() - 1.0) < 0.01
    corr, want = acc / 120, ref / 120
    assert np.abs(corr - want).max() < 0.12, (corr, want)
    assert corr[13] < corr[0] - 0.05        # the channel does vary over the slot


def test_noise_variance_follows_the_snr_draw():
    cfg = d.DevSimConfig(F=8, n_rx=1, bits_per_symbol=2, seed=2, snr_lo_db=-5.0, snr_hi_db=25.0)
    snrs = np.array([d.slot_params(cfg, k)[1] for k in range(2000)])
    assert snrs.min() >= -5 and snrs.max() <= 25 and abs(snrs.mean() - 10) < 0.5
    _, _, _, nv = d.simulate(cfg, 17)
    assert nv == pytest.approx(10 ** (-d.slot_params(cfg, 17)[1] / 10))
