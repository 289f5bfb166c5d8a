"""FP64 oracle of the receiver's input features (test infrastructure only).

Plain and slow, to be read against the paper: the network's input is the received grid
of one TTI (Sec. II, Eq. (1)) split into real and imaginary channels (Sec. II-A), next to a
least-squares channel estimate formed at the fixed pilots and interpolated linearly over
the grid (Sec. I names LS estimation with interpolation as the conventional front end).

Readings (listed in the design notes): pilots on symbols 2 and 11 (0-based), even
subcarriers, value (1+j)/sqrt(2); along a pilot symbol an odd subcarrier takes the mean
of its two even neighbours and a last odd subcarrier copies the one to its left; over
time every symbol lies on the straight line through the two pilot symbols.
"""
from __future__ import annotations

import numpy as np

PILOT_SYMBOLS = (2, 11)
PILOT = (1.0 + 1.0j) / np.sqrt(2.0)


def pilot_estimate(row: np.ndarray) -> np.ndarray:
    """LS estimate along one pilot symbol. row: (F, N) received samples -> (F, N)."""
    F = row.shape[0]
    h = np.empty(row.shape, dtype=np.complex128)
    for f in range(F):
        if f % 2 == 0:
            h[f] = row[f] / PILOT
        elif f + 1 < F:
            h[f] = 0.5 * (row[f - 1] / PILOT + row[f + 1] / PILOT)
        else:
            h[f] = row[f - 1] / PILOT
    return h


def channel_estimate(y: np.ndarray) -> np.ndarray:
    """y: (T, F, N) complex received grid of one slot -> (T, F, N) interpolated estimate."""
    T = y.shape[0]
    t0, t1 = PILOT_SYMBOLS
    h0, h1 = pilot_estimate(y[t0]), pilot_estimate(y[t1])
    out = np.empty(y.shape, dtype=np.complex128)
    for t in range(T):
        out[t] = h0 + (t - t0) / (t1 - t0) * (h1 - h0)
    return out


def features(y: np.ndarray, C_in: int, variances=None) -> np.ndarray:
    """y: (B, T, F, N) complex -> (B, T, F, C_in) float64 with channels 4n..4n+3 =
    (Re y_n, Im y_n, Re H_n, Im H_n) and zeros for antennas n >= N. With variances (B, 2) --
    the known noise and interference variances, which Sec. II-A concatenates with the
    received grid -- channels C_in - 8 and C_in - 7 hold them for every RE of the slot and
    C_in - 6 .. C_in - 1 are zero."""
    B, T, F, N = y.shape
    X = np.zeros((B, T, F, C_in), dtype=np.float64)
    if variances is not None:
        v = np.asarray(variances, dtype=np.float64)
        X[:, :, :, C_in - 8] = v[:, 0][:, None, None]
        X[:, :, :, C_in - 7] = v[:, 1][:, None, None]
    for b in range(B):
        H = channel_estimate(y[b])
        for n in range(N):
            X[b, :, :, 4 * n + 0] = y[b, :, :, n].real
            X[b, :, :, 4 * n + 1] = y[b, :, :, n].imag
            X[b, :, :, 4 * n + 2] = H[:, :, n].real
            X[b, :, :, 4 * n + 3] = H[:, :, n].imag
    return X
