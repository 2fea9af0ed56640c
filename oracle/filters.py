"""Oracle band-pass filtering of signals and model columns (TEST INFRASTRUCTURE ONLY).

The paper band-pass filters the raw signals and the model matrix before inversion (Results:
0.5-80 MHz for the simulated pairs; Methods, in vivo imaging: 1-120 MHz) without naming the
filter.  Reading used here: a zero-phase FIR band-pass designed by the window method,

    h[m] = w[m] * ( (2 f_hi / fs) sinc(2 f_hi m / fs) - (2 f_lo / fs) sinc(2 f_lo m / fs) ),
    w[m] = 0.42 + 0.5 cos(pi m / L) + 0.08 cos(2 pi m / L)          (Blackman),  |m| <= L,

with sinc(u) = sin(pi u) / (pi u), applied along time as a linear convolution truncated to
the record [0, Nt):

    y[n] = sum_{m in [0, Nt), |n - m| <= L} h[n - m] x[m].

The same filter F acts on every signal and on every model column, so the filtered model is
F A (a column with window [lo, hi] gets the window [lo - L, hi + L] clipped to [0, Nt)).
With 2L + 1 taps, band edges below about fs / (2L) are only approximated (the lower edge of
0.5 MHz leaves a DC gain of about 0.89 at L = 32 and 250 MHz).
FP64 throughout.
"""
from __future__ import annotations

import math

import numpy as np


def bandpass_taps(f_lo_hz, f_hi_hz, fs_hz, half_taps):
    """The 2L + 1 taps h[-L..L] of the windowed-sinc band-pass."""
    L = int(half_taps)
    m = np.arange(-L, L + 1, dtype=np.float64)
    lo, hi = 2.0 * f_lo_hz / fs_hz, 2.0 * f_hi_hz / fs_hz
    ideal = hi * np.sinc(hi * m) - lo * np.sinc(lo * m)
    if L == 0:
        return ideal
    w = 0.42 + 0.5 * np.cos(math.pi * m / L) + 0.08 * np.cos(2.0 * math.pi * m / L)
    return w * ideal


def filter_time(x, h):
    """Truncated linear convolution of every trace of x (last axis = time) with the centred
    taps h (length 2L + 1), written out as a sum over taps."""
    x = np.asarray(x, dtype=np.float64)
    L = (len(h) - 1) // 2
    nt = x.shape[-1]
    y = np.zeros_like(x)
    for j, hj in enumerate(h):
        d = j - L                          # y[n] += h[d] x[n - d]
        if d >= 0:
            y[..., d:] += hj * x[..., :nt - d] if d < nt else 0.0
        else:
            y[..., :nt + d] += hj * x[..., -d:] if -d < nt else 0.0
    return y


def filtered_table(H, h):
    """The filtered model F A: every column H[dy, dx, k, :] filtered along time."""
    return filter_time(H, h)


def filtered_supports(lo, hi, half_taps, nt):
    """Column windows of the filtered model: [lo - L, hi + L] clipped to [0, nt)."""
    lo = np.asarray(lo)
    hi = np.asarray(hi)
    act = lo >= 0
    flo = np.where(act, np.maximum(lo - half_taps, 0), -1)
    fhi = np.where(act, np.minimum(hi + half_taps, nt - 1), -1)
    return flo, fhi
