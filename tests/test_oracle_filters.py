"""Pins of the oracle's band-pass filter: the taps are SciPy's window-method design, the
filtering is NumPy's linear convolution cut to the record, the frequency response has the
band edges the design asks for, and filtering the model commutes with the operators
(F A x = A_f x and A_f^T y = A^T F y, since the centred taps are symmetric)."""
import numpy as np
import pytest
import scipy.signal as ss

import workloads as W
from oracle import filters, model, operators


@pytest.mark.parametrize("f_lo,f_hi,L", [(0.5e6, 80e6, 32), (1e6, 120e6, 24), (10e6, 60e6, 40)])
def test_taps_are_the_window_method_design(f_lo, f_hi, L):
    h = filters.bandpass_taps(f_lo, f_hi, 250e6, L)
    ref = ss.firwin(2 * L + 1, [f_lo, f_hi], pass_zero=False, window="blackman", scale=False,
                    fs=250e6)
    assert np.max(np.abs(h - ref)) <= 1e-15
    assert np.array_equal(h, h[::-1])          # zero phase


def test_filter_is_truncated_linear_convolution():
    h = filters.bandpass_taps(0.5e6, 80e6, 250e6, 32)
    x = W.rng(4).standard_normal((3, 5, 100))
    y = filters.filter_time(x, h)
    ref = np.apply_along_axis(lambda r: np.convolve(r, h)[32:132], -1, x)
    assert np.max(np.abs(y - ref)) <= 1e-13
    # records shorter than the filter
    xs = x[..., :20]
    ref = np.apply_along_axis(lambda r: np.convolve(r, h)[32:52], -1, xs)
    assert np.max(np.abs(filters.filter_time(xs, h) - ref)) <= 1e-13


def test_frequency_response_band_edges():
    """0.5-80 MHz at 250 MHz with 65 taps: unit gain mid-band, -6 dB at the upper edge
    (window method), Blackman stop-band below 1e-3 beyond the transition band, and the
    lower edge only approximated by a filter this short."""
    h = filters.bandpass_taps(0.5e6, 80e6, 250e6, 32)
    m = np.arange(-32, 33)
    gain = lambda f: abs(np.sum(h * np.exp(-2j * np.pi * f / 250e6 * m)))
    _, H = ss.freqz(h, worN=[50e6, 80e6, 100e6], fs=250e6)
    assert np.allclose(np.abs(H), [gain(50e6), gain(80e6), gain(100e6)], rtol=1e-12)
    assert abs(gain(50e6) - 1) < 1e-4
    assert abs(gain(80e6) - 0.5) < 1e-4
    assert gain(100e6) < 1e-3 and gain(120e6) < 1e-4
    assert 0.85 < gain(0.0) < 0.95


@pytest.fixture(scope="module")
def small():
    cfg = W.config("tiny")
    g = W.grid(6, 10e-6, 8, 10e-6, 64, 2, 1, ny=5)
    H = model.build_table(cfg["sensor"], g)
    return cfg, g, H


def test_filtered_model_commutes_with_operators(small):
    cfg, g, H = small
    h = filters.bandpass_taps(0.5e6, 80e6, g["fs_hz"], 12)
    Hf = filters.filtered_table(H, h)
    rng = W.rng(8)
    x = rng.standard_normal((g["ny"], g["nx"], g["nz"]))
    y = rng.standard_normal((g["ny"], g["nx"], g["nt"]))
    s = operators.forward(Hf, x)
    assert np.allclose(s, filters.filter_time(operators.forward(H, x), h), rtol=0,
                       atol=1e-13 * np.abs(s).max())
    xa = operators.adjoint(Hf, y)
    assert np.allclose(xa, operators.adjoint(H, filters.filter_time(y, h)), rtol=0,
                       atol=1e-13 * np.abs(xa).max())


def test_filtered_supports_bound_the_filtered_columns(small):
    cfg, g, H = small
    L = 12
    Hf = filters.filtered_table(H, filters.bandpass_taps(0.5e6, 80e6, g["fs_hz"], L))
    lo, hi = operators.supports(cfg["sensor"], g)
    flo, fhi = filters.filtered_supports(lo, hi, L, g["nt"])
    n = np.arange(g["nt"])
    outside = (n < flo[..., None]) | (n > fhi[..., None])
    assert not np.any(Hf[outside])
    assert np.array_equal(flo >= 0, lo >= 0)
    assert np.all((fhi - flo)[lo >= 0] <= (hi - lo)[lo >= 0] + 2 * L)
