"""Host-side figures of merit of the super-resolution evaluation (Fig. 2b): FWHM by linear
interpolation and the valley depth between two peaks, pinned to closed forms."""
import math

import numpy as np

from paper_2009_10173_amd import superres as S


def test_fwhm_of_triangle_is_exact():
    i = np.arange(41)
    p = np.maximum(0.0, 1.0 - 0.1 * np.abs(i - 20))      # half maximum 5 samples either side
    assert abs(S.fwhm(p, 20, 2.5) - 10 * 2.5) < 1e-12


def test_fwhm_of_gaussian():
    sigma = 4.0
    i = np.arange(81)
    p = np.exp(-0.5 * ((i - 40) / sigma) ** 2)
    assert abs(S.fwhm(p, 40, 1.0) - 2 * math.sqrt(2 * math.log(2)) * sigma) < 0.02 * sigma
    assert S.fwhm(np.ones(10), 5, 1.0) is None           # never drops to half


def _two(d, sigma=3.0, n=121):
    i = np.arange(n, dtype=np.float64)
    c = (n - 1) / 2
    return np.exp(-0.5 * ((i - c + d / 2) / sigma) ** 2) + np.exp(-0.5 * ((i - c - d / 2) / sigma) ** 2)


def test_dip_closed_forms():
    # peaks at +-d/2 = +-2 sigma: valley 2 exp(-2) against peaks 1 + exp(-8)
    p = _two(12.0)
    a, b = S.pair_peaks(p, 54, 66, 3)
    assert (a, b) == (54, 66)
    assert abs(S.dip(p, a, b) - (1 - 2 * math.exp(-2) / (1 + math.exp(-8)))) < 1e-12
    # two Gaussians closer than 2 sigma merge into one peak: no valley
    p = _two(5.0)
    a, b = S.pair_peaks(p, 57, 63, 2)
    assert S.dip(p, a, b) == 0.0
    # disjoint boxes: the valley reaches zero
    q = np.zeros(30)
    q[5:9] = 1.0
    q[20:24] = 0.5
    assert S.dip(q, 6, 21) == 1.0


def test_evaluate_on_phantom_itself():
    """The phantom's own projection: two 20 um balls 40 um apart are resolved (zeros between
    them), each 25 um wide at half maximum on the 5 um grid (5 voxels across the ball's
    centre row; the half-maximum crossings fall half-way to the empty neighbours)."""
    import workloads as W
    cfg = W.config("superres40")
    r = S.evaluate(W.make_phantom(cfg, 0), cfg)
    assert r["resolved"] and r["dip"] == 1.0
    assert r["separation_um"] == 40.0
    assert r["fwhm_um"] == [25.0, 25.0]
