"""Host logic: the seeded synthetic inputs follow their stated recipe (Poisson serving trace
with a 70 / 30 LSQR / FISTA mix over both sensors, request configurations with a tube count
proportional to the scan area, vessel phantoms and unit Gaussian noise), and the same seed
always gives the same input."""
import numpy as np

import workloads as W


def test_serving_trace_is_a_seeded_poisson_mix():
    sides, nzs = (64, 96, 128), (64, 128)
    a = W.serve_trace(4000, 2.0, 7, sides=sides, nzs=nzs)
    assert a == W.serve_trace(4000, 2.0, 7, sides=sides, nzs=nzs)
    assert a != W.serve_trace(4000, 2.0, 8, sides=sides, nzs=nzs)
    t = np.array([r["arrival_s"] for r in a])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    # exponential gaps: mean 1 / rate, coefficient of variation 1 (4000 draws: ~1.6 % s.e.)
    assert abs(gaps.mean() - 0.5) < 0.5 * 0.06
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.06
    lsqr = np.mean([r["kind"] == "lsqr" for r in a])
    four = np.mean([r["sensor"] == "4mm" for r in a])
    assert abs(lsqr - 0.7) < 0.03 and abs(four - 0.5) < 0.03
    assert {r["side"] for r in a} == set(sides) and {r["nz"] for r in a} == set(nzs)
    assert all(r["nt"] == 4 * r["nz"] and 15.0 <= r["snr_db"] <= 30.0 for r in a)
    assert [r["id"] for r in a] == list(range(4000))


def test_request_configuration_scales_the_phantom_with_the_area():
    req = dict(side=200, nz=64, nt=256, sensor="7mm", kind="fista", snr_db=20.0)
    cfg = W.serve_config(req)
    g = cfg["grid"]
    assert (g["nx"], g["ny"], g["nz"], g["nt"], g["k_half"]) == (200, 200, 64, 256, 20)
    assert cfg["phantom"]["n"] == 40 and cfg["solver"]["kind"] == "fista"
    assert cfg["sensor"]["hole_m"] > 0                      # the 7 mm sensor has its hole
    small = W.serve_config(dict(req, side=64, sensor="4mm", kind="lsqr"))
    assert small["phantom"]["n"] == max(2, round(40 * 64 * 64 / 200 ** 2))
    assert small["solver"]["kind"] == "lsqr" and small["sensor"]["hole_m"] == 0


def test_phantoms_and_noise_are_seeded_and_in_range():
    cfg = W.config("mid")
    g = cfg["grid"]
    p = W.make_phantom(cfg, 3)
    assert p.shape == (g["ny"], g["nx"], g["nz"])
    assert np.array_equal(p, W.make_phantom(cfg, 3))
    assert not np.array_equal(p, W.make_phantom(cfg, 4))
    lo, hi = cfg["phantom"]["amp"]
    vals = p[p != 0]
    assert vals.size > 0 and vals.min() >= lo and vals.max() <= hi
    n = W.unit_noise(cfg, 3)
    assert n.shape == (g["ny"], g["nx"], g["nt"])
    assert np.array_equal(n, W.unit_noise(cfg, 3))
    assert abs(n.mean()) < 0.01 and abs(n.std() - 1.0) < 0.01
