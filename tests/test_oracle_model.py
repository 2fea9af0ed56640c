"""Pins of the oracle's model (sensor discretisation, EIR, table) to facts fixed
independently of the oracle: closed forms, exact areas, symmetry, the paper's constants."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import model, operators

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(scope="module")
def tiny():
    cfg = W.config("tiny")
    H = model.build_table(cfg["sensor"], cfg["grid"])
    return cfg, H


# --- sensor sub-elements (Eq. 3) -------------------------------------------------------

@pytest.mark.parametrize("sensor", [W.SENSOR_4MM, W.SENSOR_7MM])
def test_elements_total_area_is_cap_area(sensor):
    pos, area = model.sensor_elements(sensor)
    R = sensor["radius_m"] * 1e3
    th_h = math.asin(sensor["hole_m"] / (2 * sensor["radius_m"]))
    th_m = math.asin(sensor["aperture_m"] / (2 * sensor["radius_m"]))
    cap = 2 * math.pi * R * R * (math.cos(th_h) - math.cos(th_m))
    assert abs(area.sum() - cap) / cap < 1e-14
    # every centre lies on the sphere about the focus, inside the annulus, above the focus
    r = np.linalg.norm(pos, axis=1)
    assert np.max(np.abs(r - R)) / R < 1e-14
    polar = np.arccos(-pos[:, 2] / r)
    assert np.all(polar > th_h) and np.all(polar < th_m)


@pytest.mark.parametrize("sensor", [W.SENSOR_4MM, W.SENSOR_7MM])
def test_elements_square_symmetric(sensor):
    pos, area = model.sensor_elements(sensor)

    def canon(p):
        keys = np.round(p / 1e-9).astype(np.int64)
        return keys[np.lexsort(keys.T[::-1])]

    ref = canon(pos)
    for T in ([[0, -1, 0], [1, 0, 0], [0, 0, 1]],     # rotation by 90 degrees
              [[1, 0, 0], [0, -1, 0], [0, 0, 1]],     # mirror y
              [[0, 1, 0], [1, 0, 0], [0, 0, 1]]):     # swap x, y
        assert np.array_equal(canon(pos @ np.array(T, float).T), ref)


def test_element_count_matches_paper():
    consts = {r[0]: float(r[1]) for r in _golden_rows("setup_constants.txt")}
    s7 = W.SENSOR_7MM
    assert s7["radius_m"] == consts["radius_m"] and s7["hole_m"] == consts["hole_m"]
    assert abs(s7["aperture_m"] / (2 * s7["radius_m"]) - consts["na"]) < 1e-15
    _, area = model.sensor_elements(s7)
    assert len(area) == int(consts["sub_elements"])
    # the 4 mm sensor's default discretisation stays in the paper's ~1000-1200 range
    assert 1000 <= len(model.sensor_elements(W.SENSOR_4MM)[1]) <= 1300


# --- electrical impulse response -------------------------------------------------------

def test_eir_spectrum_matches_analytic_transform():
    cfg = W.config("tiny")
    sig, om = model.eir_params(cfg["sensor"], cfg["grid"])
    h = 1.0 / 64
    tau = np.arange(-40 * sig, 40 * sig, h)
    e = model.eir(tau, sig, om)
    Om = np.linspace(0.0, np.pi, 97)              # rad / sample, up to Nyquist
    num = np.array([np.sum(e * np.cos(w * tau)) * h for w in Om])
    ana = (sig * math.sqrt(2 * math.pi) / 2
           * (np.exp(-sig ** 2 * (Om - om) ** 2 / 2) + np.exp(-sig ** 2 * (Om + om) ** 2 / 2)))
    assert np.max(np.abs(num - ana)) < 1e-10 * np.max(ana)


def test_eir_bandwidth_is_100_percent_at_50mhz():
    cfg = W.config("tiny")
    s, g = cfg["sensor"], cfg["grid"]
    sig, om = model.eir_params(s, g)
    fs = g["fs_hz"]
    h = 1.0 / 64
    tau = np.arange(-40 * sig, 40 * sig, h)
    e = model.eir(tau, sig, om)

    def amp(f_hz):
        w = 2 * math.pi * f_hz / fs
        return abs(np.sum(e * np.exp(-1j * w * tau)) * h)

    f0 = s["f0_hz"]
    peak = amp(f0)
    # -6 dB amplitude points at f0 (1 -/+ bw/2) = 25 / 75 MHz; the negative-frequency image
    # of the cosine adds ~2e-3 at the lower edge.
    assert abs(amp(25e6) / peak - 0.5) < 3e-3
    assert abs(amp(75e6) / peak - 0.5) < 3e-3
    fgrid = np.linspace(30e6, 70e6, 401)
    assert abs(fgrid[np.argmax([amp(f) for f in fgrid])] - f0) <= 0.2e6


def test_eir_derivative_matches_finite_difference():
    sig, om = model.eir_params(W.SENSOR_4MM, W.config("tiny")["grid"])
    tau = np.linspace(-6 * sig, 6 * sig, 301)
    h = 1e-5
    fd = (model.eir(tau + h, sig, om) - model.eir(tau - h, sig, om)) / (2 * h)
    assert np.max(np.abs(fd - model.eir_derivative(tau, sig, om))) < 1e-8


# --- the model table --------------------------------------------------------------------

def test_focal_voxel_closed_form(tiny):
    """At the sphere's centre every sub-element is at distance R, so the spatial impulse
    response is (cap area / (2 pi R)) delta(t - R/c): H = R (cos th_h - cos th_m) e'(n - Nt/2)."""
    cfg, H = tiny
    s, g = cfg["sensor"], cfg["grid"]
    K, nz, nt = g["k_half"], g["nz"], g["nt"]
    sig, om = model.eir_params(s, g)
    R = s["radius_m"] * 1e3
    th_m = math.asin(s["aperture_m"] / (2 * s["radius_m"]))
    n = np.arange(nt) - nt // 2
    ref = R * (1 - math.cos(th_m)) * model.eir_derivative(n, sig, om)
    ref[np.abs(n) > 5 * sig] = 0
    got = H[K, K, nz // 2]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_focal_voxel_closed_form_with_hole():
    cfg = W.config("mid7")
    s, g = cfg["sensor"], cfg["grid"]
    elems = model.sensor_elements(s)
    got = model.column(s, g, elems, 0, 0, g["nz"] // 2)
    sig, om = model.eir_params(s, g)
    R = s["radius_m"] * 1e3
    th_h, th_m = model.sensor_angles(s)
    n = np.arange(g["nt"]) - g["nt"] // 2
    ref = R * (math.cos(th_h) - math.cos(th_m)) * model.eir_derivative(n, sig, om)
    ref[np.abs(n) > 5 * sig] = 0
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def _on_axis_exact(s, g, z_mm):
    """Continuous on-axis response: the spatial impulse response of a spherical cap for an
    on-axis point at depth z is c R / |z| on [r_lo/c, r_hi/c] (r^2 = R^2 + z^2 + 2 R z cos th),
    so its convolution with e' is (c R / (|z| fs)) [e(tau_lo) - e(tau_hi)] in samples."""
    sig, om = model.eir_params(s, g)
    R = s["radius_m"] * 1e3
    th_h, th_m = model.sensor_angles(s)
    rr = [math.sqrt(R * R + z_mm * z_mm + 2 * R * z_mm * math.cos(t)) for t in (th_h, th_m)]
    r_lo, r_hi = min(rr), max(rr)
    cfs = g["c_mps"] * 1e3 / g["fs_hz"]
    n = np.arange(g["nt"]) - g["nt"] // 2
    t_lo = n - (r_lo - R) / cfs
    t_hi = n - (r_hi - R) / cfs
    return (cfs * R / abs(z_mm)) * (model.eir(t_lo, sig, om) - model.eir(t_hi, sig, om))


@pytest.mark.parametrize("k_off", [5, -16])
def test_on_axis_closed_form_second_order(k_off):
    cfg = W.config("tiny")
    s, g = cfg["sensor"], cfg["grid"]
    k = g["nz"] // 2 + k_off
    z = model.depths_mm(g)[k]
    exact = _on_axis_exact(s, g, z)
    errs = []
    for nr in (20, 40, 80):
        col = model.column(s, g, model.sensor_elements(s, n_rings=nr), 0, 0, k)
        errs.append(np.max(np.abs(col - exact)) / np.max(np.abs(exact)))
    assert errs[0] < 5e-3
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 5.0        # midpoint-ring quadrature: second order


def test_table_square_symmetry(tiny):
    _, H = tiny
    scale = np.max(np.abs(H))
    assert np.max(np.abs(H - H[::-1, :, :, :])) < 1e-13 * scale
    assert np.max(np.abs(H - H[:, ::-1, :, :])) < 1e-13 * scale
    assert np.max(np.abs(H - np.transpose(H, (1, 0, 2, 3)))) < 1e-13 * scale


def test_deeper_voxels_arrive_later(tiny):
    cfg, H = tiny
    K = cfg["grid"]["k_half"]
    e2 = H[K, K] ** 2                           # on-axis columns, [k, n]
    n = np.arange(e2.shape[1])
    centroid = (e2 @ n) / e2.sum(axis=1)        # energy arrival time per depth
    assert np.all(np.diff(centroid) > 0)
    # one depth step of dz = 10 um moves the arrival by about dz fs / c = 1.67 samples
    assert abs(np.median(np.diff(centroid)) - 10e-6 * 250e6 / 1500) < 0.1


def test_column_support_bounds_nonzeros(tiny):
    cfg, H = tiny
    s, g = cfg["sensor"], cfg["grid"]
    elems = model.sensor_elements(s)
    K = g["k_half"]
    for (a, b, k) in [(K, K, 3), (0, 2, 17), (8, 8, 31), (4, 1, 0)]:
        lo, hi = model.column_support(s, g, elems, b - K, a - K, k)
        col = H[a, b, k]
        assert np.all(col[:lo] == 0) and np.all(col[hi + 1:] == 0)
        assert col[lo] != 0 and col[hi] != 0


def test_diffraction_limit_rule_matches_paper():
    (c, flo, fhi, na, exp_um, tol), = [tuple(map(float, r)) for r in
                                       _golden_rows("diffraction_limit.txt")]
    got_um = model.diffraction_limit_mm(c, 0.5 * (flo + fhi), na) * 1e3
    assert abs(got_um - exp_um) <= tol


def test_footprint_modes():
    cfg = W.config("mid")
    s, g = cfg["sensor"], cfg["grid"]
    F = model.footprint(s, g)
    K = g["k_half"]
    # the cone always keeps the axis, is square-symmetric, and widens away from the focus
    assert F[K, K].all()
    assert np.array_equal(F, F[::-1]) and np.array_equal(F, np.transpose(F, (1, 0, 2)))
    counts = F.sum(axis=(0, 1))
    kf = g["nz"] // 2
    assert counts[0] >= counts[kf] and counts[-1] >= counts[kf]
    assert counts[kf] < (2 * K + 1) ** 2
    g0 = dict(g, footprint_mode=0)
    assert model.footprint(s, g0).all()


# --- the paper's own discretisation: trilinear voxel basis, finite-difference derivative -----

def _disc(g, basis, deriv, quad=2):
    return dict(g, voxel_basis=basis, time_derivative=deriv, basis_quad=quad)


def test_focal_voxel_closed_form_central_difference():
    """Point voxel at the focus with the central-difference derivative: every sub-element is at
    distance R, so H = R (cos th_h - cos th_m) (e5(n - Nt/2 + 1) - e5(n - Nt/2 - 1)) / 2 with
    e5 the EIR truncated at 5 sigma."""
    cfg = W.config("mid7")
    s, g = cfg["sensor"], _disc(cfg["grid"], 0, 1)
    got = model.column(s, g, model.sensor_elements(s), 0, 0, g["nz"] // 2)
    sig, om = model.eir_params(s, g)
    R = s["radius_m"] * 1e3
    th_h, th_m = model.sensor_angles(s)
    n = np.arange(g["nt"]) - g["nt"] // 2
    e5 = lambda t: np.where(np.abs(t) <= 5 * sig, model.eir(t, sig, om), 0.0)
    ref = R * (math.cos(th_h) - math.cos(th_m)) * 0.5 * (e5(n + 1.0) - e5(n - 1.0))
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_central_difference_attenuates_the_centre_frequency():
    """The central difference has the response sin(w) against w for the exact derivative:
    at 50 MHz and 250 MHz sampling (w = 0.4 pi) the focal column keeps 75.7 % of its
    amplitude."""
    cfg = W.config("tiny")
    s = cfg["sensor"]
    elems = model.sensor_elements(s)
    cols = [model.column(s, _disc(cfg["grid"], 0, d), elems, 0, 0, cfg["grid"]["nz"] // 2)
            for d in (0, 1)]
    w = 2 * math.pi * s["f0_hz"] / cfg["grid"]["fs_hz"]
    n = np.arange(cfg["grid"]["nt"])
    amp = [abs(np.sum(c * np.exp(-1j * w * n))) for c in cols]
    assert abs(amp[1] / amp[0] - math.sin(w) / w) < 2e-3


def test_trilinear_basis_quadrature():
    """The tent rule is a Gauss rule for the weight 1 - |t|: weights sum to one and the moments
    of the tent, int t^2 (1 - |t|) dt = 1/6 and int t^4 (1 - |t|) dt = 1/15, come out exactly."""
    for q in (2, 3, 4):
        t, w = model.tent_rule(q)
        assert abs(w.sum() - 1.0) < 1e-15
        assert abs(np.sum(w * t ** 2) - 1 / 6) < 1e-15
        if q >= 3:
            assert abs(np.sum(w * t ** 4) - 1 / 15) < 1e-15
    g = _disc(W.config("tiny")["grid"], 1, 0, 3)
    offs, w = model.basis_points(g)
    assert len(w) == 6 ** 3 and abs(w.sum() - 1.0) < 1e-14
    assert np.max(np.abs(offs.sum(axis=0))) < 1e-15            # symmetric about the centre


def test_trilinear_column_converges_and_reduces_to_point_voxel():
    cfg = W.config("tiny")
    s = cfg["sensor"]
    elems = model.sensor_elements(s)
    g = cfg["grid"]
    k = g["nz"] // 2 + 4
    ref = model.column(s, _disc(g, 1, 0, 8), elems, 1, 2, k)
    errs = [np.max(np.abs(model.column(s, _disc(g, 1, 0, q), elems, 1, 2, k) - ref))
            / np.max(np.abs(ref)) for q in (2, 3)]
    assert errs[0] > 10 * errs[1] and errs[1] < 1e-3          # Gauss rule: fast convergence
    # a voxel much smaller than the wavelength acts as a point absorber
    tiny_vox = dict(g, step_m=1e-8, dz_m=1e-8)
    pt = model.column(s, tiny_vox, elems, 0, 0, g["nz"] // 2)
    tri = model.column(s, _disc(tiny_vox, 1, 0, 2), elems, 0, 0, g["nz"] // 2)
    assert np.max(np.abs(tri - pt)) <= 1e-6 * np.max(np.abs(pt))


def test_trilinear_table_square_symmetry():
    cfg = W.config("tiny")
    g = _disc(W.grid(4, 10e-6, 6, 10e-6, 64, 2, 1), 1, 1, 2)
    H = model.build_table(cfg["sensor"], g, workers=1)
    scale = np.max(np.abs(H))
    assert np.max(np.abs(H - H[::-1])) < 1e-13 * scale
    assert np.max(np.abs(H - np.transpose(H, (1, 0, 2, 3)))) < 1e-13 * scale
    lo, hi = operators.supports(cfg["sensor"], g)
    n = np.arange(g["nt"])
    assert not np.any(H[(n < lo[..., None]) | (n > hi[..., None])])
