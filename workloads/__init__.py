"""Seeded synthetic workloads shared by the tests, the bench and the oracle's callers.

This module holds workload *definitions* (sensor geometry, grids, solver settings) and
seeded random draws (vessel-like phantoms, unit Gaussian noise, power-iteration start
vectors).  It contains none of the reconstruction method's arithmetic: no model, no
operator, no solver.  Both the CPU oracle and the HIP path receive what it produces as
plain arrays.

The paper's datasets (simulated paraboloids, microsphere, carbon fibres, mouse skin;
Methods, "Numerical simulations", "Phantom experiments", "In vivo mouse skin imaging")
are not available, so these synthetic vessel phantoms stand in for them.  Units are SI
(metres, seconds, Hz).
"""
from __future__ import annotations

import copy
import math

import numpy as np

# ----------------------------------------------------------------------------------------
# Sensors.  Spherical-cap PVDF detector (Methods, "Forward modeling", Eq. 3; set-up section).
# aperture_m is the cap's chord *diameter*; hole_m the diameter of a central hole (0 = none).
SENSOR_4MM = dict(radius_m=4e-3, aperture_m=3e-3, hole_m=0.0, n_rings=20,
                  f0_hz=50e6, frac_bw=1.0)
# 7 mm focal distance, NA 0.43, 0.9 mm central hole (AR-OAM set-up section).
SENSOR_7MM = dict(radius_m=7e-3, aperture_m=2 * 7e-3 * 0.43, hole_m=0.9e-3, n_rings=17,
                  f0_hz=50e6, frac_bw=1.0)


def grid(n, step, nz, dz, nt, k_half, mode, ny=None, c=1500.0, fs=250e6):
    """Scan grid == voxel lateral grid (Results, first paragraph)."""
    return dict(c_mps=c, fs_hz=fs, nx=int(n), ny=int(ny if ny is not None else n),
                step_m=step, nz=int(nz), dz_m=dz, nt=int(nt), k_half=int(k_half),
                footprint_mode=int(mode))


# ----------------------------------------------------------------------------------------
# Workloads.  Each entry: sensor, grid, phantom recipe, noise level, solver settings.
CONFIGS = {
    # Tiny plain-method case: 16x16 scan at 10 um, 16x16x32 voxels, Nt 128, 9x9 offsets.
    "tiny": dict(sensor=SENSOR_4MM, grid=grid(16, 10e-6, 32, 10e-6, 128, 4, 0),
                 phantom=dict(kind="straight", n=3, r_um=(10, 20), amp=(1.0, 1.0)),
                 snr_db=30.0, solver=dict(kind="lsqr", iters=20, lam_rule=None)),
    # Full-size plain FP32 case: 200x200 scan, 200x200x128 voxels, Nt 512, cone up to 41x41.
    "vessels200": dict(sensor=SENSOR_4MM, grid=grid(200, 10e-6, 128, 10e-6, 512, 20, 1),
                       phantom=dict(kind="curved", n=40, r_um=(5, 20), amp=(0.3, 1.0)),
                       snr_db=20.0, solver=dict(kind="lsqr", iters=50, lam_rule="l2")),
    # Sparse sub-diffraction pairs on the tiny shapes, for L1 (FISTA).
    "pairs16": dict(sensor=SENSOR_4MM, grid=grid(16, 10e-6, 32, 10e-6, 128, 4, 0),
                    phantom=dict(kind="pairs", n=2, r_um=(5, 5), amp=(1.0, 1.0),
                                 spacing_um=(15, 30), z_um=50),
                    snr_db=30.0, solver=dict(kind="fista", iters=200, lam_rule="l1",
                                             anchor_period=10)),
    # Large fine-step case: 400x400 at 5 um, 400x400x256 voxels, Nt 1024, cone up to 81x81.
    "vessels400": dict(sensor=SENSOR_4MM, grid=grid(400, 5e-6, 256, 5e-6, 1024, 40, 1),
                       phantom=dict(kind="curved", n=200, r_um=(5, 25), amp=(0.3, 1.0)),
                       snr_db=20.0, solver=dict(kind="lsqr", iters=50, lam_rule="l2",
                                                sweeps=2)),
    # Standalone 64x64 window problem at the fine step and footprint rule of vessels400
    # (5 um, K = 40 cone), with the depth range cut to +-80 um (Nt = 4 Nz) so that the CPU
    # oracle can run the FP8 refinement schedule; tube count scaled by area.
    "window400": dict(sensor=SENSOR_4MM, grid=grid(64, 5e-6, 32, 5e-6, 128, 40, 1),
                      phantom=dict(kind="curved", n=5, r_um=(5, 25), amp=(0.3, 1.0)),
                      snr_db=20.0, solver=dict(kind="lsqr", iters=50, lam_rule="l2",
                                               sweeps=2)),
    # Super-resolution pairs (Results, second simulation): 7 mm sensor with 1200 sub-elements,
    # 200 x 200 x 150 um field of view at 5 um, two 20 um absorbers at the focus 60 um or
    # 40 um apart, signals and model band-pass filtered 0.5-80 MHz, peak-normalised, no noise.
    "superres60": dict(sensor=SENSOR_7MM, grid=grid(40, 5e-6, 30, 5e-6, 128, 20, 1),
                       phantom=dict(kind="balls", diam_um=20, sep_um=60, amp=(1.0, 1.0)),
                       snr_db=None, band=dict(f_lo_hz=0.5e6, f_hi_hz=80e6, half_taps=16),
                       solver=dict(kind="both", iters_l2=50, iters_l1=200)),
    "superres40": dict(sensor=SENSOR_7MM, grid=grid(40, 5e-6, 30, 5e-6, 128, 20, 1),
                       phantom=dict(kind="balls", diam_um=20, sep_um=40, amp=(1.0, 1.0)),
                       snr_db=None, band=dict(f_lo_hz=0.5e6, f_hi_hz=80e6, half_taps=16),
                       solver=dict(kind="both", iters_l2=50, iters_l1=200)),
    # Mid-size test case: ragged in every tiled dimension, cone footprint that cuts corners.
    "mid": dict(sensor=SENSOR_4MM, grid=grid(23, 10e-6, 40, 10e-6, 200, 12, 1, ny=19),
                phantom=dict(kind="curved", n=4, r_um=(5, 20), amp=(0.3, 1.0)),
                snr_db=20.0, solver=dict(kind="lsqr", iters=30, lam_rule="l2")),
    # Mid-size case on the 7 mm sensor with a central hole.
    "mid7": dict(sensor=SENSOR_7MM, grid=grid(21, 10e-6, 48, 10e-6, 192, 10, 1, ny=17),
                 phantom=dict(kind="curved", n=4, r_um=(5, 20), amp=(0.3, 1.0)),
                 snr_db=25.0, solver=dict(kind="fista", iters=60, lam_rule="l1")),
}

# Serving mix: scan sides, depth counts (Nt = 4 Nz), both sensors, 70 % LSQR / 30 % FISTA.
SERVE_SIDES = (64, 96, 128, 192, 256, 320, 400)
SERVE_NZ = (64, 128, 256)


def config(name):
    return copy.deepcopy(CONFIGS[name])


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


# ----------------------------------------------------------------------------------------
# Phantoms: voxelised indicators of tubes (distance to the axis <= radius at voxel centres),
# maximum taken where tubes overlap.  Voxel (jy, jx, k) sits at (jx*step, jy*step, z_k) with
# z_k = (k - nz/2)*dz measured from the focal plane, positive = away from the sensor.

def _voxel_axes(g):
    xs = np.arange(g["nx"]) * g["step_m"]
    ys = np.arange(g["ny"]) * g["step_m"]
    zs = (np.arange(g["nz"]) - g["nz"] // 2) * g["dz_m"]
    return xs, ys, zs


def _box(g):
    xs, ys, zs = _voxel_axes(g)
    lo = np.array([xs[0], ys[0], zs[0]])
    hi = np.array([xs[-1], ys[-1], zs[-1]])
    return lo, hi


def _stamp_points(vol, g, pts, radius, amp):
    """Mark voxels whose centre lies within `radius` of any of the points `pts` [P,3]."""
    pts = np.asarray(pts, dtype=np.float64)
    if pts.size == 0:
        return
    st, dz = g["step_m"], g["dz_m"]
    nz2 = g["nz"] // 2
    rx = int(math.ceil(radius / st)) + 1
    rz = int(math.ceil(radius / dz)) + 1
    # candidate voxels: a box around the voxel nearest to each point
    cx = np.rint(pts[:, 0] / st).astype(np.int64)
    cy = np.rint(pts[:, 1] / st).astype(np.int64)
    cz = np.rint(pts[:, 2] / dz).astype(np.int64) + nz2
    ox, oy, oz = np.meshgrid(np.arange(-rx, rx + 1), np.arange(-rx, rx + 1),
                             np.arange(-rz, rz + 1), indexing="ij")
    ox, oy, oz = ox.ravel(), oy.ravel(), oz.ravel()
    for lo in range(0, len(pts), 4096):
        sl = slice(lo, lo + 4096)
        ix = cx[sl, None] + ox[None, :]
        iy = cy[sl, None] + oy[None, :]
        iz = cz[sl, None] + oz[None, :]
        d2 = ((ix * st - pts[sl, 0:1]) ** 2 + (iy * st - pts[sl, 1:2]) ** 2
              + ((iz - nz2) * dz - pts[sl, 2:3]) ** 2)
        ok = ((d2 <= radius * radius) & (ix >= 0) & (ix < g["nx"]) & (iy >= 0)
              & (iy < g["ny"]) & (iz >= 0) & (iz < g["nz"]))
        if not ok.any():
            continue
        flat = np.unique((iy[ok] * g["nx"] + ix[ok]) * g["nz"] + iz[ok])
        v = vol.reshape(-1)
        v[flat] = np.maximum(v[flat], amp)


def _segment_points(a, b, spacing):
    n = max(2, int(np.ceil(np.linalg.norm(b - a) / spacing)) + 1)
    t = np.linspace(0.0, 1.0, n)[:, None]
    return a[None, :] * (1 - t) + b[None, :] * t


def _straight_tubes(g, r, ph):
    lo, hi = _box(g)
    vol = np.zeros((g["ny"], g["nx"], g["nz"]))
    xs, ys, zs = _voxel_axes(g)
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="xy")  # each [ny, nx, nz]
    P = np.stack([X, Y, Z], axis=-1)
    for _ in range(ph["n"]):
        d = r.normal(size=3)
        d /= np.linalg.norm(d)
        c = lo + (hi - lo) * r.uniform(size=3)
        rad = r.uniform(*ph["r_um"]) * 1e-6
        amp = r.uniform(*ph["amp"])
        v = P - c
        along = v @ d
        dist2 = np.sum(v * v, axis=-1) - along * along
        np.maximum(vol, np.where(dist2 <= rad * rad, amp, 0.0), out=vol)
    return vol


def _bezier(ctrl, t):
    t = t[:, None]
    return ((1 - t) ** 3 * ctrl[0] + 3 * (1 - t) ** 2 * t * ctrl[1]
            + 3 * (1 - t) * t ** 2 * ctrl[2] + t ** 3 * ctrl[3])


def _curved_tubes(g, r, ph):
    lo, hi = _box(g)
    vol = np.zeros((g["ny"], g["nx"], g["nz"]))
    spacing = 0.25 * min(g["step_m"], g["dz_m"])
    curves = []
    for i in range(ph["n"]):
        ctrl = lo + (hi - lo) * r.uniform(size=(4, 3))
        if curves and r.uniform() < 0.5:
            # branch: start on a random point of an earlier tube
            parent = curves[int(r.integers(len(curves)))]
            ctrl[0] = _bezier(parent, np.array([r.uniform()]))[0]
        curves.append(ctrl)
        rad = r.uniform(*ph["r_um"]) * 1e-6
        amp = r.uniform(*ph["amp"])
        length = sum(np.linalg.norm(ctrl[j + 1] - ctrl[j]) for j in range(3))
        n = max(8, int(np.ceil(length / spacing)))
        pts = _bezier(ctrl, np.linspace(0.0, 1.0, n))
        _stamp_points(vol, g, pts, rad, amp)
    return vol


def _ball_pair(g, ph):
    """Two balls of diameter diam_um in the focal plane, sep_um apart along x, centred on the
    grid (Results, second simulation: two 20 um absorbers 60 um or 40 um apart at the focus)."""
    vol = np.zeros((g["ny"], g["nx"], g["nz"]))
    st = g["step_m"]
    cx, cy = (g["nx"] // 2) * st, (g["ny"] // 2) * st
    half = 0.5 * ph["sep_um"] * 1e-6
    pts = np.array([[cx - half, cy, 0.0], [cx + half, cy, 0.0]])
    # voxels exactly on the sphere count as inside, for both balls alike
    _stamp_points(vol, g, pts, 0.5 * ph["diam_um"] * 1e-6 * (1 + 1e-9), ph["amp"][0])
    return vol


def _line_pairs(g, r, ph):
    """Pairs of parallel straight lines in lateral planes near the focus (sub-diffraction)."""
    lo, hi = _box(g)
    vol = np.zeros((g["ny"], g["nx"], g["nz"]))
    nz2 = g["nz"] // 2
    kmax = int(round(ph["z_um"] * 1e-6 / g["dz_m"]))
    spacing = 0.25 * g["step_m"]
    for _ in range(ph["n"]):
        k = nz2 + int(r.integers(-kmax, kmax + 1))
        z = (k - nz2) * g["dz_m"]
        ang = r.uniform(0, np.pi)
        d = np.array([np.cos(ang), np.sin(ang), 0.0])
        nrm = np.array([-np.sin(ang), np.cos(ang), 0.0])
        ctr = np.array([lo[0] + (hi[0] - lo[0]) * r.uniform(0.3, 0.7),
                        lo[1] + (hi[1] - lo[1]) * r.uniform(0.3, 0.7), z])
        sep = r.uniform(*ph["spacing_um"]) * 1e-6
        half = np.hypot(hi[0] - lo[0], hi[1] - lo[1])
        rad = r.uniform(*ph["r_um"]) * 1e-6
        for sgn in (-0.5, 0.5):
            c = ctr + sgn * sep * nrm
            pts = _segment_points(c - half * d, c + half * d, spacing)
            _stamp_points(vol, g, pts, rad, ph["amp"][0])
    return vol


def make_phantom(cfg, seed):
    """Absorbed-energy phantom x0 with layout [ny][nx][nz] (float64)."""
    r = rng(1000 + seed)
    ph, g = cfg["phantom"], cfg["grid"]
    if ph["kind"] == "straight":
        return _straight_tubes(g, r, ph)
    if ph["kind"] == "balls":
        return _ball_pair(g, ph)
    if ph["kind"] == "curved":
        return _curved_tubes(g, r, ph)
    if ph["kind"] == "pairs":
        return _line_pairs(g, r, ph)
    raise ValueError(ph["kind"])


def unit_noise(cfg, seed):
    """Unit-variance white Gaussian noise of signal shape [ny][nx][nt] (float64).

    Callers scale it to the configured peak SNR: sigma = max|A x0| * 10**(-snr_db/20)
    (peak normalisation follows the simulation section's noise convention)."""
    g = cfg["grid"]
    return rng(2000 + seed).standard_normal((g["ny"], g["nx"], g["nt"]))


def start_vector(cfg, seed):
    """Seeded N(0,1) start vector for the power iteration, image shape [ny][nx][nz]."""
    g = cfg["grid"]
    return rng(3000 + seed).standard_normal((g["ny"], g["nx"], g["nz"]))


def random_image(cfg, seed):
    g = cfg["grid"]
    return rng(4000 + seed).standard_normal((g["ny"], g["nx"], g["nz"]))


def random_signal(cfg, seed):
    g = cfg["grid"]
    return rng(5000 + seed).standard_normal((g["ny"], g["nx"], g["nt"]))


def serve_trace(n_requests, rate_hz, seed, sides=SERVE_SIDES, nzs=SERVE_NZ):
    """Poisson arrival trace of mixed reconstruction requests (serving workload)."""
    r = rng(6000 + seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += r.exponential(1.0 / rate_hz)
        side = int(r.choice(sides))
        nz = int(r.choice(nzs))
        sensor = "4mm" if r.uniform() < 0.5 else "7mm"
        kind = "lsqr" if r.uniform() < 0.7 else "fista"
        snr = float(r.uniform(15.0, 30.0))
        out.append(dict(id=i, arrival_s=t, side=side, nz=nz, nt=4 * nz, sensor=sensor,
                        kind=kind, snr_db=snr, seed=int(r.integers(1 << 30))))
    return out


def serve_config(req):
    """Workload definition of one serving request (step 10 um, K = 20 cone)."""
    sensor = SENSOR_4MM if req["sensor"] == "4mm" else SENSOR_7MM
    n = req["side"]
    ntubes = max(2, int(round(40 * n * n / 200.0 ** 2)))
    solver = (dict(kind="lsqr", iters=50, lam_rule="l2") if req["kind"] == "lsqr"
              else dict(kind="fista", iters=200, lam_rule="l1"))
    return dict(sensor=copy.deepcopy(sensor),
                grid=grid(n, 10e-6, req["nz"], 10e-6, req["nt"], 20, 1),
                phantom=dict(kind="curved", n=ntubes, r_um=(5, 20), amp=(0.3, 1.0)),
                snr_db=req["snr_db"], solver=solver)
