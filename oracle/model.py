"""Oracle model: sensor sub-elements, electrical impulse response, footprint, model table.

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64 throughout; lengths in mm,
times in samples.

Reading of the paper used here (each choice is also listed in the design notes):
* Eq. 1 for a point absorber at distance r gives a pressure proportional to the time
  derivative of delta(t - r/c)/r.  Summing over sensor sub-elements (Eq. 3-4) and
  convolving with the electrical impulse response e (Results, first paragraph: the
  impulse response is the EIR convolved with the SIR) moves the derivative onto e:
      H[o][n, k] = sum_j  dS_j / (2 pi r_j) * e'(tau_nj),
      tau_nj     = (n - Nt/2) - fs (r_j - R) / c          (samples)
  The 1/(2 pi) makes the sub-element sum a quadrature of the spatial impulse response
  h(t) = int_S delta(t - r/c) / (2 pi r) dS.  Units are arbitrary (Methods, Eq. 2).
* Sample Nt/2 sits at t = R/c (the focal arrival).  Voxel depths are
  z_k = (k - Nz/2) dz from the focal plane, positive = away from the sensor.
* The EIR is a zero-phase Gaussian-modulated cosine with centre f0 and an amplitude
  -6 dB bandwidth of frac_bw * f0; a term enters the sum iff |tau| <= 5 sigma.
* The paper's own discretisation (Methods, Forward modeling: finite differences in time,
  trilinear interpolation of voxel values on the integration sphere) is available as an
  option: a trilinear (tent) voxel basis, integrated by a Gauss rule over each voxel, and a
  central difference of the band-limited signal instead of the analytic derivative.  The
  default is the point voxel with the analytic derivative.
* Lateral cut-off (Results, first paragraph; Methods, scanning symmetries: the model is
  set to zero where the sensitivity drops): offsets |dx|,|dy| <= K, and in mode 1 also
  the cone (dx^2+dy^2) step^2 <= (rho0 + |z| tan(theta_m))^2 with rho0 = 2 * 0.71 lambda/NA
  (the diffraction-limit rule of the Results section).
"""
from __future__ import annotations

import math
import os

import numpy as np

MM = 1e3  # metres -> millimetres
EIR_CUTOFF_SIGMAS = 5.0


# ---------------------------------------------------------------------------------------
# Sensor discretisation (Eq. 3: sub-elements x_j with areas dx_j; ~1000-1200 of them).

def sensor_angles(sensor):
    """Polar half-angles (theta_h, theta_m) of the cap's hole and rim, in radians."""
    R = sensor["radius_m"]
    th_m = math.asin(sensor["aperture_m"] / (2.0 * R))
    th_h = math.asin(sensor["hole_m"] / (2.0 * R)) if sensor["hole_m"] > 0 else 0.0
    return th_h, th_m


def sensor_elements(sensor, n_rings=None):
    """Sub-element centres (mm, relative to the focus) and exact patch areas (mm^2).

    The cap between theta_h and theta_m is cut into n_rings equal-angle rings.  Ring l
    (edges theta_l, theta_{l+1}, mid-angle tb) is cut into n_l = 8*max(1, floor(2 pi sin(tb)
    / (8 dtheta) + 1/2)) equal patches (a multiple of 8, so the set is invariant under the
    square's symmetry group), centred at azimuth 2 pi (m + 1/2)/n_l.  Each patch's area is
    the exact spherical-zone area R^2 (cos theta_l - cos theta_{l+1}) 2 pi / n_l.
    The sensor lies above the focus: a patch sits at R (sin tb cos phi, sin tb sin phi, -cos tb).
    """
    R = sensor["radius_m"] * MM
    th_h, th_m = sensor_angles(sensor)
    nr = int(n_rings if n_rings is not None else sensor["n_rings"])
    dth = (th_m - th_h) / nr
    pos, area = [], []
    for l in range(nr):
        t0 = th_h + (th_m - th_h) * l / nr
        t1 = th_h + (th_m - th_h) * (l + 1) / nr
        tb = 0.5 * (t0 + t1)
        n_l = 8 * max(1, int(math.floor(2.0 * math.pi * math.sin(tb) / (8.0 * dth) + 0.5)))
        a = R * R * (math.cos(t0) - math.cos(t1)) * 2.0 * math.pi / n_l
        for m in range(n_l):
            phi = 2.0 * math.pi * (m + 0.5) / n_l
            pos.append((R * math.sin(tb) * math.cos(phi),
                        R * math.sin(tb) * math.sin(phi),
                        -R * math.cos(tb)))
            area.append(a)
    return np.array(pos, dtype=np.float64), np.array(area, dtype=np.float64)


# ---------------------------------------------------------------------------------------
# Electrical impulse response (EIR), time in samples.

def eir_params(sensor, grid):
    """(sigma, omega): Gaussian envelope width in samples and carrier in rad/sample.

    The amplitude spectrum of exp(-t^2/(2 s^2)) has standard deviation 1/(2 pi s); its
    full width at half maximum is 2 sqrt(2 ln 2) sigma_f, set equal to frac_bw * f0."""
    fs, f0, bw = grid["fs_hz"], sensor["f0_hz"], sensor["frac_bw"]
    sigma_f = f0 * bw / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    sigma = fs / (2.0 * math.pi * sigma_f)
    omega = 2.0 * math.pi * f0 / fs
    return sigma, omega


def eir(tau, sigma, omega):
    """e(tau) = exp(-tau^2 / (2 sigma^2)) cos(omega tau)."""
    tau = np.asarray(tau, dtype=np.float64)
    return np.exp(-tau * tau / (2.0 * sigma * sigma)) * np.cos(omega * tau)


def eir_derivative(tau, sigma, omega):
    """de/dtau = -exp(-tau^2/(2 sigma^2)) [ (tau/sigma^2) cos(omega tau) + omega sin(omega tau) ]."""
    tau = np.asarray(tau, dtype=np.float64)
    g = np.exp(-tau * tau / (2.0 * sigma * sigma))
    return -g * ((tau / (sigma * sigma)) * np.cos(omega * tau) + omega * np.sin(omega * tau))


# ---------------------------------------------------------------------------------------
# Grid geometry and lateral footprint.

def depths_mm(grid):
    nz = grid["nz"]
    return (np.arange(nz) - nz // 2) * grid["dz_m"] * MM


def diffraction_limit_mm(c_mps, f_hz, na):
    """Acoustic diffraction-limited lateral resolution 0.71 lambda / NA (Results), in mm."""
    return 0.71 * (c_mps / f_hz) * MM / na


def footprint(sensor, grid):
    """Boolean mask F[dy+K, dx+K, k]: True where the model column is kept."""
    K = grid["k_half"]
    nz = grid["nz"]
    d = np.arange(-K, K + 1)
    DY, DX = np.meshgrid(d, d, indexing="ij")
    F = np.ones((2 * K + 1, 2 * K + 1, nz), dtype=bool)
    if grid["footprint_mode"] == 0:
        return F
    th_h, th_m = sensor_angles(sensor)
    rho0 = 2.0 * diffraction_limit_mm(grid["c_mps"], sensor["f0_hz"], math.sin(th_m))
    step = grid["step_m"] * MM
    z = depths_mm(grid)
    for k in range(nz):
        rho = rho0 + abs(z[k]) * math.tan(th_m)
        F[:, :, k] = (DX * DX + DY * DY) * step * step <= rho * rho
    return F


# ---------------------------------------------------------------------------------------
# The compressed model: columns for one scan position (Methods, scanning symmetries).

def discretisation(grid):
    """(voxel basis, time derivative, quadrature points per half axis) of a grid.

    Voxel basis 0: a point absorber at the voxel centre; 1: the trilinear (tent) basis of
    the paper's discretisation (Methods, Forward modeling: trilinear interpolation of
    neighbouring voxel values).  Time derivative 0: the analytic derivative of the EIR;
    1: the central finite difference of the paper's discretisation, applied to the
    band-limited signal (the truncated EIR)."""
    return (int(grid.get("voxel_basis", 0)), int(grid.get("time_derivative", 0)),
            int(grid.get("basis_quad", 3)))


def tent_rule(q):
    """Nodes and weights on [-1, 1] for integrals of f(t) (1 - |t|): q-point Gauss-Legendre
    on each half [-1, 0] and [0, 1] with the tent factor folded into the weights (exact when
    f (1 - |t|) is a polynomial of degree <= 2q - 1 on each half)."""
    x, w = np.polynomial.legendre.leggauss(q)            # on [-1, 1]
    t = 0.5 * (x + 1.0)                                   # on [0, 1]
    wt = 0.5 * w * (1.0 - t)
    return np.concatenate([-t[::-1], t]), np.concatenate([wt[::-1], wt])


def basis_points(grid):
    """Quadrature of the voxel basis: offsets (mm) from the voxel centre and weights.

    The trilinear basis is the product of tents 1 - |t| (t in voxel spacings, |t| <= 1) along
    x, y and z; each axis uses `tent_rule`, whose weights sum to one."""
    vb, _, Q = discretisation(grid)
    if vb == 0:
        return np.zeros((1, 3)), np.ones(1)
    t, w = tent_rule(Q)
    step, dz = grid["step_m"] * MM, grid["dz_m"] * MM
    X, Y, Z = np.meshgrid(t * step, t * step, t * dz, indexing="ij")
    WX, WY, WZ = np.meshgrid(w, w, w, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1), (WX * WY * WZ).ravel()


def derivative_kernel(tau, sigma, omega, deriv):
    """Time derivative of the electrical response truncated at 5 sigma, in samples:
    analytic e'(tau), or the central difference (e(tau + 1) - e(tau - 1)) / 2."""
    cut = EIR_CUTOFF_SIGMAS * sigma
    tau = np.asarray(tau, dtype=np.float64)
    if deriv == 0:
        v = eir_derivative(tau, sigma, omega)
        v[np.abs(tau) > cut] = 0.0
        return v
    ep = eir(tau + 1.0, sigma, omega)
    ep[np.abs(tau + 1.0) > cut] = 0.0
    em = eir(tau - 1.0, sigma, omega)
    em[np.abs(tau - 1.0) > cut] = 0.0
    return 0.5 * (ep - em)


def _kernel_reach(sigma, deriv):
    return EIR_CUTOFF_SIGMAS * sigma + (1.0 if deriv else 0.0)


def _delays(sensor, grid, elems, dx, dy, k):
    """Distances r (mm) and delays (samples) of every (basis point, sub-element) pair."""
    pos, _ = elems
    R = sensor["radius_m"] * MM
    c_over_fs = grid["c_mps"] * MM / grid["fs_hz"]          # mm per sample
    step = grid["step_m"] * MM
    p = np.array([dx * step, dy * step, depths_mm(grid)[k]])
    offs, wq = basis_points(grid)
    pts = p[None, :] + offs                                   # [Q, 3]
    r = np.sqrt(np.sum((pts[:, None, :] - pos[None, :, :]) ** 2, axis=2))   # [Q, M]
    return r, (r - R) / c_over_fs, wq


def column(sensor, grid, elems, dx, dy, k):
    """Time signal of voxel (dx, dy, k) relative to the scan position, length Nt (FP64).

    Direct sum over sub-elements (Eq. 3-4) of dS_j/(2 pi r_j) e'(tau_nj); for the trilinear
    basis, the weighted sum of that over the basis quadrature points."""
    _, area = elems
    sigma, omega = eir_params(sensor, grid)
    _, deriv, _ = discretisation(grid)
    r, delay, wq = _delays(sensor, grid, elems, dx, dy, k)
    # Only samples within the kernel's reach of some arrival can be nonzero.
    nt = grid["nt"]
    reach = _kernel_reach(sigma, deriv)
    lo = max(0, math.ceil(nt // 2 + delay.min() - reach))
    hi = min(nt - 1, math.floor(nt // 2 + delay.max() + reach))
    out = np.zeros(nt)
    if lo > hi:
        return out
    n = np.arange(lo, hi + 1, dtype=np.float64)
    acc = np.zeros(hi - lo + 1)
    for q in range(len(wq)):
        tau = (n[:, None] - nt // 2) - delay[q][None, :]     # [samples, M]
        w = area / (2.0 * math.pi * r[q])
        term = derivative_kernel(tau, sigma, omega, deriv) * w[None, :]
        acc += wq[q] * term.sum(axis=1)
    out[lo:hi + 1] = acc
    return out


def column_support(sensor, grid, elems, dx, dy, k):
    """Inclusive sample range [n_lo, n_hi] outside which the column is exactly zero."""
    sigma, _ = eir_params(sensor, grid)
    _, deriv, _ = discretisation(grid)
    _, delay, _ = _delays(sensor, grid, elems, dx, dy, k)
    reach = _kernel_reach(sigma, deriv)
    lo = math.ceil(grid["nt"] // 2 + delay.min() - reach)
    hi = math.floor(grid["nt"] // 2 + delay.max() + reach)
    return max(lo, 0), min(hi, grid["nt"] - 1)


def _depth_slab(args):
    sensor, grid, elems, k = args
    K, nt = grid["k_half"], grid["nt"]
    F = footprint(sensor, grid)
    out = np.zeros((2 * K + 1, 2 * K + 1, nt))
    for a in range(2 * K + 1):
        for b in range(2 * K + 1):
            if F[a, b, k]:
                out[a, b, :] = column(sensor, grid, elems, b - K, a - K, k)
    return k, out


def build_table(sensor, grid, depths=None, elems=None, workers=None):
    """Dense FP64 table H[dy+K, dx+K, k, n] (zero outside the footprint).

    `depths` restricts the build to a subset of depth indices (others stay zero).
    `workers` > 1 evaluates depth slabs in parallel processes (same arithmetic)."""
    K, nz, nt = grid["k_half"], grid["nz"], grid["nt"]
    if elems is None:
        elems = sensor_elements(sensor)
    H = np.zeros((2 * K + 1, 2 * K + 1, nz, nt))
    ks = list(range(nz) if depths is None else depths)
    jobs = [(sensor, grid, elems, k) for k in ks]
    if workers is None:
        workers = min(len(ks), os.cpu_count() or 1, 16)
    if workers > 1 and len(ks) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            for k, slab in pool.imap_unordered(_depth_slab, jobs):
                H[:, :, k, :] = slab
    else:
        for job in jobs:
            k, slab = _depth_slab(job)
            H[:, :, k, :] = slab
    return H


def build_depth_slabs(sensor, grid, depths, elems=None, workers=None):
    """The table restricted to the listed depth indices, H[dy+K, dx+K, i, n] for depth
    depths[i]: the same columns as `build_table`, without the zero slabs of the others."""
    K, nt = grid["k_half"], grid["nt"]
    if elems is None:
        elems = sensor_elements(sensor)
    ks = list(depths)
    H = np.zeros((2 * K + 1, 2 * K + 1, len(ks), nt))
    pos = {k: i for i, k in enumerate(ks)}
    jobs = [(sensor, grid, elems, k) for k in ks]
    if workers is None:
        workers = min(len(ks), os.cpu_count() or 1, 16)
    if workers > 1 and len(ks) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            for k, slab in pool.imap_unordered(_depth_slab, jobs):
                H[:, :, pos[k], :] = slab
    else:
        for job in jobs:
            k, slab = _depth_slab(job)
            H[:, :, pos[k], :] = slab
    return H


def table_columns_mac(H):
    """Number of nonzero entries per (offset, depth) column: nnz counts for the work model."""
    return np.count_nonzero(H, axis=-1)
