"""Oracle operators A_s u and A_s^T v, and a brute-force dense A_s on tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64.

Translational symmetry (Methods, scanning symmetries; Fig. 1b): the model entry linking
scan position i = (iy, ix) to voxel j = (jy, jx, k) depends only on the relative lateral
offset o = (jy - iy, jx - ix) and on k, so
    s[iy, ix, n] = sum_{o, (iy+dy, ix+dx) in grid}  sum_k H[o][k, n] x[iy+dy, ix+dx, k]
    x[jy, jx, k] = sum_{o, (jy-dy, jx-dx) in grid}  sum_n H[o][k, n] s[jy-dy, jx-dx, n]
Voxels outside the scanned region of interest do not exist (no padding).
Layouts: x[ny][nx][nz], s[ny][nx][nt], table H[dy+K][dx+K][k][n].
"""
from __future__ import annotations

import math

import numpy as np

from . import model


def _ranges(n, d):
    """Scan indices i with 0 <= i + d < n, as a slice for i and for i + d."""
    lo = max(0, -d)
    hi = min(n, n - d)
    return slice(lo, hi), slice(lo + d, hi + d)


def _bbox(Ho):
    """Bounding box (k range, n range) of the nonzeros of one offset block [nz, nt]."""
    nzk = np.flatnonzero(np.any(Ho != 0.0, axis=1))
    nzn = np.flatnonzero(np.any(Ho != 0.0, axis=0))
    if nzk.size == 0:
        return None
    return slice(nzk[0], nzk[-1] + 1), slice(nzn[0], nzn[-1] + 1)


def forward(H, x):
    """s = A_s x: one matrix product per lateral offset on the block's nonzero bounding box."""
    K = (H.shape[0] - 1) // 2
    ny, nx, nz = x.shape
    nt = H.shape[3]
    s = np.zeros((ny, nx, nt))
    for a in range(2 * K + 1):
        for b in range(2 * K + 1):
            bb = _bbox(H[a, b])
            if bb is None:
                continue
            ks, ns = bb
            dy, dx = a - K, b - K
            iy, jy = _ranges(ny, dy)
            ix, jx = _ranges(nx, dx)
            s[iy, ix, ns] += x[jy, jx, ks] @ H[a, b, ks, ns]
    return s


def adjoint(H, s):
    """x = A_s^T s: the transpose of `forward`, offset by offset."""
    K = (H.shape[0] - 1) // 2
    ny, nx, nt = s.shape
    nz = H.shape[2]
    x = np.zeros((ny, nx, nz))
    for a in range(2 * K + 1):
        for b in range(2 * K + 1):
            bb = _bbox(H[a, b])
            if bb is None:
                continue
            ks, ns = bb
            dy, dx = a - K, b - K
            iy, jy = _ranges(ny, dy)
            ix, jx = _ranges(nx, dx)
            x[jy, jx, ks] += s[iy, ix, ns] @ H[a, b, ks, ns].T
    return x


def dense_matrix(sensor, grid, elems=None):
    """Brute-force dense A_s from absolute coordinates (Eq. 2-4), tiny grids only.

    Rows are (iy, ix, n), columns (jy, jx, k).  Each entry is evaluated directly from the
    sensor placed at scan position i and the voxel at its absolute position, with the
    lateral cut-off applied to the absolute index difference; no table and no symmetry."""
    if elems is None:
        elems = model.sensor_elements(sensor)
    pos, area = elems
    ny, nx, nz, nt = grid["ny"], grid["nx"], grid["nz"], grid["nt"]
    K = grid["k_half"]
    F = model.footprint(sensor, grid)
    sigma, omega = model.eir_params(sensor, grid)
    R = sensor["radius_m"] * model.MM
    c_over_fs = grid["c_mps"] * model.MM / grid["fs_hz"]
    step = grid["step_m"] * model.MM
    z = model.depths_mm(grid)
    n = np.arange(nt, dtype=np.float64)
    A = np.zeros((ny * nx * nt, ny * nx * nz))
    for iy in range(ny):
        for ix in range(nx):
            focus = np.array([ix * step, iy * step, 0.0])
            elem_abs = pos + focus[None, :]
            for jy in range(ny):
                for jx in range(nx):
                    dy, dx = jy - iy, jx - ix
                    if abs(dx) > K or abs(dy) > K:
                        continue
                    for k in range(nz):
                        if not F[dy + K, dx + K, k]:
                            continue
                        vox = np.array([jx * step, jy * step, z[k]])
                        r = np.sqrt(np.sum((vox[None, :] - elem_abs) ** 2, axis=1))
                        tau = (n[:, None] - nt // 2) - ((r - R) / c_over_fs)[None, :]
                        term = (model.eir_derivative(tau, sigma, omega)
                                * (area / (2.0 * math.pi * r))[None, :])
                        term[np.abs(tau) > model.EIR_CUTOFF_SIGMAS * sigma] = 0.0
                        row0 = (iy * nx + ix) * nt
                        col = (jy * nx + jx) * nz + k
                        A[row0:row0 + nt, col] = term.sum(axis=1)
    return A


def supports(sensor, grid, elems=None):
    """Per-column inclusive sample ranges (n_lo, n_hi) over the footprint; -1 where inactive."""
    if elems is None:
        elems = model.sensor_elements(sensor)
    K, nz = grid["k_half"], grid["nz"]
    F = model.footprint(sensor, grid)
    lo = -np.ones((2 * K + 1, 2 * K + 1, nz), dtype=np.int64)
    hi = -np.ones((2 * K + 1, 2 * K + 1, nz), dtype=np.int64)
    for a in range(2 * K + 1):
        for b in range(2 * K + 1):
            for k in range(nz):
                if F[a, b, k]:
                    l, h = model.column_support(sensor, grid, elems, b - K, a - K, k)
                    if l <= h:          # an arrival window entirely outside [0, Nt) is empty
                        lo[a, b, k], hi[a, b, k] = l, h
    return lo, hi


def mac_alg(grid, lo, hi):
    """Algorithmic multiply-accumulates of one apply: sum over in-grid (scan, offset) pairs
    and kept depths of the column's support length."""
    K = grid["k_half"]
    ny, nx = grid["ny"], grid["nx"]
    total = 0
    for a in range(2 * K + 1):
        for b in range(2 * K + 1):
            dy, dx = a - K, b - K
            pairs = max(0, ny - abs(dy)) * max(0, nx - abs(dx))
            act = lo[a, b] >= 0
            total += pairs * int(np.sum((hi[a, b] - lo[a, b] + 1)[act]))
    return total
