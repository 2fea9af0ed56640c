"""Shared test helpers: oracle problem set-up (CPU) and device tensors for the HIP path."""
import functools

import numpy as np

import workloads as W
from oracle import model as omodel
from oracle import operators as oops


@functools.lru_cache(maxsize=None)
def oracle_table(name):
    cfg = W.config(name)
    return omodel.build_table(cfg["sensor"], cfg["grid"])


@functools.lru_cache(maxsize=None)
def oracle_supports(name):
    cfg = W.config(name)
    return oops.supports(cfg["sensor"], cfg["grid"])


def oracle_signals(name, seed=0):
    """s = A x0 + peak-normalised Gaussian noise, all from the oracle (FP64)."""
    cfg = W.config(name)
    H = oracle_table(name)
    x0 = W.make_phantom(cfg, seed)
    clean = oops.forward(H, x0)
    sigma = np.max(np.abs(clean)) * 10 ** (-cfg["snr_db"] / 20)
    return x0, clean + sigma * W.unit_noise(cfg, seed)


def oracle_ops(name):
    cfg = W.config(name)
    g = cfg["grid"]
    H = oracle_table(name)
    shp_x = (g["ny"], g["nx"], g["nz"])
    shp_s = (g["ny"], g["nx"], g["nt"])
    A = lambda v: oops.forward(H, v.reshape(shp_x)).ravel()
    AT = lambda u: oops.adjoint(H, u.reshape(shp_s)).ravel()
    return A, AT


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _window(lo, w, n, K):
    """Sub-grid [a, b) that holds every point within K of the window [lo, lo + w), clipped to
    the grid (outside which the model is zero), and the window's start inside it."""
    a, b = max(0, lo - K), min(n, lo + w + K)
    return a, b, lo - a


def window_apply(op, Hs, v, y0, x0, w):
    """The oracle's forward or adjoint at the lateral window [y0, y0+w) x [x0, x0+w) of a
    full grid: both operators only reach K offsets, so they run on the window's K-halo."""
    K = (Hs.shape[0] - 1) // 2
    ya, yb, oy = _window(y0, w, v.shape[0], K)
    xa, xb, ox = _window(x0, w, v.shape[1], K)
    out = op(Hs, v[ya:yb, xa:xb])
    return out[oy:oy + w, ox:ox + w]
