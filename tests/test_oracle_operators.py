"""Pins of the oracle's operators: brute-force dense matrix built from absolute coordinates,
a library convolution, the adjoint identity, shift equivariance and shift-superposition."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import model, operators


def _small_cfg():
    cfg = W.config("tiny")
    cfg["grid"] = W.grid(5, 10e-6, 6, 10e-6, 64, 2, 1, ny=4)
    return cfg


@pytest.fixture(scope="module")
def small():
    cfg = _small_cfg()
    s, g = cfg["sensor"], cfg["grid"]
    elems = model.sensor_elements(s)
    H = model.build_table(s, g, elems=elems, workers=1)
    A = operators.dense_matrix(s, g, elems=elems)
    return cfg, H, A


@pytest.fixture(scope="module")
def tiny():
    cfg = W.config("tiny")
    return cfg, model.build_table(cfg["sensor"], cfg["grid"])


def test_forward_matches_bruteforce_dense(small):
    cfg, H, A = small
    g = cfg["grid"]
    x = W.random_image(cfg, 0)
    s = operators.forward(H, x)
    ref = (A @ x.ravel()).reshape(g["ny"], g["nx"], g["nt"])
    assert np.max(np.abs(s - ref)) <= 1e-13 * np.max(np.abs(ref))
    # the cone footprint removes some offsets: the dense matrix really is sparse there
    assert np.count_nonzero(A) < A.size


def test_adjoint_matches_bruteforce_dense(small):
    cfg, H, A = small
    g = cfg["grid"]
    y = W.random_signal(cfg, 0)
    x = operators.adjoint(H, y)
    ref = (A.T @ y.ravel()).reshape(g["ny"], g["nx"], g["nz"])
    assert np.max(np.abs(x - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_mac_alg_covers_dense_nonzeros(small):
    cfg, H, A = small
    s, g = cfg["sensor"], cfg["grid"]
    lo, hi = operators.supports(s, g)
    mac = operators.mac_alg(g, lo, hi)
    assert np.count_nonzero(A) <= mac
    # each nonzero of A lies inside its column's support
    nt, nz, nx = g["nt"], g["nz"], g["nx"]
    K = g["k_half"]
    rows, cols = np.nonzero(A)
    n = rows % nt
    ipos = rows // nt
    k = cols % nz
    jpos = cols // nz
    dy = jpos // nx - ipos // nx
    dx = jpos % nx - ipos % nx
    assert np.all(n >= lo[dy + K, dx + K, k]) and np.all(n <= hi[dy + K, dx + K, k])
    # and the count equals the number of dense entries inside the supports
    count = 0
    for iy in range(g["ny"]):
        for ix in range(nx):
            for jy in range(g["ny"]):
                for jx in range(nx):
                    a, b = jy - iy + K, jx - ix + K
                    if 0 <= a <= 2 * K and 0 <= b <= 2 * K:
                        act = lo[a, b] >= 0
                        count += int(np.sum((hi[a, b] - lo[a, b] + 1)[act]))
    assert count == mac


def test_forward_adjoint_equal_library_convolution(tiny):
    """With the table as a conv weight W[n, k, dy+K, dx+K] the forward is a zero-padded 2-D
    cross-correlation (torch conv2d, FP64 on the CPU) and the adjoint its transpose."""
    cfg, H = tiny
    K = cfg["grid"]["k_half"]
    x = W.random_image(cfg, 1)
    y = W.random_signal(cfg, 1)
    Wt = torch.from_numpy(np.ascontiguousarray(np.transpose(H, (3, 2, 0, 1))))
    xt = torch.from_numpy(np.ascontiguousarray(np.transpose(x, (2, 0, 1))))[None]
    yt = torch.from_numpy(np.ascontiguousarray(np.transpose(y, (2, 0, 1))))[None]
    s_lib = torch.nn.functional.conv2d(xt, Wt, padding=K)[0].permute(1, 2, 0).numpy()
    x_lib = torch.nn.functional.conv_transpose2d(yt, Wt, padding=K)[0].permute(1, 2, 0).numpy()
    s = operators.forward(H, x)
    xa = operators.adjoint(H, y)
    assert np.max(np.abs(s - s_lib)) <= 1e-13 * np.max(np.abs(s_lib))
    assert np.max(np.abs(xa - x_lib)) <= 1e-13 * np.max(np.abs(x_lib))


def test_adjoint_identity(tiny):
    cfg, H = tiny
    x = W.random_image(cfg, 2)
    y = W.random_signal(cfg, 2)
    Ax = operators.forward(H, x)
    ATy = operators.adjoint(H, y)
    lhs, rhs = np.vdot(Ax, y), np.vdot(x, ATy)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_shift_equivariance(tiny):
    """Raster-scan translational symmetry (Fig. 1b): moving the absorber and reading the
    signals at positions moved by the same distance gives the same signals."""
    cfg, H = tiny
    g = cfg["grid"]
    K = g["k_half"]
    x = np.zeros((g["ny"], g["nx"], g["nz"]))
    x[5:8, 4:7, :] = W.random_image(cfg, 3)[5:8, 4:7, :]
    dy, dx = 2, 3
    xs = np.roll(np.roll(x, dy, axis=0), dx, axis=1)
    s0 = operators.forward(H, x)
    s1 = operators.forward(H, xs)
    # compare where both scan positions see the whole support (interior, no ROI edge)
    s0r = np.roll(np.roll(s0, dy, axis=0), dx, axis=1)
    sl = (slice(5 + dy - K, 8 + dy + K - 1 + 1), slice(4 + dx - K, 7 + dx + K))
    sl = tuple(slice(max(0, q.start), q.stop) for q in sl)
    assert np.max(np.abs(s1[sl] - s0r[sl])) <= 1e-13 * np.max(np.abs(s0))
    assert np.max(np.abs(s1[sl])) > 0


def test_shift_superposition(tiny):
    """Superposing a signal volume with a laterally shifted copy of itself equals the signals
    of the absorber plus its shifted copy (Methods, phantom experiments)."""
    cfg, H = tiny
    g = cfg["grid"]
    x = np.zeros((g["ny"], g["nx"], g["nz"]))
    x[7, 6, 16] = 1.0
    x[7, 7, 15] = 0.5
    shift = 4
    x2 = x + np.roll(x, shift, axis=1)
    s = operators.forward(H, x)
    s2 = operators.forward(H, x2)
    sup = s + np.roll(s, shift, axis=1)
    inner = (slice(None), slice(shift, g["nx"] - 1))
    assert np.max(np.abs(s2[inner] - sup[inner])) <= 1e-13 * np.max(np.abs(s2))


def test_depth_slabs_and_windows_match_full_oracle():
    """The two shortcuts the full-size parity tests use: the table restricted to a few depth
    slabs equals those slabs of the full table, and an apply on a window's K-halo equals the
    full-grid apply at the window (interior and edge windows)."""
    from tests.helpers import window_apply
    cfg = W.config("tiny")
    g = dict(cfg["grid"], nx=20, ny=18, k_half=5, footprint_mode=1)
    H = model.build_table(cfg["sensor"], g)
    ks = [3, 17, 30]
    Hs = model.build_depth_slabs(cfg["sensor"], g, ks, workers=1)
    assert np.array_equal(Hs, H[:, :, ks, :])
    rng = W.rng(5)
    x = rng.standard_normal((g["ny"], g["nx"], g["nz"]))
    y = rng.standard_normal((g["ny"], g["nx"], g["nt"]))
    s_full, x_full = operators.forward(H, x), operators.adjoint(H, y)
    for y0, x0, w in ((6, 7, 6), (0, 13, 7), (12, 0, 6)):
        s_w = window_apply(operators.forward, H, x, y0, x0, w)
        x_w = window_apply(operators.adjoint, H, y, y0, x0, w)
        assert np.allclose(s_w, s_full[y0:y0 + w, x0:x0 + w], rtol=0, atol=1e-13 * np.abs(s_full).max())
        assert np.allclose(x_w, x_full[y0:y0 + w, x0:x0 + w], rtol=0, atol=1e-13 * np.abs(x_full).max())
