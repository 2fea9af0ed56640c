"""Pins of the oracle's solvers against independent implementations and mathematical facts:
SciPy's LSQR, dense normal-equation solves, scikit-learn's Lasso, the FISTA rate bound and
the KKT conditions of the L1 problem."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as W
from oracle import model, operators, solvers


@pytest.fixture(scope="module")
def tiny():
    cfg = W.config("tiny")
    H = model.build_table(cfg["sensor"], cfg["grid"])
    x0 = W.make_phantom(cfg, 0)
    s_clean = operators.forward(H, x0)
    noise = W.unit_noise(cfg, 0) * np.max(np.abs(s_clean)) * 10 ** (-cfg["snr_db"] / 20)
    return cfg, H, (s_clean + noise).ravel()


@pytest.fixture(scope="module")
def dense_small():
    cfg = W.config("tiny")
    cfg["grid"] = W.grid(4, 10e-6, 6, 10e-6, 64, 2, 0)
    A = operators.dense_matrix(cfg["sensor"], cfg["grid"])
    rng = W.rng(7)
    x_true = np.zeros(A.shape[1])
    x_true[rng.choice(A.shape[1], 6, replace=False)] = rng.uniform(0.5, 1.0, 6)
    b = A @ x_true + 1e-3 * np.max(np.abs(A @ x_true)) * rng.standard_normal(A.shape[0])
    return A, b


def _ops(H, g):
    shp_x = (g["ny"], g["nx"], g["nz"])
    shp_s = (g["ny"], g["nx"], g["nt"])
    A = lambda v: operators.forward(H, v.reshape(shp_x)).ravel()
    AT = lambda u: operators.adjoint(H, u.reshape(shp_s)).ravel()
    return A, AT


@pytest.mark.parametrize("damp_rel", [0.0, 0.3])
def test_lsqr_iterates_match_scipy(tiny, damp_rel):
    cfg, H, s = tiny
    A, AT = _ops(H, cfg["grid"])
    n = cfg["grid"]["ny"] * cfg["grid"]["nx"] * cfg["grid"]["nz"]
    op = sla.LinearOperator((s.size, n), matvec=A, rmatvec=AT, dtype=np.float64)
    damp = damp_rel * np.linalg.norm(AT(s)) / np.linalg.norm(s)
    for iters in (1, 4, 20):
        x, _ = solvers.lsqr(A, AT, s, damp=damp, iters=iters)
        ref = sla.lsqr(op, s, damp=damp, atol=0, btol=0, conlim=0, iter_lim=iters)[0]
        assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_lsqr_residual_norm_nonincreasing(tiny):
    cfg, H, s = tiny
    A, AT = _ops(H, cfg["grid"])
    x, hist = solvers.lsqr(A, AT, s, iters=20)
    phibar = np.abs([h["phibar"] for h in hist])
    assert np.all(np.diff(phibar) <= 1e-12 * phibar[0])
    # |phibar_k| is the residual norm ||s - A x_k|| for the undamped problem
    assert abs(np.linalg.norm(s - A(x)) - phibar[-1]) <= 1e-10 * phibar[0]


def test_lsqr_converges_to_tikhonov_solution(dense_small):
    A, b = dense_small
    lam = 0.05 * np.linalg.norm(A, 2) ** 2
    x, _ = solvers.lsqr(lambda v: A @ v, lambda u: A.T @ u, b, damp=math.sqrt(lam), iters=400)
    ref = np.linalg.solve(A.T @ A + lam * np.eye(A.shape[1]), A.T @ b)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_lsqr_refinement_reaches_same_solution(dense_small):
    A, b = dense_small
    lam = 0.05 * np.linalg.norm(A, 2) ** 2
    Af, ATf = (lambda v: A @ v), (lambda u: A.T @ u)
    ref = np.linalg.solve(A.T @ A + lam * np.eye(A.shape[1]), A.T @ b)
    x_plain, _ = solvers.lsqr(Af, ATf, b, damp=math.sqrt(lam), iters=12)
    x_ref = solvers.lsqr_refined(Af, ATf, b, lam, iters=12, sweeps=2)
    # sweeps = 0 is plain LSQR; each correction solve moves towards the Tikhonov solution
    assert np.array_equal(solvers.lsqr_refined(Af, ATf, b, lam, 12, 0), x_plain)
    e_plain = np.linalg.norm(x_plain - ref)
    e_ref = np.linalg.norm(x_ref - ref)
    assert e_ref < 0.1 * e_plain
    x_long = solvers.lsqr_refined(Af, ATf, b, lam, iters=200, sweeps=2)
    assert np.linalg.norm(x_long - ref) <= 1e-10 * np.linalg.norm(ref)


def test_power_iteration_matches_spectral_norm(dense_small):
    A, _ = dense_small
    v0 = W.rng(3).standard_normal(A.shape[1])
    s2 = solvers.power_iteration(lambda v: A @ v, lambda u: A.T @ u, v0, iters=2000)
    ref = np.linalg.norm(A, 2) ** 2
    assert abs(s2 - ref) <= 1e-8 * ref
    s50 = solvers.power_iteration(lambda v: A @ v, lambda u: A.T @ u, v0, iters=50)
    assert s50 <= ref * (1 + 1e-12) and s50 > 0.5 * ref


def _kkt_violation(A, b, x, lam):
    g = 2 * A.T @ (b - A @ x)          # minus the gradient of the data term
    on = np.abs(x) > 0
    v_on = np.max(np.abs(g[on] - lam * np.sign(x[on]))) if on.any() else 0.0
    v_off = max(0.0, np.max(np.abs(g[~on])) - lam) if (~on).any() else 0.0
    return max(v_on, v_off) / lam


def test_fista_converges_to_lasso_solution(dense_small):
    from sklearn.linear_model import Lasso
    A, b = dense_small
    lam = 0.05 * np.max(np.abs(2 * A.T @ b))
    L = solvers.lipschitz(np.linalg.norm(A, 2) ** 2)
    Af, ATf = (lambda v: A @ v), (lambda u: A.T @ u)
    x, objs = solvers.fista(Af, ATf, b, lam, L, iters=20000)
    assert _kkt_violation(A, b, x, lam) < 1e-6
    m = A.shape[0]
    sk = Lasso(alpha=lam / (2 * m), fit_intercept=False, tol=1e-14, max_iter=200000)
    sk.fit(A, b)
    F = lambda z: float(np.sum((b - A @ z) ** 2) + lam * np.sum(np.abs(z)))
    assert abs(F(x) - F(sk.coef_)) <= 1e-8 * F(sk.coef_)
    assert np.linalg.norm(x - sk.coef_) <= 1e-4 * np.linalg.norm(sk.coef_)


def test_fista_rate_bound(dense_small):
    """Beck-Teboulle: F(x_k) - F* <= 2 L ||x0 - x*||^2 / (k+1)^2."""
    A, b = dense_small
    lam = 0.05 * np.max(np.abs(2 * A.T @ b))
    L = solvers.lipschitz(np.linalg.norm(A, 2) ** 2)
    Af, ATf = (lambda v: A @ v), (lambda u: A.T @ u)
    xs, _ = solvers.fista(Af, ATf, b, lam, L, iters=20000)
    F = lambda z: float(np.sum((b - A @ z) ** 2) + lam * np.sum(np.abs(z)))
    Fs = F(xs)
    _, objs = solvers.fista(Af, ATf, b, lam, L, iters=300, record=True)
    k = np.arange(1, 301)
    bound = 2 * L * np.dot(xs, xs) / (k + 1) ** 2
    assert np.all(np.array(objs) - Fs <= bound + 1e-12 * Fs)


def test_fista_anchored_equals_plain_in_fp64(tiny):
    cfg, H, s = tiny
    A, AT = _ops(H, cfg["grid"])
    sig2 = solvers.power_iteration(A, AT, W.start_vector(cfg, 0), iters=50)
    L = solvers.lipschitz(sig2)
    lam = solvers.lam_l1(AT(s))
    x_plain, _ = solvers.fista(A, AT, s, lam, L, iters=40)
    for period, warmup in ((10, 0), (5, 12)):
        x_anch = solvers.fista_anchored(A, AT, s, lam, L, iters=40, period=period, warmup=warmup)
        assert np.linalg.norm(x_anch - x_plain) <= 1e-10 * np.linalg.norm(x_plain)
    assert np.count_nonzero(x_plain) < x_plain.size      # L1 gives a sparse image


def test_soft_threshold_is_l1_prox():
    """prox_{t|.|}(v) = argmin_z 0.5 (z - v)^2 + t |z|, checked by brute-force minimisation."""
    v = np.linspace(-3, 3, 61)
    t = 0.7
    zs = np.linspace(-4, 4, 800001)
    brute = np.array([zs[np.argmin(0.5 * (zs - vi) ** 2 + t * np.abs(zs))] for vi in v])
    assert np.max(np.abs(solvers.soft_threshold(v, t) - brute)) <= 1e-5
