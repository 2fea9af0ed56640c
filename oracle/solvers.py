"""Oracle solvers for Eq. 5: LSQR (Tikhonov, Eq. 6), FISTA (L1, Eq. 7), refinement schedules.

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64, vectors flattened.

Conventions (Methods, Eq. 5-7, read literally: no factor 1/2 on the data term):
* Tikhonov:  min ||s - A x||^2 + lam ||x||^2   == LSQR with damp = sqrt(lam).
* L1:        min ||s - A x||^2 + lam ||x||_1;  f = ||s - A x||^2 has gradient
             2 A^T (A x - s) and Lipschitz constant 2 sigma_max(A)^2, so the proximal step
             is a soft threshold at lam / L.
* Fixed iteration counts from x0 = 0, no early stopping, no positivity constraint.
"""
from __future__ import annotations

import math

import numpy as np


def lam_l2(ATs):
    """Tikhonov weight rule: 1e-2 * ||A^T s||_2."""
    return 1e-2 * float(np.linalg.norm(ATs.ravel()))


def lam_l1(ATs):
    """L1 weight rule: 5e-3 * max |A^T s|."""
    return 5e-3 * float(np.max(np.abs(ATs)))


def lsqr(A, AT, b, damp=0.0, iters=10):
    """LSQR of Paige and Saunders (the method the paper cites for MB-L2).

    Minimises ||b - A x||^2 + damp^2 ||x||^2 by Golub-Kahan bidiagonalisation
    (beta u = A v - alpha u, alpha v = A^T u - beta v) followed by plane rotations that
    first eliminate the damping row and then update the QR factor of the bidiagonal.
    Returns x after exactly `iters` iterations (fewer only on an exact breakdown, when
    both rhobar and beta vanish) and the history of (alpha, beta, phibar, rhobar)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    beta = float(np.linalg.norm(b))
    u = b / beta if beta > 0 else b.copy()
    v = AT(u)
    alpha = float(np.linalg.norm(v))
    v = v / alpha if alpha > 0 else v
    n = v.size
    x = np.zeros(n)
    w = v.copy()
    phibar, rhobar = beta, alpha
    hist = [dict(alpha=alpha, beta=beta, phibar=phibar, rhobar=rhobar)]
    if alpha * beta == 0.0:
        return x, hist
    for _ in range(iters):
        u = A(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0:
            u = u / beta
        v = AT(u) - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0:
            v = v / alpha
        # rotation that eliminates the damping term
        rhobar1 = math.sqrt(rhobar * rhobar + damp * damp)
        if rhobar1 == 0.0 or rhobar1 * rhobar1 + beta * beta == 0.0:
            break           # exact breakdown: the Krylov space is exhausted, x is final
        cs1 = rhobar / rhobar1
        phibar = cs1 * phibar
        # rotation that eliminates the subdiagonal beta
        rho = math.sqrt(rhobar1 * rhobar1 + beta * beta)
        cs = rhobar1 / rho
        sn = beta / rho
        theta = sn * alpha
        rhobar = -cs * alpha
        phi = cs * phibar
        phibar = sn * phibar
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        hist.append(dict(alpha=alpha, beta=beta, phibar=phibar, rhobar=rhobar))
    return x, hist


def power_iteration(A, AT, v0, iters=50):
    """Largest eigenvalue of A^T A by the power method (Rayleigh quotient at the last
    normalised iterate).  Returns sigma_max(A)^2 estimate."""
    v = np.asarray(v0, dtype=np.float64).ravel()
    v = v / np.linalg.norm(v)
    rq = 0.0
    for _ in range(iters):
        w = AT(A(v))
        rq = float(np.dot(v, w))
        nw = float(np.linalg.norm(w))
        if nw == 0.0:
            return 0.0
        v = w / nw
    return rq


def lipschitz(sigma2, safety=1.01):
    """Lipschitz constant of grad ||s - A x||^2 = 2 sigma_max^2, with a safety factor."""
    return 2.0 * safety * sigma2


def soft_threshold(v, tau):
    """Proximal map of tau*||.||_1: sign(v) max(|v| - tau, 0)."""
    return np.sign(v) * np.maximum(np.abs(v) - tau, 0.0)


def l1_objective(A, s, x, lam):
    r = A(x) - s
    return float(np.dot(r, r) + lam * np.sum(np.abs(x)))


def fista(A, AT, s, lam, L, iters, x0=None, record=False):
    """FISTA of Beck and Teboulle (the method the paper cites for MB-L1), constant step 1/L.

    x_k = S_{lam/L}(y_k - (1/L) 2 A^T (A y_k - s));  t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2;
    y_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1})."""
    s = np.asarray(s, dtype=np.float64).ravel()
    n = AT(s).size
    x_prev = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    y = x_prev.copy()
    t = 1.0
    objs = []
    for _ in range(iters):
        g = 2.0 * AT(A(y) - s)
        x = soft_threshold(y - g / L, lam / L)
        t_next = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
        y = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev, t = x, t_next
        if record:
            objs.append(l1_objective(A, s, x, lam))
    return x_prev, objs


def lsqr_refined(A, AT, s, lam, iters, sweeps):
    """Residual-correction refinement schedule for Tikhonov LSQR.

    x <- LSQR(s; damp = sqrt(lam)); then per sweep: the residual of the normal equations
    g = A^T (s - A x) - lam x; the correction d solves (A^T A + lam I) d = g, written as the
    least-squares problem  min || [A; sqrt(lam) I] d - [0; g / sqrt(lam)] ||  and solved by
    LSQR (damp = 0) with the same iteration count; x <- x + d.  In the HIP path the
    corrections run at low precision and g (both products) at high precision, so the fixed
    point is the high-precision solution; here every step is FP64."""
    s = np.asarray(s, dtype=np.float64).ravel()
    damp = math.sqrt(lam)
    x, _ = lsqr(A, AT, s, damp=damp, iters=iters)
    if sweeps > 0 and damp == 0.0:
        raise ValueError("refinement needs lam > 0")
    m = s.size
    for _ in range(sweeps):
        g = AT(s - A(x)) - lam * x

        def As(v):
            return np.concatenate([A(v), damp * v])

        def ATs(u):
            return AT(u[:m]) + damp * u[m:]

        rhs = np.concatenate([np.zeros(m), g / damp])
        d, _ = lsqr(As, ATs, rhs, damp=0.0, iters=iters)
        x = x + d
    return x


def fista_anchored(A, AT, s, lam, L, iters, period, warmup=0):
    """Anchored-gradient schedule of FISTA: during the first `warmup` iterations and then
    every `period` iterations an anchor gradient g_a = 2 A^T (A x_a - s) is formed at high
    precision (x_a = the current y), and in between the gradient at y is
    g_a + 2 A^T A (y - x_a) with low-precision products.  In exact arithmetic this is plain
    FISTA; here (FP64) it is evaluated exactly as written."""
    s = np.asarray(s, dtype=np.float64).ravel()
    n = AT(s).size
    x_prev = np.zeros(n)
    y = x_prev.copy()
    t = 1.0
    xa, ga = None, None
    for it in range(iters):
        if it < warmup or (it - warmup) % period == 0:
            xa = y.copy()
            ga = 2.0 * AT(A(xa) - s)
            g = ga
        else:
            g = ga + 2.0 * AT(A(y - xa))
        x = soft_threshold(y - g / L, lam / L)
        t_next = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
        y = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev, t = x, t_next
    return x_prev
