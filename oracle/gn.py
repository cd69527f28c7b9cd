"""Brute-force local optimisation of model (1) for tiny graphs (test
infrastructure only).

Residuals of model (1) per edge, Sigma1 = tau I, Sigma2 = kappa I:
    sqrt(tau)   * Im(t~_j - t~_i - p_i t~_ij p_i^*)      (3 components; the real
                                                            part is 0 for unit p_i)
    sqrt(kappa) * (p_j^* p_i q~_ij - 1)                   (4 components)
with p_i = x_i / ||x_i|| for free x_i in R^4.  The minimiser is scipy's
Levenberg-Marquardt (a library routine), run from a given start or from many
random starts.
"""
import numpy as np
from scipy.optimize import least_squares


def _qmul(a, b):
    a0, a1, a2, a3 = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    b0, b1, b2, b3 = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                     a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2,
                     a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1,
                     a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0], -1)


def _conj(a):
    return a * np.array([1.0, -1.0, -1.0, -1.0])


def _unpack(x, n):
    P = x[: 4 * n].reshape(n, 4)
    P = P / np.linalg.norm(P, axis=1, keepdims=True)
    return P, x[4 * n:].reshape(n, 3)


def residual(x, n, ei, ej, qm, tm, kappa, tau):
    p, t = _unpack(x, n)
    th = np.concatenate([np.zeros((len(ei), 1)), tm], 1)
    rot = _qmul(_qmul(p[ei], th), _conj(p[ei]))[:, 1:]
    rt = np.sqrt(tau)[:, None] * (t[ej] - t[ei] - rot)
    rq = np.sqrt(kappa)[:, None] * (_qmul(_qmul(_conj(p[ej]), p[ei]), qm) - np.array([1.0, 0, 0, 0]))
    return np.concatenate([rt.ravel(), rq.ravel()])


def model_cost(p, t, ei, ej, qm, tm, kappa, tau):
    x = np.concatenate([np.asarray(p).ravel(), np.asarray(t).ravel()])
    r = residual(x, len(p), ei, ej, qm, tm, kappa, tau)
    return float(r @ r)


def local_min(p0, t0, ei, ej, qm, tm, kappa, tau, tol=1e-15):
    """Levenberg-Marquardt on model (1) from (p0, t0); returns (cost, p, t)."""
    n = len(p0)
    x0 = np.concatenate([np.asarray(p0, float).ravel(), np.asarray(t0, float).ravel()])
    args = (n, np.asarray(ei), np.asarray(ej), np.asarray(qm, float), np.asarray(tm, float),
            np.asarray(kappa, float), np.asarray(tau, float))
    sol = least_squares(residual, x0, args=args, method="lm", xtol=tol, ftol=tol, gtol=tol,
                        max_nfev=20000)
    p, t = _unpack(sol.x, n)
    r = residual(sol.x, *args)
    return float(r @ r), p, t


def multistart_min(n, ei, ej, qm, tm, kappa, tau, starts=50, seed=0):
    """Smallest local-minimum cost over random starts (uniform rotations,
    Gaussian translations)."""
    rng = np.random.default_rng(seed)
    best = np.inf
    for _ in range(starts):
        p0 = rng.standard_normal((n, 4))
        t0 = rng.standard_normal((n, 3)) * 3.0
        c, _, _ = local_min(p0, t0, ei, ej, qm, tm, kappa, tau, tol=1e-12)
        best = min(best, c)
    return best
