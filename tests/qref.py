"""Test-local quaternion product and the split objective of eq. (2) in numpy.

Written independently of the oracle so that the oracle's closed-form steps
(App. B) can be checked against the objective they claim to minimise.
"""
import numpy as np


def qmul(a, b):
    a0, a1, a2, a3 = np.moveaxis(np.asarray(a, float), -1, 0)
    b0, b1, b2, b3 = np.moveaxis(np.asarray(b, float), -1, 0)
    return np.stack([a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                     a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2,
                     a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1,
                     a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0], -1)


def qconj(a):
    a = np.asarray(a, float)
    return np.concatenate([a[..., :1], -a[..., 1:]], -1)


def hat(v):
    v = np.asarray(v, float)
    return np.concatenate([np.zeros(v.shape[:-1] + (1,)), v], -1)


ONE = np.array([1.0, 0, 0, 0])


def f_split(ei, ej, tau, tm, p, q, t, s):
    r = hat(t[ej]) - hat(s[ei]) - qmul(qmul(q[ei], hat(tm)), qconj(p[ei]))
    return float((tau * (r * r).sum(1)).sum())


def g_split(ei, ej, kappa, qm, p, q):
    r = qmul(qmul(qconj(p[ej]), q[ei]), qm) - ONE
    return float((kappa * (r * r).sum(1)).sum())


def rodrigues(axis, theta):
    """R = cos(th) I + (1 - cos(th)) n n^T + sin(th) [n]x  (App. A.2)."""
    n = np.asarray(axis, float)
    n = n / np.linalg.norm(n)
    K = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    return np.cos(theta) * np.eye(3) + (1 - np.cos(theta)) * np.outer(n, n) + np.sin(theta) * K
