"""PRADMM with a general translation weight per edge -- oracle, FP64, CPU,
test infrastructure only.

The model of the Model section weighs the translation residual with
Sigma1 = diag(c, Omega1^{-1}) and the rotation residual with Sigma2 = kappa I.
Here every edge carries its own 3x3 information matrix S_e = Omega_e^{-1}
(symmetric positive definite) and c_e = trace(S_e) / 3 (the arbitrary c of
the Model section; with S_e = tau_e I it is tau_e, the isotropic reading).
Then A1 of the p-subproblem is no longer a multiple of I, and the update is
the sphere-constrained quadratic of Lemma 1.  Its multiplier is taken from
the characterisation of Lemma B.1 (ii): with A1 = W diag(a) W^T and
g = W^T b1, lambda* > -a_min solves h(lambda) = sum g_k^2 / (a_k + lambda)^2
- 1 = 0 (a library bracketing root finder on that equation), p =
-(A1 + lambda* I)^{-1} b1; in the hard case (g vanishing on the lowest
eigenspace and h(-a_min) <= 0) lambda* = -a_min and p is the pseudo-inverse
solution plus the lowest-eigenspace component that brings the norm to 1,
the one of those minimisers nearest p^k.  That lambda* is the rightmost real eigenvalue of
Alg. 2's 8x8 matrix is a pin (tests), not the method used here, because a
nonsymmetric eigensolver loses accuracy near the hard case.

  A1 = 2 sum_out G1^T Sigma1 G1 + 2 sum_in kappa G2^T G2 + (beta + h1) I,
  b1 = -2 sum_out G1^T Sigma1 (t~_j - s~_i) - 2 sum_in kappa G2^T 1
       - beta q_i - lambda_i - h1 p_i                       (App. B.1);
  A2 = sum_out 2 (G3^T Sigma1 G3 + kappa G4^T G4) + (beta + h2) I,
  b2 = sum_out 2 (G3^T Sigma1 (t~_j - s~_i) + kappa G4^T 1) + beta p_i
       - lambda_i + h2 q_i,   q_i = A2^{-1} b2                (App. B.2);
  A3 = sum_in 2 S_e + (beta + h3) I,
  b3 = sum_in 2 S_e (s_l + c_li) + beta s_i + z_i + h3 t_i      (App. B.3);
  A4 = sum_out 2 S_e + (beta + h4) I,
  b4 = sum_out 2 S_e (t_j - c_ij) + beta t_i - z_i + h4 s_i    (App. B.4);
  lambda -= gamma beta (p - q),  z -= gamma beta (t - s).

The G matrices and every reading are those of oracle/pradmm.py.
"""
import numpy as np
import scipy.optimize
import torch

from . import prep
from .pradmm import DEFAULT_H, _sum_into, _T, _c
from .quat import F64, D4, ONE, Mmat, Wmat, hat, mv, qconj, qmul


def prepare(n, ei, ej, Rm, tm, kappa, S, R0, t0):
    """The boundary preparation of prep.prepare plus the 4x4 Sigma1 per edge."""
    S = torch.as_tensor(np.asarray(S, np.float64).reshape(-1, 3, 3))
    c = S.diagonal(dim1=1, dim2=2).sum(-1) / 3.0
    P, p0, t0 = prep.prepare(n, ei, ej, Rm, tm, kappa, c.numpy(), R0, t0)
    Sig1 = torch.zeros(S.shape[0], 4, 4, dtype=F64)
    Sig1[:, 0, 0] = c
    Sig1[:, 1:, 1:] = S
    P = dict(P, S=S, Sig1=Sig1)
    return P, p0, t0


def trs_sphere(A, b, p_prev):
    """argmin over ||x|| = 1 of 1/2 x^T A x + b^T x for one symmetric A, and
    its multiplier lambda* (Lemma B.1)."""
    A = A.numpy() if torch.is_tensor(A) else np.asarray(A, np.float64)
    b = b.numpy() if torch.is_tensor(b) else np.asarray(b, np.float64)
    w, V = np.linalg.eigh(A)
    g = V.T @ b
    nb = float(np.linalg.norm(b))
    scale = max(1.0, float(np.abs(w).max()), nb)
    low = np.abs(w - w[0]) <= 1e-12 * scale            # the lowest eigenspace
    g_low = float(np.linalg.norm(g[low]))
    rest = lambda lam: float(np.sum(g[~low] ** 2 / (w[~low] + lam) ** 2))
    h = lambda lam: rest(lam) + g_low ** 2 / (w[0] + lam) ** 2 - 1.0
    hard = g_low <= 1e-14 * scale and rest(-w[0]) <= 1.0
    if not hard:
        lo = -w[0] + max(g_low, 1e-300)              # h(lo) >= 0 when g_low > 0
        while h(lo) <= 0.0:
            lo = -w[0] + (lo + w[0]) * 1e-3
        hi = nb - w[0]                               # ||x(hi)|| <= ||b|| / (w_min + hi) = 1
        while h(hi) > 0.0:
            hi = -w[0] + (hi + w[0]) * (1.0 + 1e-12)
        lam = scipy.optimize.brentq(h, lo, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps,
                                    maxiter=1000)
        return -np.linalg.solve(A + lam * np.eye(A.shape[0]), b), lam
    lam = -float(w[0])
    x0 = -(V[:, ~low] @ (g[~low] / (w[~low] + lam)))
    rem = max(0.0, 1.0 - float(x0 @ x0))
    # the minimisers are x0 + y, y in the lowest eigenspace with |y|^2 = rem;
    # take the one nearest p_prev: y along p_prev's projection on that space
    Vl = V[:, low]
    u = Vl @ (Vl.T @ np.asarray(p_prev, np.float64))
    nu = float(np.linalg.norm(u))
    u = u / nu if nu > 0.0 else Vl[:, 0]
    return x0 + np.sqrt(rem) * u, lam


def alg2_multiplier(A, b):
    """The rightmost real lambda with Q y = -lambda y, Q = [[A, -b b^T],
    [-I, A]] (Alg. 2 as printed) -- used to pin trs_sphere."""
    n = A.shape[0]
    Q = np.block([[A, -np.outer(b, b)], [-np.eye(n), A]])
    mu = np.linalg.eigvals(Q)
    real = np.abs(mu.imag) <= 1e-7 * (1.0 + np.abs(mu.real))
    return float(np.max(-mu.real[real]))


def step_p(P, st, beta, h=DEFAULT_H):
    n, ei, ej = P["n"], P["ei"], P["ej"]
    kappa, tm, qm, Sig1 = P["kappa"], P["tm"], P["qm"], P["Sig1"]
    q, t, s, lam, p = st["q"], st["t"], st["s"], st["lam"], st["p"]
    G1 = Mmat(q[ei]) @ Mmat(hat(tm)) @ D4
    r = hat(t[ej] - s[ei])
    G2 = Wmat(qm) @ Wmat(q[ei]) @ D4
    I4 = torch.eye(4, dtype=F64)
    A1 = (_sum_into(n, ei, 2.0 * (_T(G1) @ Sig1 @ G1))
          + _sum_into(n, ej, 2.0 * kappa[:, None, None] * (_T(G2) @ G2)) + (beta + h[0]) * I4)
    b1 = (-_sum_into(n, ei, 2.0 * mv(_T(G1) @ Sig1, r))
          - _sum_into(n, ej, 2.0 * kappa[:, None] * mv(_T(G2), ONE.expand(G2.shape[0], 4)))
          - beta * q - lam - h[0] * p)
    out = torch.empty_like(p)
    for i in range(n):
        x, _ = trs_sphere(A1[i], b1[i], p[i].numpy())
        out[i] = torch.as_tensor(x)
    return out


def step_q(P, st, p_new, beta, h=DEFAULT_H):
    n, ei, ej = P["n"], P["ei"], P["ej"]
    kappa, tm, qm, Sig1 = P["kappa"], P["tm"], P["qm"], P["Sig1"]
    q, t, s, lam = st["q"], st["t"], st["s"], st["lam"]
    G3 = _T(Wmat(p_new[ei])) @ Wmat(hat(tm))
    G4 = Wmat(qm) @ _T(Mmat(p_new[ej]))
    r = hat(t[ej] - s[ei])
    A_e = 2.0 * (_T(G3) @ Sig1 @ G3 + kappa[:, None, None] * (_T(G4) @ G4))
    b_e = 2.0 * (mv(_T(G3) @ Sig1, r) + kappa[:, None] * mv(_T(G4), ONE.expand(G4.shape[0], 4)))
    I4 = torch.eye(4, dtype=F64)
    A2 = _sum_into(n, ei, A_e) + (beta + h[1]) * I4
    b2 = _sum_into(n, ei, b_e) + beta * p_new - lam + h[1] * q
    return torch.linalg.solve(A2, b2)


def step_t(P, st, p_new, q_new, beta, h=DEFAULT_H):
    n, ei, ej, S, tm = P["n"], P["ei"], P["ej"], P["S"], P["tm"]
    t, s, z = st["t"], st["s"], st["z"]
    c = _c(p_new, q_new, tm, ei)
    I3 = torch.eye(3, dtype=F64)
    A3 = _sum_into(n, ej, 2.0 * S) + (beta + h[2]) * I3
    b3 = _sum_into(n, ej, 2.0 * mv(S, s[ei] + c)) + beta * s + z + h[2] * t
    return torch.linalg.solve(A3, b3)


def step_s(P, st, p_new, q_new, t_new, beta, h=DEFAULT_H):
    n, ei, ej, S, tm = P["n"], P["ei"], P["ej"], P["S"], P["tm"]
    s, z = st["s"], st["z"]
    c = _c(p_new, q_new, tm, ei)
    I3 = torch.eye(3, dtype=F64)
    A4 = _sum_into(n, ei, 2.0 * S) + (beta + h[3]) * I3
    b4 = _sum_into(n, ei, 2.0 * mv(S, t_new[ej] - c)) + beta * t_new - z + h[3] * s
    return torch.linalg.solve(A4, b4)


def sweep(P, st, beta, gamma, h=DEFAULT_H):
    p = step_p(P, st, beta, h)
    q = step_q(P, st, p, beta, h)
    t = step_t(P, st, p, q, beta, h)
    s = step_s(P, st, p, q, t, beta, h)
    return dict(p=p, q=q, t=t, s=s, lam=st["lam"] - gamma * beta * (p - q),
                z=st["z"] - gamma * beta * (t - s))


def iterate(P, st, k, beta, gamma, h=DEFAULT_H, return_prev=False):
    prev = st
    for _ in range(k):
        prev, st = st, sweep(P, st, beta, gamma, h)
    return (st, prev) if return_prev else st


def split_f(P, p, q, t, s):
    """f of eq. 2 with Sigma1 = diag(c, S) per edge."""
    ei, ej = P["ei"], P["ej"]
    r = hat(t[ej] - s[ei]) - qmul(qmul(q[ei], hat(P["tm"])), qconj(p[ei]))
    return (r.unsqueeze(-2) @ P["Sig1"] @ r.unsqueeze(-1)).sum()


def split_g(P, p, q):
    ei, ej = P["ei"], P["ej"]
    a = qmul(qmul(qconj(p[ej]), q[ei]), P["qm"]) - ONE
    return (P["kappa"] * (a * a).sum(1)).sum()


def cost(P, p, t):
    """Model (1) with the per-edge Sigma1 at p = q, s = t."""
    return split_f(P, p, p, t, t) + split_g(P, p, p)


def aug_lagrangian(P, st, beta):
    p, q, t, s, lam, z = (st[k] for k in ("p", "q", "t", "s", "lam", "z"))
    return (split_f(P, p, q, t, s) + split_g(P, p, q) - (lam * (p - q)).sum()
            + 0.5 * beta * ((p - q) ** 2).sum() - (z * (t - s)).sum() + 0.5 * beta * ((t - s) ** 2).sum())
