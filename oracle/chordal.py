"""Rotation-matrix (chordal) rendering of the PRADMM sweep -- oracle, FP64,
test infrastructure only.

This is not the paper's quaternion model: it is the same splitting applied
to the chordal pose-graph cost (chordal distance of App. A.4),

    F(R, t) = sum_e tau_e |t_j - t_i - R_i t~_e|^2 + kappa_e |R_i R~_e - R_j|_F^2,

split with duplicates P = Q (P_i in SO(3), Q_i free 3x3) and t = s:

    f = sum_e tau_e |t_j - s_i - P_i t~_e|^2,   g = sum_e kappa_e |Q_i R~_e - P_j|_F^2,
    L_beta = f + g - <Lambda, P - Q> + beta/2 |P - Q|^2 - <z, t - s> + beta/2 |t - s|^2,

and the iteration (3a)-(3f) with proximal terms h_s/2 |x - x^k|^2.  Every
subproblem is closed form:

  P_i = argmax_{P in SO(3)} <P, M_i>,  M_i = 2 sum_out tau (t_j - s_i) t~^T
        + 2 sum_in kappa Q_l R~_li + beta Q_i + Lambda_i + H1 P_i
        (using |P t~| = |t~|, |P|^2 = 3: f, g and the penalty are linear in P),
        solved by the SVD M = U S V^T: P = U diag(1, 1, det(U V^T)) V^T;
  Q_i = (2 sum_out kappa P_j R~^T + beta P_i - Lambda_i + H2 Q_i) / (2 sum_out kappa + beta + H2);
  t_i = (2 sum_in tau (s_l + P_l t~) + beta s_i + z_i + H3 t_i) / (2 sum_in tau + beta + H3);
  s_i = (2 sum_out tau (t_j - P_i t~) + beta t_i - z_i + H4 s_i) / (2 sum_out tau + beta + H4);
  Lambda -= gamma beta (P - Q),   z -= gamma beta (t - s).
"""
import torch

from .pradmm import DEFAULT_H, _sum_into
from .quat import F64


def project_so3(M):
    U, _, Vh = torch.linalg.svd(M)
    d = torch.linalg.det(U @ Vh)
    D = torch.diag_embed(torch.stack([torch.ones_like(d), torch.ones_like(d), d], -1))
    return U @ D @ Vh


def prepare(n, ei, ej, Rm, tm, kappa, tau, R0, t0):
    ei = torch.as_tensor(ei, dtype=torch.int64)
    ej = torch.as_tensor(ej, dtype=torch.int64)
    m = ei.shape[0]
    prob = dict(n=n, m=m, ei=ei, ej=ej,
                Rm=project_so3(torch.as_tensor(Rm, dtype=F64).reshape(m, 3, 3)),
                tm=torch.as_tensor(tm, dtype=F64).reshape(m, 3).clone(),
                kappa=torch.as_tensor(kappa, dtype=F64).reshape(m).clone(),
                tau=torch.as_tensor(tau, dtype=F64).reshape(m).clone())
    P0 = project_so3(torch.as_tensor(R0, dtype=F64).reshape(n, 3, 3))
    return prob, P0, torch.as_tensor(t0, dtype=F64).reshape(n, 3).clone()


def prepare_graph(g):
    return prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau, g.R0, g.t0)


def init_state(P0, t0):
    n = P0.shape[0]
    return dict(P=P0.clone(), Q=P0.clone(), t=t0.clone(), s=t0.clone(),
                L=torch.zeros(n, 3, 3, dtype=F64), z=torch.zeros(n, 3, dtype=F64))


def _mv(A, x):
    return (A @ x.unsqueeze(-1)).squeeze(-1)


def step_P(Pb, st, beta, h=DEFAULT_H):
    n, ei, ej, tau, kappa, tm, Rm = (Pb[k] for k in ("n", "ei", "ej", "tau", "kappa", "tm", "Rm"))
    r = st["t"][ej] - st["s"][ei]
    out_terms = 2.0 * tau[:, None, None] * (r.unsqueeze(-1) @ tm.unsqueeze(-2))
    in_terms = 2.0 * kappa[:, None, None] * (st["Q"][ei] @ Rm)           # in-edges of the head ej
    M = (_sum_into(n, ei, out_terms) + _sum_into(n, ej, in_terms) + beta * st["Q"] + st["L"]
         + h[0] * st["P"])
    return project_so3(M)


def step_Q(Pb, st, P_new, beta, h=DEFAULT_H):
    n, ei, ej, kappa, Rm = (Pb[k] for k in ("n", "ei", "ej", "kappa", "Rm"))
    num = (_sum_into(n, ei, 2.0 * kappa[:, None, None] * (P_new[ej] @ Rm.transpose(-1, -2)))
           + beta * P_new - st["L"] + h[1] * st["Q"])
    den = _sum_into(n, ei, 2.0 * kappa) + beta + h[1]
    return num / den[:, None, None]


def step_t(Pb, st, P_new, beta, h=DEFAULT_H):
    n, ei, ej, tau, tm = (Pb[k] for k in ("n", "ei", "ej", "tau", "tm"))
    c = _mv(P_new[ei], tm)
    num = _sum_into(n, ej, 2.0 * tau[:, None] * (st["s"][ei] + c)) + beta * st["s"] + st["z"] + h[2] * st["t"]
    den = _sum_into(n, ej, 2.0 * tau) + beta + h[2]
    return num / den[:, None]


def step_s(Pb, st, P_new, t_new, beta, h=DEFAULT_H):
    n, ei, ej, tau, tm = (Pb[k] for k in ("n", "ei", "ej", "tau", "tm"))
    c = _mv(P_new[ei], tm)
    num = _sum_into(n, ei, 2.0 * tau[:, None] * (t_new[ej] - c)) + beta * t_new - st["z"] + h[3] * st["s"]
    den = _sum_into(n, ei, 2.0 * tau) + beta + h[3]
    return num / den[:, None]


def sweep(Pb, st, beta, gamma, h=DEFAULT_H):
    P = step_P(Pb, st, beta, h)
    Q = step_Q(Pb, st, P, beta, h)
    t = step_t(Pb, st, P, beta, h)
    s = step_s(Pb, st, P, t, beta, h)
    L = st["L"] - gamma * beta * (P - Q)
    z = st["z"] - gamma * beta * (t - s)
    return dict(P=P, Q=Q, t=t, s=s, L=L, z=z)


def iterate(Pb, st, k, beta, gamma, h=DEFAULT_H, return_prev=False):
    prev = st
    for _ in range(k):
        prev, st = st, sweep(Pb, st, beta, gamma, h)
    return (st, prev) if return_prev else st


def cost(Pb, P, t):
    ei, ej, tau, kappa, tm, Rm = (Pb[k] for k in ("ei", "ej", "tau", "kappa", "tm", "Rm"))
    rt = t[ej] - t[ei] - _mv(P[ei], tm)
    rr = P[ei] @ Rm - P[ej]
    return (tau * (rt * rt).sum(1) + kappa * (rr * rr).sum((1, 2))).sum()


def aug_lagrangian(Pb, st, beta):
    ei, ej, tau, kappa, tm, Rm = (Pb[k] for k in ("ei", "ej", "tau", "kappa", "tm", "Rm"))
    P, Q, t, s, L, z = (st[k] for k in ("P", "Q", "t", "s", "L", "z"))
    rf = t[ej] - s[ei] - _mv(P[ei], tm)
    rg = Q[ei] @ Rm - P[ej]
    return ((tau * (rf * rf).sum(1)).sum() + (kappa * (rg * rg).sum((1, 2))).sum()
            - (L * (P - Q)).sum() + 0.5 * beta * ((P - Q) ** 2).sum()
            - (z * (t - s)).sum() + 0.5 * beta * ((t - s) ** 2).sum())


def residuals(Pb, prev, st, beta):
    """[|P-Q|, |t-s|, e, beta|dQ|, beta|ds|, F] as for the quaternion model."""
    sq = lambda x: float((x * x).sum())
    d = {k: st[k] - prev[k] for k in ("Q", "t", "s", "L", "z")}
    e = (sq(d["L"]) + sq(d["z"])) / beta + beta * (sq(d["Q"]) + sq(d["t"]))
    return [sq(st["P"] - st["Q"]) ** 0.5, sq(st["t"] - st["s"]) ** 0.5, e,
            beta * sq(d["Q"]) ** 0.5, beta * sq(d["s"]) ** 0.5, float(cost(Pb, st["P"], st["t"]))]
