"""PRADMM iteration, FP64, CPU -- the oracle (test infrastructure only).

Follows the iterative scheme (3a)-(3f) and Alg. 1 step by step, with each
subproblem in the G-matrix form of App. B:

  p-subproblem (App. B.1, Alg. 1 step 2, scalar Sigma case):
      G1 = M(q_i) M(t~_ij) D                 for (i,j) in E_i^out
      G2 = W(q~_li) W(q_l) D                 for (l,i) in E_i^in
      b1 = -2 sum_out G1^T Sigma1 (t~_j - s~_i) - 2 sum_in G2^T Sigma2 1
           - beta q_i - lambda_i - H1 p_i
      p_i = -b1 / ||b1||        (p_i kept when b1 = 0)
  q-subproblem (App. B.2, Alg. 1 step 3):
      G3 = W(p_i)^T W(t~_ij),  G4 = W(q~_ij) M(p_j)^T     for (i,j) in E_i^out
      A2 = sum_out 2 (G3^T Sigma1 G3 + G4^T Sigma2 G4) + beta I + H2
      b2 = sum_out 2 (G3^T Sigma1 (t~_j - s~_i) + G4^T Sigma2 1) + beta p_i
           - lambda_i + H2 q_i
      q_i = A2^{-1} b2          (a dense 4x4 solve)
  t-subproblem (App. B.3, Alg. 1 step 4), c_li = Im(q_l t~_li p_l^*):
      A3 = sum_in 2 Sigma1^ + beta I + H3,
      b3 = sum_in 2 Sigma1^ (s_l + c_li) + beta s_i + z_i + H3 t_i
  s-subproblem (App. B.4, Alg. 1 step 5), c_ij = Im(q_i t~_ij p_i^*):
      A4 = sum_out 2 Sigma1^ + beta I + H4,
      b4 = sum_out 2 Sigma1^ (t_j - c_ij) + beta t_i - z_i + H4 s_i
  multipliers (eq. 3e, 3f, Alg. 1 step 6), relaxation gamma in (0, 2):
      lambda -= gamma beta (p - q),   z -= gamma beta (t - s)

Readings of the text that this file takes (each is listed with its reason in
the design notes of the repository):
  * the in-edge matrix G2 carries the factor D (the printed G2 lacks it, but
    only with D does G2 p_i equal p_i^* q_l q~_li, the term of g in eq. 2);
  * c_li is built from the tail l of the in-edge (the printed indices of
    App. B.3 are those of an out-edge);
  * the s-subproblem's argmin variable is s_i (printed as t_i);
  * proximal centres are x^k (App. B prints x^{k+1/2}, a left-over of an
    inertial variant whose extrapolation is never defined);
  * Sigma1 = tau_e I_4 (so c = tau_e) and Sigma2 = kappa_e I_4 per edge, one
    penalty beta = beta1 = beta2, H_s = h_s I;
  * q^0 = p^0, s^0 = t^0, lambda^0 = 0, z^0 = 0 in R^{3n}.

Within one phase every vertex reads the previous phase's values (Jacobi
inside a phase, Gauss-Seidel across phases), as eq. 3 prescribes.
"""
import torch

from .quat import F64, D4, ONE, Mmat, Wmat, hat, mv, qconj, qmul

DEFAULT_H = (1.0, 1e-3, 1e-3, 1e-3)   # H1 in {0.1, 1, 10}, H2..4 = 0.001 (experiment settings)


def _sum_into(n, idx, vals):
    out = torch.zeros((n,) + tuple(vals.shape[1:]), dtype=vals.dtype)
    return out.index_add(0, idx, vals)


def _T(A):
    return A.transpose(-1, -2)


def init_state(p0, t0):
    n = p0.shape[0]
    return dict(p=p0.clone(), q=p0.clone(), t=t0.clone(), s=t0.clone(),
                lam=torch.zeros(n, 4, dtype=F64), z=torch.zeros(n, 3, dtype=F64))


def step_p(P, st, beta, h=DEFAULT_H):
    """p-subproblem, eq. (3a) / App. B.1; returns p^{k+1}."""
    n, ei, ej = P["n"], P["ei"], P["ej"]
    tau, kappa, tm, qm = P["tau"], P["kappa"], P["tm"], P["qm"]
    q, t, s, lam, p = st["q"], st["t"], st["s"], st["lam"], st["p"]
    G1 = Mmat(q[ei]) @ Mmat(hat(tm)) @ D4                      # out-edges (i -> j), i = ei
    r = hat(t[ej] - s[ei])                                     # t~_j^k - s~_i^k
    out_terms = 2.0 * tau[:, None] * mv(_T(G1), r)
    G2 = Wmat(qm) @ Wmat(q[ei]) @ D4                           # in-edges (l -> i), l = ei, i = ej
    in_terms = 2.0 * kappa[:, None] * mv(_T(G2), ONE.expand(G2.shape[0], 4))
    b1 = -_sum_into(n, ei, out_terms) - _sum_into(n, ej, in_terms) - beta * q - lam - h[0] * p
    nb = b1.norm(dim=1, keepdim=True)
    return torch.where(nb > 0, -b1 / torch.where(nb > 0, nb, torch.ones_like(nb)), p)


def step_q(P, st, p_new, beta, h=DEFAULT_H):
    """q-subproblem, eq. (3b) / App. B.2; returns q^{k+1}."""
    n, ei, ej = P["n"], P["ei"], P["ej"]
    tau, kappa, tm, qm = P["tau"], P["kappa"], P["tm"], P["qm"]
    q, t, s, lam = st["q"], st["t"], st["s"], st["lam"]
    G3 = _T(Wmat(p_new[ei])) @ Wmat(hat(tm))
    G4 = Wmat(qm) @ _T(Mmat(p_new[ej]))
    r = hat(t[ej] - s[ei])
    A_e = 2.0 * (tau[:, None, None] * (_T(G3) @ G3) + kappa[:, None, None] * (_T(G4) @ G4))
    b_e = 2.0 * (tau[:, None] * mv(_T(G3), r) + kappa[:, None] * mv(_T(G4), ONE.expand(G4.shape[0], 4)))
    I4 = torch.eye(4, dtype=F64)
    A2 = _sum_into(n, ei, A_e) + (beta + h[1]) * I4
    b2 = _sum_into(n, ei, b_e) + beta * p_new - lam + h[1] * q
    return torch.linalg.solve(A2, b2)


def _c(p, q, tm, tail):
    """c_e = Im(q_l t~_e p_l^*) with l the tail of edge e (App. B.3 prints the
    indices of an out-edge; the t-subproblem sums over in-edges)."""
    return qmul(qmul(q[tail], hat(tm)), qconj(p[tail]))[:, 1:]


def step_t(P, st, p_new, q_new, beta, h=DEFAULT_H):
    """t-subproblem, eq. (3c) / App. B.3; returns t^{k+1}."""
    n, ei, ej, tau, tm = P["n"], P["ei"], P["ej"], P["tau"], P["tm"]
    t, s, z = st["t"], st["s"], st["z"]
    c = _c(p_new, q_new, tm, ei)
    I3 = torch.eye(3, dtype=F64)
    A3 = _sum_into(n, ej, 2.0 * tau[:, None, None] * I3) + (beta + h[2]) * I3
    b3 = _sum_into(n, ej, 2.0 * tau[:, None] * (s[ei] + c)) + beta * s + z + h[2] * t
    return torch.linalg.solve(A3, b3)


def step_s(P, st, p_new, q_new, t_new, beta, h=DEFAULT_H):
    """s-subproblem, eq. (3d) / App. B.4; returns s^{k+1}."""
    n, ei, ej, tau, tm = P["n"], P["ei"], P["ej"], P["tau"], P["tm"]
    s, z = st["s"], st["z"]
    c = _c(p_new, q_new, tm, ei)
    I3 = torch.eye(3, dtype=F64)
    A4 = _sum_into(n, ei, 2.0 * tau[:, None, None] * I3) + (beta + h[3]) * I3
    b4 = _sum_into(n, ei, 2.0 * tau[:, None] * (t_new[ej] - c)) + beta * t_new - z + h[3] * s
    return torch.linalg.solve(A4, b4)


def sweep(P, st, beta, gamma, h=DEFAULT_H):
    """One iteration k -> k+1 of Alg. 1 (steps 2-6). Pure function."""
    p = step_p(P, st, beta, h)
    q = step_q(P, st, p, beta, h)
    t = step_t(P, st, p, q, beta, h)
    s = step_s(P, st, p, q, t, beta, h)
    lam = st["lam"] - gamma * beta * (p - q)
    z = st["z"] - gamma * beta * (t - s)
    return dict(p=p, q=q, t=t, s=s, lam=lam, z=z)


def iterate(P, st, k, beta, gamma, h=DEFAULT_H, return_prev=False):
    prev = st
    for _ in range(k):
        prev, st = st, sweep(P, st, beta, gamma, h)
    return (st, prev) if return_prev else st


# ----------------------------------------------------------------------------
# objective functions
# ----------------------------------------------------------------------------
def cost(P, p, t):
    """Model (1): sum_e ||t~_j - t~_i - p_i t~_ij p_i^*||^2_{Sigma1}
    + ||p_j^* p_i q~_ij - 1||^2_{Sigma2} at (p, t)."""
    ei, ej, tau, kappa, tm, qm = P["ei"], P["ej"], P["tau"], P["kappa"], P["tm"], P["qm"]
    rt = hat(t[ej]) - hat(t[ei]) - qmul(qmul(p[ei], hat(tm)), qconj(p[ei]))
    rq = qmul(qmul(qconj(p[ej]), p[ei]), qm) - ONE
    return (tau * (rt * rt).sum(1) + kappa * (rq * rq).sum(1)).sum()


def split_f(P, p, q, t, s):
    """f of eq. (2)."""
    ei, ej, tau, tm = P["ei"], P["ej"], P["tau"], P["tm"]
    r = hat(t[ej]) - hat(s[ei]) - qmul(qmul(q[ei], hat(tm)), qconj(p[ei]))
    return (tau * (r * r).sum(1)).sum()


def split_g(P, p, q):
    """g of eq. (2)."""
    ei, ej, kappa, qm = P["ei"], P["ej"], P["kappa"], P["qm"]
    r = qmul(qmul(qconj(p[ej]), q[ei]), qm) - ONE
    return (kappa * (r * r).sum(1)).sum()


def aug_lagrangian(P, st, beta):
    """L_beta of the PRADMM section (beta1 = beta2 = beta)."""
    p, q, t, s, lam, z = (st[k] for k in ("p", "q", "t", "s", "lam", "z"))
    return (split_f(P, p, q, t, s) + split_g(P, p, q)
            - (lam * (p - q)).sum() + 0.5 * beta * ((p - q) ** 2).sum()
            - (z * (t - s)).sum() + 0.5 * beta * ((t - s) ** 2).sum())


def residuals(P, prev, st, beta):
    """[||p-q||, ||t-s||, e, beta||dq||, beta||ds||, F] where e is the
    iteration residual of App. E.1:
        e = (||dlambda||^2 + ||dz||^2)/beta + beta (||dq||^2 + ||dt||^2)."""
    d = {k: st[k] - prev[k] for k in ("q", "t", "s", "lam", "z")}
    sq = lambda x: float((x * x).sum())
    e = (sq(d["lam"]) + sq(d["z"])) / beta + beta * (sq(d["q"]) + sq(d["t"]))
    return [sq(st["p"] - st["q"]) ** 0.5, sq(st["t"] - st["s"]) ** 0.5, e,
            beta * sq(d["q"]) ** 0.5, beta * sq(d["s"]) ** 0.5, float(cost(P, st["p"], st["t"]))]


def rotations(p):
    """Rotation matrices R(p_i) (App. A.2 sandwich)."""
    from .quat import rotmat
    return rotmat(p)


# ----------------------------------------------------------------------------
# reference adjoint (automatic differentiation through the unrolled sweeps)
# ----------------------------------------------------------------------------
def unrolled_loss(P, p0, t0, K, beta, gamma, t_target, h=DEFAULT_H):
    st = init_state(p0, t0)
    for _ in range(K):
        st = sweep(P, st, beta, gamma, h)
    return ((st["t"] - t_target) ** 2).sum()


def unrolled_grad(P, p0, t0, K, beta, gamma, t_target, h=DEFAULT_H):
    """Loss sum_i ||t_i^K - t_i^target||^2 after K sweeps and its gradient
    with respect to kappa_e, tau_e, t~_e and the right rotation perturbation
    omega_e (R~_e <- R~_e Exp(omega_e), i.e. q~_e <- q~_e [cos(|w|/2),
    sin(|w|/2) w/|w|]), whose gradient at 0 is 1/2 Im(q~_e^* g_q~)."""
    kappa = P["kappa"].clone().requires_grad_(True)
    tau = P["tau"].clone().requires_grad_(True)
    tm = P["tm"].clone().requires_grad_(True)
    qm = P["qm"].clone().requires_grad_(True)
    P2 = dict(P, kappa=kappa, tau=tau, tm=tm, qm=qm)
    L = unrolled_loss(P2, p0, t0, K, beta, gamma, t_target, h)
    gk, gt, gtm, gq = torch.autograd.grad(L, [kappa, tau, tm, qm])
    g_omega = 0.5 * qmul(qconj(qm.detach()), gq)[:, 1:]
    return float(L.detach()), dict(kappa=gk, tau=gt, tm=gtm, omega=g_omega)
