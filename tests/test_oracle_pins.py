"""Pins of the FP64 oracle's iteration against what the paper and the
mathematics fix, independently of the oracle's own closed forms:

  V1  noise-free graph at ground truth is a fixed point with zero cost
  V2  unit norm of p after every sweep, R(p) in SO(3)
  V3  equivariance under a global rigid transform (Model section)
  V4  the multiplier identities implied by the q- and s-subproblem optimality
      conditions (App. D, optimality of each subproblem / proof of Lemma 3)
  V5  each phase is the argmin of its subproblem (eq. 3a-3d): brute force on
      the sphere for p, vanishing gradient for q, t, s
  V6  tree graphs reach zero cost
  V7  with rotations frozen, t/s/z converge to the weighted translation least
      squares (library lstsq)
  V8  tiny graphs: final cost equals an independent Levenberg-Marquardt local
      minimum of model (1) from the same start, and is not below the best of
      many random starts
  V9  merit L_beta + alpha1/(gamma beta) ||dlambda||^2 nonincreasing for large
      beta (Theorem 1)
  KKT converged points satisfy the stationarity system (Lemma, Optimality
      Conditions, App. D)
  cost of model (1) equals its rotation-matrix form with the quaternion
      distance identity of App. A.4
"""
import numpy as np
import pytest
import torch

import pgo_synth as S
from oracle import gn, prep
from oracle import pradmm as O
from oracle.quat import qmul, rotmat
from tests import qref

F64 = torch.float64


def abar(P):
    n = P["n"]
    d = (2 * O._sum_into(n, P["ei"], P["tau"] * (P["tm"] ** 2).sum(1) + P["kappa"])
         + 2 * O._sum_into(n, P["ej"], P["kappa"]))
    return float(d.mean())


def npstate(st):
    return {k: v.detach().numpy().copy() for k, v in st.items()}


def npprob(P):
    return {k: (v.numpy() if torch.is_tensor(v) else v) for k, v in P.items()}


def small_problem(seed=0, n=6, extra=5, sR=0.1, st=0.1, warm=3):
    g = S.random_small(n, extra, seed=seed, sigma_R=sR, sigma_t=st)
    P, p0, t0 = prep.prepare_graph(g)
    beta = 0.05 * abar(P)
    s = O.iterate(P, O.init_state(p0, t0), warm, beta, 1.4)  # non-trivial multipliers
    return P, s, beta


# ---------------------------------------------------------------------------
def test_V1_noise_free_fixed_point():
    for g in (S.circle(100, 10.0, 20, 10, 0.0, 0.0, init="gt"),
              S.grid(4, 4, 4, p=0.5, sigma_R=0.0, sigma_t=0.0, init="gt")):
        P, p0, t0 = prep.prepare_graph(g)
        st = O.init_state(p0, t0)
        beta = 0.01 * abar(P)
        st1 = O.iterate(P, st, 3, beta, 1.4)
        for k in st:
            sc = beta if k in ("lam", "z") else 1.0      # multipliers compared as lambda/beta, z/beta
            assert float((st1[k] - st[k]).abs().max()) / sc < 1e-12, k
        assert float(O.cost(P, p0, t0)) < 1e-20 * g.m * 1e4


def test_V2_unit_norm_and_so3():
    g = S.make_config("grid-1k")
    P, p0, t0 = prep.prepare_graph(g)
    st = O.init_state(p0, t0)
    beta = 0.01 * abar(P)
    for _ in range(10):
        st = O.sweep(P, st, beta, 1.4)
        assert float((st["p"].norm(dim=1) - 1).abs().max()) < 4e-16
        R = rotmat(st["p"])
        assert float((R.transpose(-1, -2) @ R - torch.eye(3, dtype=F64)).abs().max()) < 2e-15
        assert float((torch.linalg.det(R) - 1).abs().max()) < 2e-15


def test_V3_global_rigid_transform():
    P, st, beta = small_problem(seed=3)
    rng = np.random.default_rng(0)
    qg = torch.as_tensor(rng.standard_normal(4), dtype=F64)
    qg = qg / qg.norm()
    Rg = rotmat(qg)
    tg = torch.as_tensor(rng.standard_normal(3), dtype=F64)

    def transform(s):
        L = lambda x: qmul(qg.expand_as(x), x)
        return dict(p=L(s["p"]), q=L(s["q"]), lam=L(s["lam"]), t=s["t"] @ Rg.T + tg,
                    s=s["s"] @ Rg.T + tg, z=s["z"] @ Rg.T)

    a = O.iterate(P, transform(st), 5, beta, 1.4)
    b = transform(O.iterate(P, st, 5, beta, 1.4))
    for k in a:
        scale = 1.0 + float(b[k].abs().max())
        assert float((a[k] - b[k]).abs().max()) < 1e-11 * scale, k
    assert abs(float(O.cost(P, a["p"], a["t"])) - float(O.cost(P, b["p"], b["t"]))) < 1e-9


def _fd_grad(fun, x, h):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        g[i] = (fun(xp) - fun(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("gamma", [1.0, 1.4, 1.8])
def test_V4_multiplier_identities(gamma):
    """lambda^{k+1} = (1-g) lambda^k - g (grad_q (f+g)(p',q',t,s) + H2 dq)
       z^{k+1}      = (1-g) z^k      - g (grad_s f(p',q',t',s') + H4 ds)
    with the gradients taken by central differences of eq. (2)'s f and g
    (exact for these quadratics up to rounding)."""
    P, st, beta = small_problem(seed=1)
    h = O.DEFAULT_H
    new = O.sweep(P, st, beta, gamma)
    A, B = npstate(st), npstate(new)
    pp = npprob(P)
    ei, ej = pp["ei"], pp["ej"]
    fg_q = lambda q: (qref.f_split(ei, ej, pp["tau"], pp["tm"], B["p"], q, A["t"], A["s"])
                      + qref.g_split(ei, ej, pp["kappa"], pp["qm"], B["p"], q))
    gq = _fd_grad(fg_q, B["q"], 1e-3)
    lam_pred = (1 - gamma) * A["lam"] - gamma * (gq + h[1] * (B["q"] - A["q"]))
    assert np.abs(lam_pred - B["lam"]).max() < 1e-7 * (1 + np.abs(B["lam"]).max())
    f_s = lambda s: qref.f_split(ei, ej, pp["tau"], pp["tm"], B["p"], B["q"], B["t"], s)
    gs = _fd_grad(f_s, B["s"], 1e-3)
    z_pred = (1 - gamma) * A["z"] - gamma * (gs + h[3] * (B["s"] - A["s"]))
    assert np.abs(z_pred - B["z"]).max() < 1e-7 * (1 + np.abs(B["z"]).max())


def test_V5_each_phase_is_its_argmin():
    P, st, beta = small_problem(seed=2)
    h = O.DEFAULT_H
    A = npstate(st)
    pp = npprob(P)
    ei, ej, tau, kappa, tm, qm = pp["ei"], pp["ej"], pp["tau"], pp["kappa"], pp["tm"], pp["qm"]
    p1 = O.step_p(P, st, beta).numpy()
    # --- p: brute force over the unit sphere, vertex by vertex ---------------
    rng = np.random.default_rng(0)

    def phi(i, pv):
        out = np.nonzero(ei == i)[0]
        inn = np.nonzero(ej == i)[0]
        val = 0.0
        for e in out:
            r = (qref.hat(A["t"][ej[e]]) - qref.hat(A["s"][i])
                 - qref.qmul(qref.qmul(A["q"][i], qref.hat(tm[e])), qref.qconj(pv)))
            val += tau[e] * (r * r).sum(-1)
        for e in inn:
            r = qref.qmul(qref.qmul(qref.qconj(pv), A["q"][ei[e]]), qm[e]) - qref.ONE
            val += kappa[e] * (r * r).sum(-1)
        d = pv - A["q"][i]
        val = val - (d * A["lam"][i]).sum(-1) + 0.5 * beta * (d * d).sum(-1)
        dp = pv - A["p"][i]
        return val + 0.5 * h[0] * (dp * dp).sum(-1)

    for i in range(P["n"]):
        cands = []
        for sc in (1e-5, 1e-3, 1e-1, 1.0):
            c = p1[i] + sc * rng.standard_normal((5000, 4))
            cands.append(c / np.linalg.norm(c, axis=1, keepdims=True))
        cands = np.concatenate(cands)
        best = phi(i, p1[i])
        vals = phi(i, cands)
        assert vals.min() >= best - 1e-9 * abs(best), i
    # --- q, t, s: the subproblem gradient vanishes ----------------------------
    P1 = torch.as_tensor(p1)
    q1 = O.step_q(P, st, P1, beta).numpy()
    psi_q = lambda q: (qref.f_split(ei, ej, tau, tm, p1, q, A["t"], A["s"])
                       + qref.g_split(ei, ej, kappa, qm, p1, q)
                       - (A["lam"] * (p1 - q)).sum() + 0.5 * beta * ((p1 - q) ** 2).sum()
                       + 0.5 * h[1] * ((q - A["q"]) ** 2).sum())
    gq = _fd_grad(psi_q, q1, 1e-3)
    assert np.abs(gq).max() < 1e-6 * (1 + beta)
    Q1 = torch.as_tensor(q1)
    t1 = O.step_t(P, st, P1, Q1, beta).numpy()
    psi_t = lambda t: (qref.f_split(ei, ej, tau, tm, p1, q1, t, A["s"])
                       - (A["z"] * (t - A["s"])).sum() + 0.5 * beta * ((t - A["s"]) ** 2).sum()
                       + 0.5 * h[2] * ((t - A["t"]) ** 2).sum())
    assert np.abs(_fd_grad(psi_t, t1, 1e-3)).max() < 1e-6 * (1 + beta)
    T1 = torch.as_tensor(t1)
    s1 = O.step_s(P, st, P1, Q1, T1, beta).numpy()
    psi_s = lambda s: (qref.f_split(ei, ej, tau, tm, p1, q1, t1, s)
                       - (A["z"] * (t1 - s)).sum() + 0.5 * beta * ((t1 - s) ** 2).sum()
                       + 0.5 * h[3] * ((s - A["s"]) ** 2).sum())
    assert np.abs(_fd_grad(psi_s, s1, 1e-3)).max() < 1e-6 * (1 + beta)


def test_V6_tree_reaches_zero_cost():
    rng = np.random.default_rng(5)
    n = 12
    par = np.array([rng.integers(0, k) for k in range(1, n)])
    kids = np.arange(1, n)
    R_gt = S.so3_exp(rng.standard_normal((n, 3)))
    t_gt = rng.standard_normal((n, 3)) * 2
    g = S._measure(R_gt, t_gt, par, kids, 0.1, 0.1, rng, init="gt")
    g.R0 = g.R0 @ S.so3_exp(rng.standard_normal((n, 3)) * 0.2)
    g.t0 = g.t0 + rng.standard_normal((n, 3)) * 0.3
    P, p0, t0 = prep.prepare_graph(g)
    c0 = float(O.cost(P, p0, t0))
    st = O.iterate(P, O.init_state(p0, t0), 2000, 0.01 * abar(P), 1.4)
    assert float(O.cost(P, st["p"], st["t"])) < 1e-5 * c0


def test_V7_frozen_rotations_give_translation_least_squares():
    g = S.grid(3, 3, 2, p=0.7, sigma_R=0.05, sigma_t=0.1, seed=4)
    P, p0, t0 = prep.prepare_graph(g)
    n, ei, ej = P["n"], P["ei"].numpy(), P["ej"].numpy()
    beta = 50.0
    st = O.init_state(p0, t0)
    for _ in range(3000):
        t = O.step_t(P, st, p0, p0, beta)
        s = O.step_s(P, st, p0, p0, t, beta)
        st = dict(st, t=t, s=s, z=st["z"] - 1.4 * beta * (t - s))
    c = (rotmat(p0)[ei] @ P["tm"][..., None])[..., 0].numpy()
    w = np.sqrt(P["tau"].numpy())
    A = np.zeros((3 * len(ei), 3 * n))
    b = np.zeros(3 * len(ei))
    for e in range(len(ei)):
        for d in range(3):
            A[3 * e + d, 3 * ej[e] + d] = w[e]
            A[3 * e + d, 3 * ei[e] + d] = -w[e]
            b[3 * e + d] = w[e] * c[e, d]
    A0 = A[:, 3:]                                   # gauge: t_0 fixed at 0
    sol = np.linalg.lstsq(A0, b, rcond=None)[0].reshape(n - 1, 3)
    got = (st["t"] - st["t"][0]).numpy()[1:]
    assert np.abs(got - sol).max() < 1e-8


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_V8_tiny_graphs_vs_gauss_newton(seed):
    g = S.random_small(5, 4, seed=seed, sigma_R=0.1, sigma_t=0.1)
    P, p0, t0 = prep.prepare_graph(g)
    pp = npprob(P)
    args = (pp["ei"], pp["ej"], pp["qm"], pp["tm"], pp["kappa"], pp["tau"])
    c_gn, _, _ = gn.local_min(p0.numpy(), t0.numpy(), *args)
    c_ms = gn.multistart_min(g.n, *args, starts=20, seed=seed)
    st = O.iterate(P, O.init_state(p0, t0), 3000, 0.03 * abar(P), 1.4)
    c = float(O.cost(P, st["p"], st["t"]))
    assert abs(c - c_gn) <= 1e-9 * c_gn
    assert c >= c_ms * (1 - 1e-9)
    assert abs(gn.model_cost(st["p"].numpy(), st["t"].numpy(), *args) - c) < 1e-10 * c


@pytest.mark.parametrize("gamma", [1.0, 1.4])
def test_V9_merit_nonincreasing_for_large_beta(gamma):
    g = S.random_small(6, 5, seed=2, sigma_R=0.1, sigma_t=0.1)
    P, p0, t0 = prep.prepare_graph(g)
    beta = 10 * abar(P)
    a1 = abs(1 - gamma) / (1 - abs(1 - gamma))
    st = O.init_state(p0, t0)
    vals = []
    for _ in range(200):
        prev, st = st, O.sweep(P, st, beta, gamma)
        dl = float(((st["lam"] - prev["lam"]) ** 2).sum())
        vals.append(float(O.aug_lagrangian(P, st, beta)) + a1 / (gamma * beta) * dl)
    v = np.array(vals)
    assert np.all(np.diff(v[10:]) <= 1e-10 * np.abs(v[10:]).max())


def test_KKT_at_convergence():
    g = S.random_small(5, 4, seed=0, sigma_R=0.1, sigma_t=0.1)
    P, p0, t0 = prep.prepare_graph(g)
    st = O.iterate(P, O.init_state(p0, t0), 3000, 0.03 * abar(P), 1.4)
    A = npstate(st)
    pp = npprob(P)
    ei, ej = pp["ei"], pp["ej"]
    fg = lambda p, q, t, s: (qref.f_split(ei, ej, pp["tau"], pp["tm"], p, q, t, s)
                             + qref.g_split(ei, ej, pp["kappa"], pp["qm"], p, q))
    p, q, t, s, lam, z = (A[k] for k in ("p", "q", "t", "s", "lam", "z"))
    scale = 1 + np.abs(lam).max() + np.abs(z).max()
    assert np.abs(p - q).max() < 1e-9 and np.abs(t - s).max() < 1e-9
    g1 = _fd_grad(lambda x: fg(x, q, t, s), p, 1e-4) - lam
    g1 = g1 - (g1 * p).sum(1, keepdims=True) * p            # projection onto T_p S^3
    g2 = _fd_grad(lambda x: fg(p, x, t, s), q, 1e-4) + lam
    g3 = _fd_grad(lambda x: fg(p, q, x, s), t, 1e-4) - z
    g4 = _fd_grad(lambda x: fg(p, q, t, x), s, 1e-4) + z
    for gr in (g1, g2, g3, g4):
        assert np.abs(gr).max() < 1e-6 * scale


def test_cost_equals_rotation_matrix_form():
    g = S.make_config("grid-1k")
    P, p0, t0 = prep.prepare_graph(g)
    pp = npprob(P)
    ei, ej = pp["ei"], pp["ej"]
    Ri, Rj = g.R0[ei], g.R0[ej]
    rt = t0.numpy()[ej] - t0.numpy()[ei] - np.einsum("kab,kb->ka", Ri, g.tm)
    Rerr = np.transpose(Ri @ g.Rm, (0, 2, 1)) @ Rj
    th = np.arccos(np.clip((np.trace(Rerr, axis1=1, axis2=2) - 1) / 2, -1, 1))
    ref = (g.tau * (rt ** 2).sum(1)).sum() + (g.kappa * (2 * np.sin(th / 4)) ** 2).sum()
    assert abs(float(O.cost(P, p0, t0)) - ref) < 1e-9 * ref
