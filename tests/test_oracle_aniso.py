"""Pins of the general-Sigma oracle (oracle/aniso.py): it reduces to the
pinned scalar oracle when every S_e = tau_e I; its p-step (Alg. 2) is the
global minimiser on the sphere (brute force) and satisfies Lemma B.1 (i);
the hard case; Q/T/S steps are their subproblems' argmins (vanishing
gradient of the split objective written out here); noise-free fixed point."""
import numpy as np
import pytest
import torch

import pgo_synth as S
from oracle import aniso as A
from oracle import prep
from oracle import pradmm as O

F64 = torch.float64


def abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def setup(g, info):
    P, p0, t0 = A.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, info, g.R0, g.t0)
    return P, O.init_state(p0, t0)


def test_isotropic_reduces_to_the_scalar_oracle():
    g = S.grid(4, 3, 3, p=0.5, sigma_R=0.05, sigma_t=0.1, seed=3)
    beta = 0.05 * abar(g)
    P, st = setup(g, g.tau[:, None, None] * np.eye(3))
    Ps, p0, t0 = prep.prepare_graph(g)
    a = A.iterate(P, st, 6, beta, 1.4)
    b = O.iterate(Ps, O.init_state(p0, t0), 6, beta, 1.4)
    for k in a:
        sc = beta if k in ("lam", "z") else 1.0
        assert float((a[k] - b[k]).abs().max()) / sc < 1e-10, k


def _objective(Aq, bq, x):
    return 0.5 * x @ Aq @ x + bq @ x


def test_p_step_is_the_global_minimiser_on_the_sphere():
    g = S.random_small(6, 5, seed=2, sigma_R=0.1, sigma_t=0.1)
    info = S.random_info(g.m, g.tau, 20.0, seed=1)
    P, st = setup(g, info)
    st = A.iterate(P, st, 3, 0.05 * abar(g), 1.4)
    rng = np.random.default_rng(0)
    for trial in range(30):
        M = rng.standard_normal((4, 4))
        Aq = M + M.T + rng.uniform(-3, 3) * np.eye(4)   # indefinite as well
        bq = rng.standard_normal(4) * rng.choice([1e-3, 0.3, 3.0])
        x, lam = A.trs_sphere(Aq, bq, np.array([1.0, 0, 0, 0]))
        assert abs(np.linalg.norm(x) - 1) < 1e-10
        assert np.abs((Aq + lam * np.eye(4)) @ x + bq).max() < 1e-10 * (1 + np.abs(bq).max())
        if np.abs(bq).max() > 0.1:   # Alg. 2's 8x8 eigenvalue gives the same multiplier
            assert abs(A.alg2_multiplier(Aq, bq) - lam) < 1e-7 * (1 + abs(lam))
        assert np.linalg.eigvalsh(Aq + lam * np.eye(4))[0] > -1e-9
        Y = rng.standard_normal((20000, 4))
        Y /= np.linalg.norm(Y, axis=1, keepdims=True)
        vals = 0.5 * np.einsum("ka,ab,kb->k", Y, Aq, Y) + Y @ bq
        assert _objective(Aq, bq, x) <= vals.min() + 1e-12
    # and on the real p-subproblem of a sweep
    p1 = A.step_p(P, st, 0.05 * abar(g))
    assert float((p1.norm(dim=1) - 1).abs().max()) < 1e-10


def test_hard_case():
    w = np.array([-2.0, -2.0, 1.0, 3.0])
    V = np.linalg.qr(np.random.default_rng(5).standard_normal((4, 4)))[0]
    Aq = V @ np.diag(w) @ V.T
    bq = V[:, 2] * 0.5 + V[:, 3] * 0.2          # orthogonal to the lowest eigenspace
    x, lam = A.trs_sphere(Aq, bq, V[:, 0])
    assert abs(lam - 2.0) < 1e-9
    assert abs(np.linalg.norm(x) - 1) < 1e-12
    assert np.abs((Aq + lam * np.eye(4)) @ x + bq).max() < 1e-9
    Y = np.random.default_rng(1).standard_normal((50000, 4))
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    vals = 0.5 * np.einsum("ka,ab,kb->k", Y, Aq, Y) + Y @ bq
    assert _objective(Aq, bq, x) <= vals.min() + 1e-12
    # every minimiser is x0 + y with y in span(V0, V1), |y|^2 = 1 - |x0|^2;
    # the step takes the one nearest the previous iterate
    x0 = -(V[:, 2] * 0.5 / (1.0 + 2.0) + V[:, 3] * 0.2 / (3.0 + 2.0))
    r = np.sqrt(1.0 - x0 @ x0)
    assert np.abs(x - (x0 + r * V[:, 0])).max() < 1e-12
    prev = V[:, 0] - 2.0 * V[:, 1] + 0.7 * V[:, 2]
    x2, _ = A.trs_sphere(Aq, bq, prev)
    u = (V[:, 0] - 2.0 * V[:, 1]) / np.sqrt(5.0)
    assert np.abs(x2 - (x0 + r * u)).max() < 1e-12
    ang = np.random.default_rng(2).uniform(0, 2 * np.pi, 2000)
    cand = x0[None] + r * (np.cos(ang)[:, None] * V[:, 0] + np.sin(ang)[:, None] * V[:, 1])
    assert np.allclose(0.5 * np.einsum("ka,ab,kb->k", cand, Aq, cand) + cand @ bq,
                       _objective(Aq, bq, x2), atol=1e-12)
    assert np.linalg.norm(x2 - prev) <= np.linalg.norm(cand - prev, axis=1).min() + 1e-12


def fd(f, x, h=1e-6):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        a, b = x.copy(), x.copy()
        a[it.multi_index] += h
        b[it.multi_index] -= h
        g[it.multi_index] = (f(a) - f(b)) / (2 * h)
    return g


def test_q_t_s_steps_are_their_argmins():
    g = S.random_small(6, 5, seed=4, sigma_R=0.1, sigma_t=0.1)
    info = S.random_info(g.m, g.tau, 10.0, seed=3)
    P, st = setup(g, info)
    beta, hh = 0.05 * abar(g), O.DEFAULT_H
    st = A.iterate(P, st, 2, beta, 1.4)
    T = lambda x: torch.as_tensor(x)
    # f with Sigma1 = diag(c, S) per edge, written out here
    S_ = P["S"].numpy(); c_ = np.trace(S_, axis1=1, axis2=2) / 3
    qm = P["qm"].numpy(); tm = P["tm"].numpy(); kap = P["kappa"].numpy()

    def qm_(a, b):
        return O.qmul(T(a), T(b)).numpy()

    def conj(a):
        return a * np.array([1, -1, -1, -1])

    def f_g(p, q, t, s):
        r = np.concatenate([np.zeros((g.m, 1)), t[g.ej] - s[g.ei]], 1) - \
            qm_(qm_(q[g.ei], np.concatenate([np.zeros((g.m, 1)), tm], 1)), conj(p[g.ei]))
        f = (c_ * r[:, 0] ** 2).sum() + np.einsum("ka,kab,kb->", r[:, 1:], S_, r[:, 1:])
        a = qm_(qm_(conj(p[g.ej]), q[g.ei]), qm) - np.array([1, 0, 0, 0])
        return f + (kap * (a * a).sum(1)).sum()

    X = {k: v.numpy() for k, v in st.items()}
    p1 = A.step_p(P, st, beta).numpy()
    q1 = A.step_q(P, st, T(p1), beta).numpy()
    psi_q = lambda q: (f_g(p1, q, X["t"], X["s"]) - (X["lam"] * (p1 - q)).sum()
                       + 0.5 * beta * ((p1 - q) ** 2).sum() + 0.5 * hh[1] * ((q - X["q"]) ** 2).sum())
    assert np.abs(fd(psi_q, q1.copy())).max() < 1e-5 * (1 + beta)
    t1 = A.step_t(P, st, T(p1), T(q1), beta).numpy()
    psi_t = lambda t: (f_g(p1, q1, t, X["s"]) - (X["z"] * (t - X["s"])).sum()
                       + 0.5 * beta * ((t - X["s"]) ** 2).sum() + 0.5 * hh[2] * ((t - X["t"]) ** 2).sum())
    assert np.abs(fd(psi_t, t1.copy())).max() < 1e-5 * (1 + beta)
    s1 = A.step_s(P, st, T(p1), T(q1), T(t1), beta).numpy()
    psi_s = lambda s: (f_g(p1, q1, t1, s) - (X["z"] * (t1 - s)).sum()
                       + 0.5 * beta * ((t1 - s) ** 2).sum() + 0.5 * hh[3] * ((s - X["s"]) ** 2).sum())
    assert np.abs(fd(psi_s, s1.copy())).max() < 1e-5 * (1 + beta)
    # the p-step against small rotations of p1 (on the sphere)
    psi_p = lambda p: (f_g(p, X["q"], X["t"], X["s"]) - (X["lam"] * (p - X["q"])).sum()
                       + 0.5 * beta * ((p - X["q"]) ** 2).sum() + 0.5 * hh[0] * ((p - X["p"]) ** 2).sum())
    base = psi_p(p1)
    rng = np.random.default_rng(2)
    for _ in range(200):
        d = rng.standard_normal(p1.shape) * 1e-3
        pp = p1 + d
        pp /= np.linalg.norm(pp, axis=1, keepdims=True)
        assert psi_p(pp) >= base - 1e-9 * abs(base)


def test_noise_free_fixed_point():
    g = S.grid(4, 3, 3, p=0.5, sigma_R=0.0, sigma_t=0.0, init="gt", seed=1)
    info = S.random_info(g.m, np.full(g.m, 100.0), 30.0, seed=2)
    P, st = setup(g, info)
    st1 = A.iterate(P, st, 3, 0.01 * abar(g), 1.4)
    for k in st:
        sc = 1.0 if k not in ("lam", "z") else 1.0
        assert float((st1[k] - st[k]).abs().max()) < 1e-10, k
    assert float(A.cost(P, st["p"], st["t"])) < 1e-18
