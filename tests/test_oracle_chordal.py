"""Pins of the rotation-matrix (chordal) rendering of the sweep, oracle side:
fixed point, SO(3) after every sweep, rigid equivariance, each phase the
argmin of its subproblem (brute force over SO(3) for P, vanishing gradient
for Q, t, s, all from the split objective written out here), multiplier
identities, and agreement with a Levenberg-Marquardt local minimum of the
chordal cost on tiny graphs."""
import numpy as np
import pytest
import scipy.optimize
import torch

import pgo_synth as S
from oracle import chordal as C

F64 = torch.float64


def abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def npd(st):
    return {k: v.numpy().copy() for k, v in st.items()}


def f_g(P, Q, t, s, pb):
    ei, ej, tau, kappa, tm, Rm = (pb[k] for k in ("ei", "ej", "tau", "kappa", "tm", "Rm"))
    rf = t[ej] - s[ei] - np.einsum("kab,kb->ka", P[ei], tm)
    rg = Q[ei] @ Rm - P[ej]
    return float((tau * (rf ** 2).sum(1)).sum() + (kappa * (rg ** 2).sum((1, 2))).sum())


def fd(fun, x, h=1e-3):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        a, b = x.copy(), x.copy()
        a[i] += h
        b[i] -= h
        g[i] = (fun(a) - fun(b)) / (2 * h)
    return g


def small(seed=2):
    g = S.random_small(6, 5, seed=seed, sigma_R=0.1, sigma_t=0.1)
    Pb, P0, t0 = C.prepare_graph(g)
    beta = 0.05 * abar(g)
    st = C.iterate(Pb, C.init_state(P0, t0), 3, beta, 1.4)
    return g, Pb, st, beta


def test_noise_free_fixed_point():
    g = S.grid(4, 4, 3, p=0.5, sigma_R=0.0, sigma_t=0.0, init="gt")
    Pb, P0, t0 = C.prepare_graph(g)
    st = C.init_state(P0, t0)
    beta = 0.01 * abar(g)
    st1 = C.iterate(Pb, st, 3, beta, 1.4)
    for k in st:
        sc = beta if k in ("L", "z") else 1.0
        assert float((st1[k] - st[k]).abs().max()) / sc < 1e-12, k
    assert float(C.cost(Pb, P0, t0)) < 1e-20


def test_so3_after_every_sweep():
    g = S.make_config("grid-1k")
    Pb, P0, t0 = C.prepare_graph(g)
    st = C.init_state(P0, t0)
    for _ in range(5):
        st = C.sweep(Pb, st, 0.01 * abar(g), 1.4)
        P = st["P"]
        assert float((P.transpose(-1, -2) @ P - torch.eye(3, dtype=F64)).abs().max()) < 1e-14
        assert float((torch.linalg.det(P) - 1).abs().max()) < 1e-14


def test_rigid_equivariance():
    g, Pb, st, beta = small(3)
    rng = np.random.default_rng(1)
    Rg = torch.as_tensor(S.so3_exp(rng.standard_normal((1, 3)))[0])
    tg = torch.as_tensor(rng.standard_normal(3))
    tr = lambda s: dict(P=Rg @ s["P"], Q=Rg @ s["Q"], L=Rg @ s["L"], t=s["t"] @ Rg.T + tg,
                        s=s["s"] @ Rg.T + tg, z=s["z"] @ Rg.T)
    a = C.iterate(Pb, tr(st), 4, beta, 1.4)
    b = tr(C.iterate(Pb, st, 4, beta, 1.4))
    for k in a:
        assert float((a[k] - b[k]).abs().max()) < 1e-10 * (1 + float(b[k].abs().max())), k


def test_each_phase_is_its_argmin():
    g, Pb, st, beta = small(2)
    h = C.DEFAULT_H
    A = npd(st)
    pb = {k: (v.numpy() if torch.is_tensor(v) else v) for k, v in Pb.items()}
    ei, ej = pb["ei"], pb["ej"]
    P1 = C.step_P(Pb, st, beta).numpy()

    def phi_P(P):  # the P-subproblem objective of the split model, all of it
        return (f_g(P, A["Q"], A["t"], A["s"], pb) - (A["L"] * (P - A["Q"])).sum()
                + 0.5 * beta * ((P - A["Q"]) ** 2).sum() + 0.5 * h[0] * ((P - A["P"]) ** 2).sum())

    base = phi_P(P1)
    rng = np.random.default_rng(0)
    for i in range(g.n):
        for sc in (1e-4, 1e-2, 0.3, 3.0):
            R = S.so3_exp(sc * rng.standard_normal((300, 3)))
            for Rk in R:
                P = P1.copy()
                P[i] = P1[i] @ Rk
                assert phi_P(P) >= base - 1e-9 * abs(base)
    Q1 = C.step_Q(Pb, st, torch.as_tensor(P1), beta).numpy()
    psi_Q = lambda Q: (f_g(P1, Q, A["t"], A["s"], pb) - (A["L"] * (P1 - Q)).sum()
                       + 0.5 * beta * ((P1 - Q) ** 2).sum() + 0.5 * h[1] * ((Q - A["Q"]) ** 2).sum())
    assert np.abs(fd(psi_Q, Q1)).max() < 1e-6 * (1 + beta)
    t1 = C.step_t(Pb, st, torch.as_tensor(P1), beta).numpy()
    psi_t = lambda t: (f_g(P1, Q1, t, A["s"], pb) - (A["z"] * (t - A["s"])).sum()
                       + 0.5 * beta * ((t - A["s"]) ** 2).sum() + 0.5 * h[2] * ((t - A["t"]) ** 2).sum())
    assert np.abs(fd(psi_t, t1)).max() < 1e-6 * (1 + beta)
    s1 = C.step_s(Pb, st, torch.as_tensor(P1), torch.as_tensor(t1), beta).numpy()
    psi_s = lambda s: (f_g(P1, Q1, t1, s, pb) - (A["z"] * (t1 - s)).sum()
                       + 0.5 * beta * ((t1 - s) ** 2).sum() + 0.5 * h[3] * ((s - A["s"]) ** 2).sum())
    assert np.abs(fd(psi_s, s1)).max() < 1e-6 * (1 + beta)


@pytest.mark.parametrize("gamma", [1.0, 1.6])
def test_multiplier_identities(gamma):
    """Lambda' = (1-g) Lambda - g (grad_Q g(P', Q') + H2 dQ),
       z'      = (1-g) z      - g (grad_s f(P', t', s') + H4 ds)."""
    g, Pb, st, beta = small(1)
    h = C.DEFAULT_H
    new = C.sweep(Pb, st, beta, gamma)
    A, B = npd(st), npd(new)
    pb = {k: (v.numpy() if torch.is_tensor(v) else v) for k, v in Pb.items()}
    gQ = fd(lambda Q: f_g(B["P"], Q, A["t"], A["s"], pb), B["Q"])
    pred = (1 - gamma) * A["L"] - gamma * (gQ + h[1] * (B["Q"] - A["Q"]))
    assert np.abs(pred - B["L"]).max() < 1e-7 * (1 + np.abs(B["L"]).max())
    gs = fd(lambda s: f_g(B["P"], B["Q"], B["t"], s, pb), B["s"])
    pred = (1 - gamma) * A["z"] - gamma * (gs + h[3] * (B["s"] - A["s"]))
    assert np.abs(pred - B["z"]).max() < 1e-7 * (1 + np.abs(B["z"]).max())


def _lm_chordal(g, Pb, P0, t0):
    """Levenberg-Marquardt on the chordal cost with R_i = Exp(w_i) R_i^0."""
    n = g.n
    ei, ej = g.ei, g.ej
    tau, kappa = Pb["tau"].numpy(), Pb["kappa"].numpy()
    tm, Rm = Pb["tm"].numpy(), Pb["Rm"].numpy()
    R0, T0 = P0.numpy(), t0.numpy()

    def res(x):
        R = S.so3_exp(x[:3 * n].reshape(n, 3)) @ R0
        t = T0 + x[3 * n:].reshape(n, 3)
        rt = np.sqrt(tau)[:, None] * (t[ej] - t[ei] - np.einsum("kab,kb->ka", R[ei], tm))
        rr = np.sqrt(kappa)[:, None, None] * (R[ei] @ Rm - R[ej])
        return np.concatenate([rt.ravel(), rr.ravel()])
    sol = scipy.optimize.least_squares(res, np.zeros(6 * n), method="lm", xtol=1e-15, ftol=1e-15,
                                       gtol=1e-15, max_nfev=20000)
    r = res(sol.x)
    return float(r @ r)


@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_graphs_reach_the_local_minimum(seed):
    g = S.random_small(5, 4, seed=seed, sigma_R=0.1, sigma_t=0.1)
    Pb, P0, t0 = C.prepare_graph(g)
    c_lm = _lm_chordal(g, Pb, P0, t0)
    st = C.iterate(Pb, C.init_state(P0, t0), 3000, 0.03 * abar(g), 1.4)
    c = float(C.cost(Pb, st["P"], st["t"]))
    assert abs(c - c_lm) <= 1e-8 * c_lm
