"""Pins of the chordal-initialisation oracle: exact recovery from
noise-free measurements, the odometry composition on chains, first-order
optimality of both least-squares steps (finite differences of objectives
written out here), per-component anchors, and the chordal point beating the
odometry start on the 1000-pose grid."""
import numpy as np
import pytest
import torch

import pgo_synth as S
from oracle import chordal as C
from oracle import chordal_init as CI


def perturbed(g, scale=0.3, seed=0):
    """The same graph with every non-anchor given pose moved away."""
    rng = np.random.default_rng(seed)
    R0 = g.R0 @ S.so3_exp(scale * rng.standard_normal((g.n, 3)))
    t0 = g.t0 + scale * rng.standard_normal((g.n, 3))
    R0[0], t0[0] = g.R0[0], g.t0[0]
    return R0, t0


def test_noise_free_measurements_give_ground_truth():
    g = S.grid(4, 4, 3, p=0.5, sigma_R=0.0, sigma_t=0.0, init="gt", seed=1)
    R0, t0 = perturbed(g)
    R, t = CI.chordal_init(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau, R0, t0)
    assert np.abs(R - g.R_gt).max() < 1e-10
    assert np.abs(t - g.t_gt).max() < 1e-10


def test_chain_gives_the_odometry_composition():
    g = S.tree(12, seed=4, sigma_R=0.1, sigma_t=0.2)   # odometry init = composed measurements
    R0, t0 = perturbed(g, seed=2)
    R, t = CI.chordal_init(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau, R0, t0)
    assert np.abs(R - g.R0).max() < 1e-10
    assert np.abs(t - g.t0).max() < 1e-10


def fd_grad(f, x, h=1e-6):
    out = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        a, b = x.copy(), x.copy()
        a[it.multi_index] += h
        b[it.multi_index] -= h
        out[it.multi_index] = (f(a) - f(b)) / (2 * h)
    return out


def test_both_steps_are_least_squares_optima():
    g = S.random_small(7, 6, seed=5, sigma_R=0.2, sigma_t=0.3)
    R, t, Rrel = CI.chordal_init_graph(g, return_relaxed=True)
    Rm = C.project_so3(torch.as_tensor(g.Rm)).numpy()

    def f_rot(x):
        X = Rrel.copy()
        X[1:] = x
        r = X[g.ei] @ Rm - X[g.ej]
        return float((g.kappa * (r * r).sum((1, 2))).sum())

    gr = fd_grad(f_rot, Rrel[1:].copy())
    assert np.abs(gr).max() < 1e-6 * (1 + f_rot(Rrel[1:].copy()))

    def f_tr(x):
        T = t.copy()
        T[1:] = x
        r = T[g.ej] - T[g.ei] - np.einsum("kab,kb->ka", R[g.ei], g.tm)
        return float((g.tau * (r * r).sum(1)).sum())

    gt_ = fd_grad(f_tr, t[1:].copy())
    assert np.abs(gt_).max() < 1e-6 * (1 + f_tr(t[1:].copy()))
    # projected rotations are rotations
    assert np.abs(np.transpose(R, (0, 2, 1)) @ R - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(R) - 1).max() < 1e-12


def test_each_component_keeps_its_anchor():
    a = S.tree(5, seed=1)
    b = S.tree(4, seed=2)
    n = a.n + b.n
    ei = np.concatenate([a.ei, b.ei + a.n])
    ej = np.concatenate([a.ej, b.ej + a.n])
    Rm = np.concatenate([a.Rm, b.Rm]); tm = np.concatenate([a.tm, b.tm])
    kap = np.concatenate([a.kappa, b.kappa]); tau = np.concatenate([a.tau, b.tau])
    R0 = np.concatenate([a.R0, b.R0]); t0 = np.concatenate([a.t0, b.t0])
    rng = np.random.default_rng(0)
    R0p = R0 @ S.so3_exp(0.2 * rng.standard_normal((n, 3)))
    t0p = t0 + 0.2 * rng.standard_normal((n, 3))
    lab, anchor = CI.components(n, ei, ej)
    assert list(np.nonzero(anchor)[0]) == [0, a.n]
    R, t = CI.chordal_init(n, ei, ej, Rm, tm, kap, tau, R0p, t0p)
    for v in (0, a.n):
        assert np.abs(R[v] - C.project_so3(torch.as_tensor(R0p[v])).numpy()).max() < 1e-14
        assert np.abs(t[v] - t0p[v]).max() == 0
    # each chain is its anchor's composition of measurements
    Ra, ta = S.odometry_init(R[a.n], t[a.n], b.Rm, b.tm)
    assert np.abs(R[a.n:] - Ra).max() < 1e-10 and np.abs(t[a.n:] - ta).max() < 1e-10


def test_chordal_point_beats_odometry_on_grid_1k():
    g = S.make_config("grid-1k")
    Pb, P0, t0 = C.prepare_graph(g)
    R, t = CI.chordal_init_graph(g)
    F_odo = float(C.cost(Pb, P0, t0))
    F_ch = float(C.cost(Pb, torch.as_tensor(R), torch.as_tensor(t)))
    assert F_ch < 0.1 * F_odo
