"""Pins of the oracle's reductions that the sweeps do not exercise:

  * the iteration residual e of App. E.1 and the dual residuals
    beta |dq|, beta |ds| (quaternion model, oracle/pradmm.residuals; chordal
    rendering, oracle/chordal.residuals): single-block perturbations of a
    state whose values App. E.1's definition fixes by hand (a change of t
    alone gives beta |dt|^2, of lambda alone |dlambda|^2 / beta, of s or p
    alone 0 ...), and the identity that eq. 3e / 3f force on e after a real
    sweep (dlambda = -gamma beta (p - q), dz = -gamma beta (t - s));
  * the augmented Lagrangian L_beta of the PRADMM section in both models:
    it is linear in the multipliers with slopes -(p - q), -(t - s), linear
    in beta with slope (|p - q|^2 + |t - s|^2) / 2, equals the cost where the
    duplicates agree; the chordal one also against its rotation term written
    through |Q R~ - P|^2 = |Q|^2 - 2 tr(R~^T Q^T P) + 3 (R~, P orthogonal)
    and Theorem 1's merit descent at large beta;
  * the information model's cost (Model section, eq. 1 with
    Sigma1 = diag(c_e, S_e)) against the rotation-matrix residual
    r = t_j - t_i - R(p_i) t~ weighted by S_e, with the rotation term
    2 - 2 Re(p_j^* p_i q~) of a unit quaternion, on noisy states; and its
    split f against the componentwise c_e r_0^2 + r_v^T S_e r_v.

Each expected value is written from the definition, not by calling the
function under test, so a swapped block (ds for dt), a dropped 1/beta, a
sign of a multiplier term or a wrong weighting fails one of these.
"""
import numpy as np
import pytest
import torch

import pgo_synth as S
from oracle import aniso as A
from oracle import chordal as C
from oracle import prep
from oracle import pradmm as O
from tests import qref

F64 = torch.float64
BETA = 7.0   # not 1, so that a dropped or misplaced beta shows


def _abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def _quat_state(seed=1):
    g = S.random_small(6, 5, seed=seed, sigma_R=0.1, sigma_t=0.1)
    P, p0, t0 = prep.prepare_graph(g)
    st = O.iterate(P, O.init_state(p0, t0), 4, 0.05 * _abar(g), 1.4)
    return g, P, st


def _chordal_state(seed=1):
    g = S.random_small(6, 5, seed=seed, sigma_R=0.1, sigma_t=0.1)
    Pb, P0, t0 = C.prepare_graph(g)
    st = C.iterate(Pb, C.init_state(P0, t0), 4, 0.05 * _abar(g), 1.4)
    return g, Pb, st


# perturbations on vertex 3 with hand-known squared norms
D4 = torch.tensor([0.1, 0.2, -0.2, 0.4], dtype=F64)      # |.|^2 = 0.25
D3 = torch.tensor([0.3, -0.4, 0.0], dtype=F64)           # |.|^2 = 0.25
D9 = torch.tensor([[0.0, 0.6, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, -0.8]], dtype=F64)  # |.|_F^2 = 1


def _perturbed(st, key, delta, v=3):
    out = {k: x.clone() for k, x in st.items()}
    out[key][v] = out[key][v] + delta
    return out


# (block, delta, |delta|^2, e, beta|dq|, beta|ds|) for the quaternion model;
# App. E.1: e = (|dlambda|^2 + |dz|^2) / beta + beta (|dq|^2 + |dt|^2)
QUAT_CASES = [
    ("t", D3, 0.25, BETA * 0.25, 0.0, 0.0),
    ("s", D3, 0.25, 0.0, 0.0, BETA * 0.5),
    ("q", D4, 0.25, BETA * 0.25, BETA * 0.5, 0.0),
    ("p", D4, 0.25, 0.0, 0.0, 0.0),
    ("lam", D4, 0.25, 0.25 / BETA, 0.0, 0.0),
    ("z", D3, 0.25, 0.25 / BETA, 0.0, 0.0),
]


@pytest.mark.parametrize("key,delta,sq,e,bdq,bds", QUAT_CASES)
def test_quat_residual_e_and_duals_single_block(key, delta, sq, e, bdq, bds):
    _, P, prev = _quat_state()
    st = _perturbed(prev, key, delta)
    r = O.residuals(P, prev, st, BETA)
    assert abs(r[2] - e) <= 1e-14 * max(1.0, e), (key, r[2], e)
    assert abs(r[3] - bdq) <= 1e-13, (key, r[3])
    assert abs(r[4] - bds) <= 1e-13, (key, r[4])
    assert float(torch.norm(delta) ** 2) == pytest.approx(sq, abs=1e-15)


def test_quat_primal_residuals_single_vertex():
    _, P, st = _quat_state()
    st = dict(st, q=st["p"].clone(), s=st["t"].clone())
    st["q"][2] += D4           # p - q = -D4 on vertex 2 only
    st["s"][4] += D3
    r = O.residuals(P, st, st, BETA)
    assert r[0] == pytest.approx(0.5, abs=1e-14)
    assert r[1] == pytest.approx(0.5, abs=1e-14)
    assert r[2] == 0.0 and r[3] == 0.0 and r[4] == 0.0


@pytest.mark.parametrize("gamma", [0.6, 1.4, 1.9])
def test_quat_residual_after_a_sweep_follows_the_multiplier_steps(gamma):
    """eq. 3e / 3f: dlambda = -gamma beta (p - q), dz = -gamma beta (t - s), so
    e = gamma^2 beta (|p - q|^2 + |t - s|^2) + beta (|dq|^2 + |dt|^2)."""
    _, P, prev = _quat_state(seed=4)
    st = O.sweep(P, prev, BETA, gamma)
    r = O.residuals(P, prev, st, BETA)
    dt2 = float(((st["t"] - prev["t"]) ** 2).sum())
    want = gamma ** 2 * BETA * (r[0] ** 2 + r[1] ** 2) + r[3] ** 2 / BETA + BETA * dt2
    assert abs(r[2] - want) <= 1e-12 * want
    assert r[5] == pytest.approx(float(O.cost(P, st["p"], st["t"])), rel=1e-15)


def test_quat_aug_lagrangian_structure():
    _, P, st = _quat_state(seed=5)
    p, q, t, s = st["p"], st["q"], st["t"], st["s"]
    L = lambda x, b=BETA: float(O.aug_lagrangian(P, x, b))
    base = L(st)
    rng = np.random.default_rng(0)
    dl = torch.as_tensor(rng.standard_normal(st["lam"].shape))
    dz = torch.as_tensor(rng.standard_normal(st["z"].shape))
    # linear in the multipliers with slopes -(p - q), -(t - s)
    assert L(dict(st, lam=st["lam"] + dl)) - base == pytest.approx(-float((dl * (p - q)).sum()),
                                                                    rel=1e-9, abs=1e-12)
    assert L(dict(st, z=st["z"] + dz)) - base == pytest.approx(-float((dz * (t - s)).sum()),
                                                               rel=1e-9, abs=1e-12)
    # linear in beta with slope (|p - q|^2 + |t - s|^2) / 2
    slope = 0.5 * float(((p - q) ** 2).sum() + ((t - s) ** 2).sum())
    assert L(st, BETA + 3.0) - base == pytest.approx(3.0 * slope, rel=1e-9, abs=1e-14)
    assert slope > 0
    # where the duplicates agree it is the cost of model (1), whatever the multipliers
    agree = dict(st, q=p.clone(), s=t.clone())
    assert L(agree) == pytest.approx(float(O.cost(P, p, t)), rel=1e-13)


# ---------------------------------------------------------------------------
# chordal rendering
CHORDAL_CASES = [
    ("t", D3, BETA * 0.25, 0.0, 0.0),
    ("s", D3, 0.0, 0.0, BETA * 0.5),
    ("Q", D9, BETA * 1.0, BETA * 1.0, 0.0),
    ("P", D9, 0.0, 0.0, 0.0),
    ("L", D9, 1.0 / BETA, 0.0, 0.0),
    ("z", D3, 0.25 / BETA, 0.0, 0.0),
]


@pytest.mark.parametrize("key,delta,e,bdq,bds", CHORDAL_CASES)
def test_chordal_residual_e_and_duals_single_block(key, delta, e, bdq, bds):
    _, Pb, prev = _chordal_state()
    st = _perturbed(prev, key, delta)
    r = C.residuals(Pb, prev, st, BETA)
    assert abs(r[2] - e) <= 1e-14 * max(1.0, e), (key, r[2], e)
    assert abs(r[3] - bdq) <= 1e-13, (key, r[3])
    assert abs(r[4] - bds) <= 1e-13, (key, r[4])


@pytest.mark.parametrize("gamma", [0.6, 1.4])
def test_chordal_residual_after_a_sweep_follows_the_multiplier_steps(gamma):
    _, Pb, prev = _chordal_state(seed=4)
    st = C.sweep(Pb, prev, BETA, gamma)
    r = C.residuals(Pb, prev, st, BETA)
    dt2 = float(((st["t"] - prev["t"]) ** 2).sum())
    want = gamma ** 2 * BETA * (r[0] ** 2 + r[1] ** 2) + r[3] ** 2 / BETA + BETA * dt2
    assert abs(r[2] - want) <= 1e-12 * want


def _chordal_L_ref(Pb, st, beta):
    """L_beta with the rotation term in trace form: for orthogonal R~ and P,
    |Q R~ - P|_F^2 = |Q|_F^2 - 2 tr(R~^T Q^T P) + 3; per-edge loop."""
    ei, ej = Pb["ei"].numpy(), Pb["ej"].numpy()
    tau, kappa, tm, Rm = (Pb[k].numpy() for k in ("tau", "kappa", "tm", "Rm"))
    P, Q, t, s, L, z = (st[k].numpy() for k in ("P", "Q", "t", "s", "L", "z"))
    f = g = 0.0
    for e in range(len(ei)):
        i, j = ei[e], ej[e]
        r = t[j] - s[i] - P[i] @ tm[e]
        f += tau[e] * float(r @ r)
        g += kappa[e] * (np.sum(Q[i] * Q[i]) - 2 * np.trace(Rm[e].T @ Q[i].T @ P[j]) + 3.0)
    return (f + g - np.sum(L * (P - Q)) + 0.5 * beta * np.sum((P - Q) ** 2)
            - np.sum(z * (t - s)) + 0.5 * beta * np.sum((t - s) ** 2))


def test_chordal_aug_lagrangian_against_trace_form():
    for seed in (1, 2, 3):
        _, Pb, st = _chordal_state(seed=seed)
        got = float(C.aug_lagrangian(Pb, st, BETA))
        assert got == pytest.approx(_chordal_L_ref(Pb, st, BETA), rel=1e-12)


def test_chordal_aug_lagrangian_structure():
    _, Pb, st = _chordal_state(seed=5)
    P, Q, t, s = st["P"], st["Q"], st["t"], st["s"]
    L = lambda x, b=BETA: float(C.aug_lagrangian(Pb, x, b))
    base = L(st)
    rng = np.random.default_rng(1)
    dL = torch.as_tensor(rng.standard_normal(st["L"].shape))
    dz = torch.as_tensor(rng.standard_normal(st["z"].shape))
    assert L(dict(st, L=st["L"] + dL)) - base == pytest.approx(-float((dL * (P - Q)).sum()),
                                                                rel=1e-9, abs=1e-12)
    assert L(dict(st, z=st["z"] + dz)) - base == pytest.approx(-float((dz * (t - s)).sum()),
                                                               rel=1e-9, abs=1e-12)
    slope = 0.5 * float(((P - Q) ** 2).sum() + ((t - s) ** 2).sum())
    assert L(st, BETA + 3.0) - base == pytest.approx(3.0 * slope, rel=1e-9, abs=1e-14)
    agree = dict(st, Q=P.clone(), s=t.clone())
    assert L(agree) == pytest.approx(float(C.cost(Pb, P, t)), rel=1e-13)


@pytest.mark.parametrize("gamma", [1.0, 1.4])
def test_chordal_merit_nonincreasing_for_large_beta(gamma):
    """Theorem 1 for the chordal splitting: L_beta + a1/(gamma beta) |dLambda|^2
    is eventually nonincreasing at a large penalty."""
    g = S.random_small(6, 5, seed=2, sigma_R=0.1, sigma_t=0.1)
    Pb, P0, t0 = C.prepare_graph(g)
    beta = 10 * _abar(g)
    a1 = abs(1 - gamma) / (1 - abs(1 - gamma))
    st = C.init_state(P0, t0)
    vals = []
    for _ in range(200):
        prev, st = st, C.sweep(Pb, st, beta, gamma)
        dl = float(((st["L"] - prev["L"]) ** 2).sum())
        vals.append(float(C.aug_lagrangian(Pb, st, beta)) + a1 / (gamma * beta) * dl)
    v = np.array(vals)
    assert np.all(np.diff(v[10:]) <= 1e-10 * np.abs(v[10:]).max())


# ---------------------------------------------------------------------------
# information model
def _rotmat(p):
    """R(p) of a unit quaternion, written out (App. A.2)."""
    w, x, y, z = p
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _info_problem(seed, aniso=10.0):
    g = S.random_small(7, 6, seed=seed, sigma_R=0.1, sigma_t=0.1)
    info = S.random_info(g.m, g.tau, aniso, seed=seed)
    P, p0, t0 = A.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, info, g.R0, g.t0)
    st = A.iterate(P, O.init_state(p0, t0), 3, 0.05 * _abar(g), 1.4)
    return g, info, P, st


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_info_cost_against_weighted_rotation_matrix_residual(seed):
    g, info, P, st = _info_problem(seed)
    p, t = st["p"].numpy(), st["t"].numpy()
    tm, kappa = g.tm, g.kappa
    qm = P["qm"].numpy()
    F = 0.0
    for e in range(g.m):
        i, j = g.ei[e], g.ej[e]
        r = t[j] - t[i] - _rotmat(p[i]) @ tm[e]
        a = qref.qmul(qref.qmul(qref.qconj(p[j]), p[i]), qm[e])
        F += float(r @ info[e] @ r) + kappa[e] * (2.0 - 2.0 * a[0])
    assert float(A.cost(P, st["p"], st["t"])) == pytest.approx(F, rel=1e-11)
    # the anisotropy matters: the isotropic weight c_e = tr(S_e)/3 gives another value
    iso = sum(np.trace(info[e]) / 3 * np.sum((t[g.ej[e]] - t[g.ei[e]] - _rotmat(p[g.ei[e]]) @ tm[e]) ** 2)
              for e in range(g.m))
    rot = sum(kappa[e] * (2 - 2 * qref.qmul(qref.qmul(qref.qconj(p[g.ej[e]]), p[g.ei[e]]), qm[e])[0])
              for e in range(g.m))
    assert abs(iso + rot - F) > 1e-6 * F


@pytest.mark.parametrize("seed", [0, 3])
def test_info_split_f_componentwise(seed):
    g, info, P, st = _info_problem(seed)
    p, q, t, s = (st[k].numpy() for k in ("p", "q", "t", "s"))
    f = 0.0
    for e in range(g.m):
        i, j = g.ei[e], g.ej[e]
        r = qref.hat(t[j] - s[i]) - qref.qmul(qref.qmul(q[i], qref.hat(g.tm[e])), qref.qconj(p[i]))
        c = np.trace(info[e]) / 3.0
        f += c * r[0] ** 2 + float(r[1:] @ info[e] @ r[1:])
    assert float(A.split_f(P, st["p"], st["q"], st["t"], st["s"])) == pytest.approx(f, rel=1e-11)
    assert np.abs(p - q).max() > 1e-6   # a split state, so the real part of r counts


def test_info_cost_isotropic_equals_scalar_cost():
    g = S.random_small(7, 6, seed=4, sigma_R=0.1, sigma_t=0.1)
    P, p0, t0 = A.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau[:, None, None] * np.eye(3),
                          g.R0, g.t0)
    Ps, _, _ = prep.prepare_graph(g)
    st = A.iterate(P, O.init_state(p0, t0), 3, 0.05 * _abar(g), 1.4)
    assert float(A.cost(P, st["p"], st["t"])) == pytest.approx(
        float(O.cost(Ps, st["p"], st["t"])), rel=1e-13)
