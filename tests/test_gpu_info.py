"""GPU parity of the information model (pgo_create_info: a full 3x3
translation information matrix per edge, Lemma 1's sphere-constrained p
update) against the FP64 CPU oracle of oracle/aniso.py on the same seeded
inputs.  Tolerances as the isotropic tests (tests/tolerance.py): the state
after 10 sweeps, max-abs per block, multipliers over beta, unscaled; FP64
1e-10, FP32 max(1e-4, 4 x the departure of this model's oracle run in
float32 from its float64 run)."""
import numpy as np
import pytest
import torch

import pgo_synth as S
from oracle import aniso as A
from oracle import pradmm as O
from tests import tolerance as T

pytestmark = pytest.mark.gpu

GAMMA = 1.4


def abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def pack(st):
    return np.concatenate([st[k].numpy() for k in ("p", "q", "t", "s", "lam", "z")], 1)


def check(label, prec, got, ref, beta, floor=None):
    T.assert_within("info " + label, prec, T.block_errors(got, ref, beta), floor)


def oracle_run(g, info, k, beta):
    P, p0, t0 = A.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, info, g.R0, g.t0)
    st, prev = A.iterate(P, O.init_state(p0, t0), k, beta, GAMMA, return_prev=True)
    return P, st, prev


def gpu_run(pgo, g, info, k, beta, **opt):
    with pgo.PoseGraph.from_graph(g, info=info, **opt) as h:
        h.iterate(k, beta, GAMMA)
        return h.state(), h.cost()[0], h.residuals()[0]


CASES = [("circle-100", 30.0), ("grid-1k", 10.0)]


@pytest.mark.parametrize("name,aniso", CASES)
@pytest.mark.parametrize("sched", ["phase", "graph"])
def test_fp64_parity_10_sweeps(pgo, name, aniso, sched):
    g = S.make_config(name)
    info = S.random_info(g.m, g.tau, aniso, seed=1)
    beta = 0.01 * abar(g)
    P, st, _ = oracle_run(g, info, 10, beta)
    ref = pack(st)
    _, p0, t0 = A.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, info, g.R0, g.t0)
    f64 = T.info_floor(P, O.init_state(p0, t0), beta, GAMMA, 10, ref=ref, dtype=torch.float64)
    got, _, _ = gpu_run(pgo, g, info, 10, beta, precision="fp64", schedule=sched)
    check(f"{name}/{sched}", "fp64", got, ref, beta, f64)


@pytest.mark.parametrize("name,aniso", CASES)
def test_fp32_parity_10_sweeps(pgo, name, aniso):
    g = S.make_config(name)
    info = S.random_info(g.m, g.tau, aniso, seed=1)
    beta = 0.01 * abar(g)
    P, st, _ = oracle_run(g, info, 10, beta)
    ref = pack(st)
    _, p0, t0 = A.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, info, g.R0, g.t0)
    floor = T.info_floor(P, O.init_state(p0, t0), beta, GAMMA, 10, ref=ref)
    for sched in ("phase", "graph"):
        got, _, _ = gpu_run(pgo, g, info, 10, beta, precision="fp32", schedule=sched)
        check(f"{name}/{sched}", "fp32", got, ref, beta, floor)


def test_isotropic_information_equals_the_isotropic_model(pgo):
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    info = g.tau[:, None, None] * np.eye(3)
    a, Fa, ra = gpu_run(pgo, g, info, 10, beta, precision="fp64")
    b, Fb, rb = gpu_run(pgo, g, None, 10, beta, precision="fp64")
    check("isotropic S = tau I vs the isotropic model", "fp64", a, b, beta)
    assert abs(Fa - Fb) <= 1e-11 * Fb


def test_schedules_and_blocks_bitwise(pgo):
    g = S.make_config("sphere-2.5k")
    info = S.random_info(g.m, g.tau, 10.0, seed=2)
    beta = 0.01 * abar(g)
    for prec in ("fp64", "fp32"):
        ref = None
        for sched in ("phase", "graph"):
            for block in (64, 256):
                got, _, _ = gpu_run(pgo, g, info, 6, beta, precision=prec, schedule=sched, block=block)
                if ref is None:
                    ref = got
                assert np.array_equal(got, ref), (prec, sched, block)
        assert np.abs(np.linalg.norm(ref[:, 0:4], axis=1) - 1).max() < (1e-14 if prec == "fp64" else 1e-6)


def test_cost_residuals_merit_and_batch(pgo):
    g = S.make_config("grid-1k")
    info = S.random_info(g.m, g.tau, 10.0, seed=3)
    beta = 0.01 * abar(g)
    P, st, prev = oracle_run(g, info, 7, beta)
    a1 = abs(1 - GAMMA) / (1 - abs(1 - GAMMA))
    L_ref = float(A.aug_lagrangian(P, st, beta))
    psi_ref = L_ref + a1 / (GAMMA * beta) * float(((st["lam"] - prev["lam"]) ** 2).sum())
    F_ref = float(A.cost(P, st["p"], st["t"]))
    res_ref = O.residuals(P, prev, st, beta)
    with pgo.PoseGraph.from_graph(g, info=info, precision="fp64") as h:
        h.iterate(7, beta, GAMMA)
        F, res, mer = h.cost()[0], h.residuals()[0], h.merit()[0]
    assert abs(F - F_ref) <= 1e-11 * F_ref
    assert np.allclose(res[:5], res_ref[:5], rtol=1e-9, atol=1e-12)
    assert abs(mer[0] - L_ref) <= 1e-10 * abs(L_ref) and abs(mer[1] - psi_ref) <= 1e-10 * abs(psi_ref)
    # a batch equals its graphs one by one, bit for bit
    b = S.batched(4096, first=300, count=5)
    infos = [S.random_info(gr.m, gr.tau, 10.0, seed=k) for k, gr in enumerate(b.graphs)]
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    voff, _ = b.offsets()
    with pgo.PoseGraph.from_batch(b, info=np.concatenate(infos), precision="fp32") as h:
        h.iterate(6, betas, GAMMA)
        allst = h.state()
    for k, gr in enumerate(b.graphs):
        got, _, _ = gpu_run(pgo, gr, infos[k], 6, betas[k], precision="fp32")
        assert np.array_equal(allst[voff[k]:voff[k + 1]], got), k


def test_solve_and_unsupported_calls(pgo):
    g = S.make_config("circle-100")
    info = S.random_info(g.m, g.tau, 10.0, seed=4)
    with pgo.PoseGraph.from_graph(g, info=info) as h:
        F0 = h.cost()[0]
        _, done, _ = h.solve(200, 50, GAMMA, np.array([0.01 * abar(g)]))
        assert done[0] == 200 and h.cost()[0] < F0
        assert h.info()["model"] == pgo.MODEL_QUAT_INFO
        with pytest.raises(pgo.PgoError) as ex:
            pgo.pgo_forward_record(h.h, 3, 1.0, GAMMA, 1)
        assert ex.value.name == "PGO_ESTATE"


def scrambled_state(g, beta, seed):
    """A state far from every subproblem's solution: random unit p, q near
    p, positions and splits off the initial ones, multipliers of size beta."""
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((g.n, 4))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    q = p + 0.3 * rng.standard_normal((g.n, 4))
    t = g.t0 + rng.standard_normal((g.n, 3))
    s = t + 0.5 * rng.standard_normal((g.n, 3))
    lam = beta * rng.standard_normal((g.n, 4))
    z = beta * rng.standard_normal((g.n, 3))
    return np.concatenate([p, q, t, s, lam, z], 1)


@pytest.mark.parametrize("name,aniso", CASES)
@pytest.mark.parametrize("beta_scale", [0.01, 1.0])
def test_p_update_from_scrambled_states(pgo, name, aniso, beta_scale):
    """The sphere-constrained p update warm-starts its multiplier from p^k; a
    random p^k makes it leave that start (bracketing, bisection, and the
    eigen-decomposition fallback where the factorisation path gives up)."""
    g = S.make_config(name)
    info = S.random_info(g.m, g.tau, aniso, seed=5)
    beta = beta_scale * abar(g)
    st0 = scrambled_state(g, beta, seed=6)
    P, _, _ = A.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, info, g.R0, g.t0)
    cols = dict(p=(0, 4), q=(4, 8), t=(8, 11), s=(11, 14), lam=(14, 18), z=(18, 21))
    ost = {k: torch.tensor(st0[:, a:b]) for k, (a, b) in cols.items()}
    ref = A.iterate(P, ost, 3, beta, GAMMA)
    with pgo.PoseGraph.from_graph(g, info=info, precision="fp64") as h:
        h.set_state(st0)
        h.iterate(3, beta, GAMMA)
        got = h.state()
    check(f"{name}/scrambled/beta x{beta_scale}", "fp64", got, pack(ref), beta)
