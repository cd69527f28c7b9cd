"""GPU tests of the outer loop: merit values against the oracle, the
per-graph stopping rule (App. E.1) and the penalty check (descent of the
merit of Theorem 1, as the experiments section describes)."""
import numpy as np
import pytest

import pgo_synth as S
from oracle import prep
from oracle import pradmm as O

pytestmark = pytest.mark.gpu

GAMMA = 1.4


def abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_merit_matches_oracle(pgo, prec, rtol):
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    P, p0, t0 = prep.prepare_graph(g)
    st, prev = O.iterate(P, O.init_state(p0, t0), 7, beta, GAMMA, return_prev=True)
    L = float(O.aug_lagrangian(P, st, beta))
    a1 = abs(1 - GAMMA) / (1 - abs(1 - GAMMA))
    psi = L + a1 / (GAMMA * beta) * float(((st["lam"] - prev["lam"]) ** 2).sum())
    with pgo.PoseGraph.from_graph(g, precision=prec) as h:
        h.iterate(7, beta, GAMMA)
        m = h.merit()[0]
    assert abs(m[0] - L) <= rtol * abs(L)
    assert abs(m[1] - psi) <= rtol * abs(psi)


def test_solve_without_rejections_equals_iterate(pgo):
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    with pgo.PoseGraph.from_graph(g) as h:
        b, done, conv = h.solve(200, 50, GAMMA, beta, tol=0.0, beta_growth=2.0)
        a = h.state()
    assert done[0] == 200 and not conv[0] and b[0] == beta
    with pgo.PoseGraph.from_graph(g) as h:
        h.iterate(200, beta, GAMMA)
        assert np.array_equal(h.state(), a)


def test_solve_stopping_rule(pgo):
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    tol = 1e-4
    with pgo.PoseGraph.from_graph(g) as h:
        _, done, conv = h.solve(20000, 10, GAMMA, beta, tol=tol, beta_growth=1.0)
        e = h.residuals()[0, 2]
    assert conv[0] and e < tol and done[0] < 20000
    # one chunk earlier the residual was still above tol
    with pgo.PoseGraph.from_graph(g) as h:
        h.iterate(int(done[0]) - 10, beta, GAMMA)
        assert h.residuals()[0, 2] >= tol


def test_penalty_check_rescues_a_diverging_graph(pgo):
    """Graph 106 of the batch diverges with beta = 0.01 abar (the FP64 oracle
    diverges too); with the merit check the penalty grows and the cost falls."""
    b = S.batched(4096, first=106, count=1)
    g = b.graphs[0]
    beta0 = 0.01 * abar(g)
    with pgo.PoseGraph.from_graph(g) as h:
        c0 = h.cost()[0]
        h.iterate(600, beta0, GAMMA)
        c_fixed = h.cost()[0]
    assert not c_fixed < c0
    with pgo.PoseGraph.from_graph(g) as h:
        bfin, done, _ = h.solve(600, 50, GAMMA, beta0, tol=0.0, beta_growth=2.0)
        c_adapt = h.cost()[0]
        psi = h.merit()[0, 1]
    assert bfin[0] > beta0 and done[0] == 600
    assert c_adapt < 1e-2 * c0 and np.isfinite(psi)


def test_batched_solve_matches_single_solves(pgo):
    b = S.batched(4096, first=100, count=8)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    voff, _ = b.offsets()
    for prec in ("fp64", "fp32"):
        with pgo.PoseGraph.from_batch(b, precision=prec) as h:
            bb, done, conv = h.solve(300, 50, GAMMA, betas, tol=1e-3, beta_growth=2.0)
            allst = h.state()
        for k, gr in enumerate(b.graphs):
            with pgo.PoseGraph.from_graph(gr, precision=prec) as h1:
                b1, d1, c1 = h1.solve(300, 50, GAMMA, betas[k], tol=1e-3, beta_growth=2.0)
                assert b1[0] == bb[k] and d1[0] == done[k] and c1[0] == conv[k]
                assert np.array_equal(h1.state(), allst[voff[k]:voff[k + 1]]), (prec, k)


def test_solve_with_rejections_same_in_both_schedules(pgo):
    """The merit-checked solve undoes a rejected chunk from a snapshot that
    the per-graph kernel takes as it starts each graph, where the per-phase
    schedule copies the state in a pass of its own: with rejections on the
    way (graph 106 diverges at 0.01 abar), both give the same penalties,
    sweep counts and state, bit for bit."""
    b = S.batched(4096, first=100, count=8)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    for prec in ("fp64", "fp32"):
        out = {}
        for sched in ("graph", "phase"):
            with pgo.PoseGraph.from_batch(b, precision=prec, schedule=sched) as h:
                bb, done, conv = h.solve(300, 50, GAMMA, betas, tol=0.0, beta_growth=2.0)
                out[sched] = (bb, done, h.state())
        assert np.any(out["graph"][0] > betas), prec  # some chunk was rejected
        assert np.array_equal(out["graph"][0], out["phase"][0]), prec
        assert np.array_equal(out["graph"][1], out["phase"][1]), prec
        assert np.array_equal(out["graph"][2], out["phase"][2]), prec


def test_solve_argument_checks(pgo):
    g = S.make_config("circle-100")
    with pgo.PoseGraph.from_graph(g) as h:
        for args in ((100, 30, GAMMA, 0.0, 2.0, 1.0), (100, 50, 2.0, 0.0, 2.0, 1.0),
                     (100, 50, GAMMA, 0.0, 0.5, 1.0), (100, 50, GAMMA, 0.0, 2.0, -1.0)):
            with pytest.raises(pgo.PgoError):
                pgo.pgo_solve(h.h, *args)


def test_reaches_the_oracle_minimum(pgo):
    """grid-1k from its odometry start: the sweeps reach the minimum of model
    (1) that the oracle's least squares found (tests/golden/fstar_grid1k.json,
    written by tests/golden/make_fstar.py) to 1e-6 relative, and no iterate's
    cost falls below it."""
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fstar_grid1k.json")
    F_star = json.load(open(path))["F_star"]
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    for prec, floor in (("fp64", 1e-9), ("fp32", 1e-6)):
        with pgo.PoseGraph.from_graph(g, precision=prec) as h:
            best = np.inf
            for _ in range(30):
                h.iterate(100, beta, GAMMA)
                F = h.cost()[0]
                assert F >= F_star * (1 - floor), (prec, F, F_star)
                best = min(best, F)
        assert best <= F_star * (1 + 1e-6), (prec, best, F_star)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_evaluate_equals_the_three_calls(pgo, prec):
    """pgo_evaluate (one reduction pass) returns exactly what pgo_cost,
    pgo_residuals and pgo_merit return."""
    b = S.batched(4096, first=10, count=4)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    with pgo.PoseGraph.from_batch(b, precision=prec) as h:
        h.iterate(7, betas, GAMMA)
        F, res, mer = h.evaluate()
        assert np.array_equal(F, h.cost())
        assert np.array_equal(res, h.residuals())
        assert np.array_equal(mer, h.merit())


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_stopping_inside_the_kernel_equals_the_host_loop(pgo, prec):
    """pgo_iterate_until in the per-graph schedule (the stopping rule e < tol
    evaluated inside the persistent kernel) stops every graph after the same
    number of sweeps as the host-checked loops (the per-phase schedule, and
    pgo_solve without penalty control), with the same bits."""
    b = S.batched(4096, first=200, count=12)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    with pgo.PoseGraph.from_batch(b, precision=prec, schedule="graph") as h:
        h.iterate(200, betas, GAMMA)
        e200 = h.residuals()[:, 2]
    tol = float(np.median(e200))   # about half of the graphs stop before 200 sweeps
    runs = {}
    for label, sched in (("kernel", "graph"), ("host", "phase")):
        with pgo.PoseGraph.from_batch(b, precision=prec, schedule=sched) as h:
            done = h.iterate_until(400, 20, betas, GAMMA, tol)
            runs[label] = (done, h.state(), h.residuals())
    with pgo.PoseGraph.from_batch(b, precision=prec, schedule="graph") as h:
        beta_out, done_solve, conv = h.solve(400, 20, GAMMA, betas.copy(), tol=tol, beta_growth=1.0)
        runs["solve"] = (done_solve, h.state(), None)
    assert np.array_equal(runs["kernel"][0], runs["host"][0]), (runs["kernel"][0], runs["host"][0])
    assert np.array_equal(runs["kernel"][0], runs["solve"][0])
    assert np.array_equal(runs["kernel"][1], runs["host"][1])
    assert np.array_equal(runs["kernel"][1], runs["solve"][1])
    done, _, res = runs["kernel"]
    stopped = done < 400
    assert stopped.any() and np.all(res[stopped, 2] < tol) and np.all(done % 20 == 0)
    assert np.all(conv[stopped] == 1)


@pytest.mark.parametrize("model", ["chordal", "info"])
def test_stopping_rule_of_the_other_models(pgo, model):
    """pgo_iterate_until for the chordal and information models (chunks
    checked on the host) stops each graph where pgo_solve without penalty
    control does, with the same bits."""
    b = S.batched(4096, first=300, count=6)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    kw = dict(precision="fp32", schedule="graph")
    info = None
    if model == "info":
        info = np.concatenate([S.random_info(gr.m, gr.tau, 10.0, seed=k) for k, gr in enumerate(b.graphs)])
    else:
        kw["model"] = model

    def make():
        return pgo.PoseGraph.from_batch(b, info=info, **kw)

    with make() as h:
        h.iterate(100, betas, GAMMA)
        tol = float(np.median(h.residuals()[:, 2]))
    with make() as h:
        done = h.iterate_until(300, 20, betas, GAMMA, tol)
        state = h.state()
    with make() as h:
        _, done_solve, _ = h.solve(300, 20, GAMMA, betas.copy(), tol=tol, beta_growth=1.0)
        assert np.array_equal(done, done_solve) and np.array_equal(state, h.state())
    assert (done < 300).any()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_keeps_state_penalties_and_residual_history(pgo, prec):
    """pgo_autotune times its candidates on the handle's state and puts it
    back: the state, the per-graph penalties, gamma and the residual history
    that pgo_evaluate (cost, residuals, merit) reads are those of before."""
    b = S.batched(4096, first=60, count=4)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs]) * np.array([1.0, 2.0, 3.0, 4.0])
    with pgo.PoseGraph.from_batch(b, precision=prec) as h:
        h.iterate(5, betas, 1.7)
        state = h.state()
        before = pgo.pgo_evaluate(h.h)
        pgo.pgo_autotune(h.h, float(np.median(betas)), 1.4, 3)
        assert np.array_equal(h.state(), state)
        after = pgo.pgo_evaluate(h.h)
        for x, y in zip(before, after):
            assert np.array_equal(x, y)
