"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU
oracle on the same seeded inputs.

Tolerances (tests/tolerance.py): the state after 10 sweeps, max-abs per
block (p, q, t, s, lambda/beta, z/beta), unscaled; FP64 path 1e-10, FP32 path
max(1e-4, 4 x the departure of the oracle itself run in float32 from its
float64 run on the same input); final cost 1e-6 relative.  Multipliers are
compared as lambda/beta and z/beta: they scale with beta.  Every comparison's
raw errors are printed at the end of the session.
"""
import numpy as np
import pytest
import torch

import pgo_synth as S
from oracle import prep
from oracle import pradmm as O
from tests import tolerance as T

pytestmark = pytest.mark.gpu

GAMMA = 1.4


def abar(g):
    n = g.n
    d = np.zeros(n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def oracle_run(g, k, beta, gamma=GAMMA):
    P, p0, t0 = prep.prepare_graph(g)
    st, prev = O.iterate(P, O.init_state(p0, t0), k, beta, gamma, return_prev=True)
    return P, st, prev


def pack(st):
    return np.concatenate([st[k].numpy() for k in ("p", "q", "t", "s", "lam", "z")], 1)


def floor(g, k, beta, ref, prec, gamma=GAMMA):
    """What the arithmetic costs on this input (tests/tolerance.py): the
    oracle's departure in float32 (fp32), or under a shuffled edge order
    (fp64), from its float64 run ref."""
    P, p0, t0 = prep.prepare_graph(g)
    return T.quat_floor(P, O.init_state(p0, t0), beta, gamma, k, ref=ref,
                        dtype=torch.float64 if prec == "fp64" else torch.float32)


def check(label, prec, got, ref, beta, floor=None):
    T.assert_within(label, prec, T.block_errors(got, ref, beta), floor)


def gpu_run(pgo, g, k, beta, gamma=GAMMA, **opt):
    with pgo.PoseGraph.from_graph(g, **opt) as h:
        h.iterate(k, beta, gamma)
        return h.state(), h.cost()[0], h.residuals()[0]


def edge_case_graphs():
    rng = np.random.default_rng(11)
    out = []
    # duplicate and reverse edges, plus an isolated vertex (index 6)
    g = S.random_small(6, 4, seed=3, sigma_R=0.05, sigma_t=0.05)
    dup = np.array([0, 1], np.int64)
    g2 = S._measure(
        np.concatenate([g.R_gt, S.so3_exp(rng.standard_normal((1, 3)))]),
        np.concatenate([g.t_gt, rng.standard_normal((1, 3))]),
        np.concatenate([g.ei, g.ei[dup], g.ej[dup]]), np.concatenate([g.ej, g.ej[dup], g.ei[dup]]),
        0.05, 0.05, rng, init="gt")
    g2.R0 = g2.R0 @ S.so3_exp(rng.standard_normal((g2.n, 3)) * 0.1)
    g2.t0 = g2.t0 + 0.1 * rng.standard_normal((g2.n, 3))
    out.append(("dup-reverse-isolated", g2))
    # no edges at all
    g3 = S.tree(3, seed=1)
    g3.ei, g3.ej = g3.ei[:0], g3.ej[:0]
    g3.Rm, g3.tm, g3.kappa, g3.tau = g3.Rm[:0], g3.tm[:0], g3.kappa[:0], g3.tau[:0]
    out.append(("no-edges", g3))
    out.append(("single-edge", S.tree(2, seed=2)))
    # ragged: several tiles plus a tail for every block size tried
    out.append(("ragged-grid", S.grid(7, 11, 9, p=0.4, sigma_R=0.05, sigma_t=0.1, seed=5)))
    return out


# ---------------------------------------------------------------------------
def test_prepared_quaternions_match_oracle(pgo):
    g = S.make_config("grid-1k")
    P, p0, _ = prep.prepare_graph(g)
    with pgo.PoseGraph.from_graph(g) as h:
        qe, pv = h.prepared()
    assert np.abs(pv - p0.numpy()).max() < 1e-14
    assert np.abs(qe - P["qm"].numpy()).max() < 1e-14


@pytest.mark.parametrize("name", ["circle-100", "grid-1k", "sphere-2.5k"])
@pytest.mark.parametrize("sched", ["phase", "graph", "coop"])
def test_fp64_state_parity_10_sweeps(pgo, name, sched):
    g = S.make_config(name)
    beta = 0.01 * abar(g)
    _, st, _ = oracle_run(g, 10, beta)
    ref = pack(st)
    got, _, _ = gpu_run(pgo, g, 10, beta, precision="fp64", schedule=sched)
    check(f"{name}/{sched}", "fp64", got, ref, beta, floor(g, 10, beta, ref, "fp64"))


@pytest.mark.parametrize("label,g", edge_case_graphs(), ids=lambda x: x if isinstance(x, str) else "")
def test_fp64_edge_cases(pgo, label, g):
    beta = 0.05 * max(abar(g), 1.0)
    _, st, _ = oracle_run(g, 10, beta)
    for sched in ("phase", "graph", "coop"):
        for block in (64, 256):
            got, _, _ = gpu_run(pgo, g, 10, beta, precision="fp64", schedule=sched, block=block)
            check(f"{label}/{sched}/{block}", "fp64", got, pack(st), beta)


@pytest.mark.parametrize("name", ["circle-100", "grid-1k", "sphere-2.5k"])
def test_fp32_state_parity_10_sweeps(pgo, name):
    g = S.make_config(name)
    beta = 0.01 * abar(g)
    _, st, _ = oracle_run(g, 10, beta)
    ref = pack(st)
    f32 = floor(g, 10, beta, ref, "fp32")
    for sched in ("phase", "graph", "coop"):
        got, _, _ = gpu_run(pgo, g, 10, beta, precision="fp32", schedule=sched)
        check(f"{name}/{sched}", "fp32", got, ref, beta, f32)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cost_and_residuals_match_oracle(pgo, prec):
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    P, st, prev = oracle_run(g, 7, beta)
    ref = np.array(O.residuals(P, prev, st, beta))
    _, F, res = gpu_run(pgo, g, 7, beta, precision=prec)
    rtol = 1e-12 if prec == "fp64" else 1e-4
    assert abs(F - ref[5]) <= rtol * ref[5]
    assert np.allclose(res, ref, rtol=rtol if prec == "fp64" else 2e-3, atol=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_final_cost_500_sweeps(pgo, prec):
    """grid-1k, 500 sweeps: final cost within 1e-6 relative of the oracle's."""
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    P, st, _ = oracle_run(g, 500, beta)
    F_ref = float(O.cost(P, st["p"], st["t"]))
    _, F, _ = gpu_run(pgo, g, 500, beta, precision=prec)
    assert abs(F - F_ref) <= 1e-6 * F_ref


def test_schedules_and_block_sizes_bitwise_identical(pgo):
    g = S.make_config("sphere-2.5k")
    beta = 0.01 * abar(g)
    for prec in ("fp64", "fp32"):
        ref = None
        for sched in ("phase", "graph", "coop"):
            for block in (64, 256, 1024):
                got, _, _ = gpu_run(pgo, g, 6, beta, precision=prec, schedule=sched, block=block)
                if ref is None:
                    ref = got
                assert np.array_equal(got, ref), (prec, sched, block)


def test_batched_equals_single_bitwise(pgo):
    b = S.batched(4096, first=0, count=9)
    beta = 200.0
    for prec in ("fp64", "fp32"):
        with pgo.PoseGraph.from_batch(b, precision=prec) as h:
            h.iterate(8, beta, GAMMA)
            allst = h.state()
            costs = h.cost()
        voff, _ = b.offsets()
        for k, gr in enumerate(b.graphs):
            got, F, _ = gpu_run(pgo, gr, 8, beta, precision=prec)
            assert np.array_equal(allst[voff[k]:voff[k + 1]], got), (prec, k)
            assert costs[k] == F


def test_batched_parity_with_oracle(pgo):
    b = S.batched(4096, first=100, count=5)
    beta = 200.0
    with pgo.PoseGraph.from_batch(b, precision="fp64") as h:
        h.iterate(10, beta, GAMMA)
        allst = h.state()
    voff, _ = b.offsets()
    for k, gr in enumerate(b.graphs):
        _, st, _ = oracle_run(gr, 10, beta)
        ref = pack(st)
        check(gr.name, "fp64", allst[voff[k]:voff[k + 1]], ref, beta, floor(gr, 10, beta, ref, "fp64"))


@pytest.mark.parametrize("sched", ["phase", "graph", "coop"])
def test_per_graph_beta(pgo, sched):
    """pgo_iterate_graphs: graph g of a batch with its own beta equals the
    graph alone with that beta (bitwise) and the oracle (1e-10); the
    residual e uses each graph's beta."""
    b = S.batched(4096, first=20, count=6)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    voff, _ = b.offsets()
    with pgo.PoseGraph.from_batch(b, precision="fp64", schedule=sched) as h:
        h.iterate(6, betas, GAMMA)
        allst = h.state()
        res = h.residuals()
    for k, gr in enumerate(b.graphs):
        got, _, r1 = gpu_run(pgo, gr, 6, betas[k], precision="fp64", schedule=sched)
        assert np.array_equal(allst[voff[k]:voff[k + 1]], got)
        assert np.allclose(res[k], r1, rtol=1e-13, atol=0)
        P, st, prev = oracle_run(gr, 6, betas[k])
        ref = pack(st)
        check(f"{gr.name}/{sched}", "fp64", got, ref, betas[k], floor(gr, 6, betas[k], ref, "fp64"))
        assert np.allclose(res[k], O.residuals(P, prev, st, betas[k]), rtol=1e-9)
    with pgo.PoseGraph.from_batch(b) as h:
        with pytest.raises(pgo.PgoError):
            pgo.pgo_iterate_graphs(h.h, 1, np.r_[betas[:-1], 0.0], GAMMA)
        with pytest.raises(ValueError):
            pgo.pgo_iterate_graphs(h.h, 1, betas[:-1], GAMMA)


def test_resume_and_determinism(pgo):
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    for prec in ("fp64", "fp32"):
        with pgo.PoseGraph.from_graph(g, precision=prec) as h:
            h.iterate(10, beta, GAMMA)
            ref = h.state()
        with pgo.PoseGraph.from_graph(g, precision=prec) as h:
            h.iterate(4, beta, GAMMA)
            mid = h.state()
        with pgo.PoseGraph.from_graph(g, precision=prec) as h:
            h.set_state(mid)
            h.iterate(6, beta, GAMMA)
            assert np.array_equal(h.state(), ref), prec


def test_unit_norm_so3_after_every_sweep(pgo):
    g = S.make_config("sphere-2.5k")
    beta = 0.01 * abar(g)
    for prec, tol in (("fp64", 1e-15), ("fp32", 1e-6)):
        with pgo.PoseGraph.from_graph(g, precision=prec) as h:
            for _ in range(5):
                h.iterate(1, beta, GAMMA)
                p = h.state()[:, 0:4]
                assert np.abs(np.linalg.norm(p, axis=1) - 1).max() < 4 * tol
                R, _ = h.poses()
                assert np.abs(np.transpose(R, (0, 2, 1)) @ R - np.eye(3)).max() < 10 * tol
                assert np.abs(np.linalg.det(R) - 1).max() < 10 * tol


def test_noise_free_fixed_point(pgo):
    g = S.grid(5, 5, 4, p=0.5, sigma_R=0.0, sigma_t=0.0, init="gt")
    beta = 0.01 * abar(g)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        with pgo.PoseGraph.from_graph(g, precision=prec) as h:
            s0 = h.state()
            h.iterate(5, beta, GAMMA)
            err = T.block_errors(h.state(), s0, beta)
            assert max(err.values()) <= tol, (prec, err)
            assert h.cost()[0] < (1e-16 if prec == "fp64" else 1e-6) * g.m * 1e4


def test_error_paths(pgo):
    g = S.make_config("circle-100")
    with pgo.PoseGraph.from_graph(g) as h:
        for k, b, gm in ((1, 1.0, 2.0), (1, 1.0, 0.0), (1, 0.0, 1.0), (-1, 1.0, 1.0), (1, np.nan, 1.0)):
            with pytest.raises(pgo.PgoError) as ex:
                h.iterate(k, b, gm)
            assert ex.value.name == "PGO_EINVAL"
        s0 = h.state()
        h.iterate(0, 1.0, 1.0)
        assert np.array_equal(h.state(), s0)
        bad = s0.copy()
        bad[3, 9] = np.nan
        h.set_state(bad)
        with pytest.raises(pgo.PgoError) as ex:
            h.cost()
        assert ex.value.name == "PGO_ENUMERIC"
    Rm = g.Rm.copy()
    Rm[5] = -Rm[5]
    with pytest.raises(pgo.PgoError) as ex:
        pgo.pgo_create(g.n, g.R0.reshape(-1, 9), g.t0, g.ei, g.ej, Rm.reshape(-1, 9), g.tm, g.kappa,
                       g.tau)
    assert ex.value.name == "PGO_EINVAL" and "edge 5" in str(ex.value)


def test_full_size_grid_100k_parity(pgo):
    """The 100k-pose grid at full size in the per-phase schedule, FP32 and
    FP64, against the oracle after 10 sweeps; the cooperative schedule gives
    the same bits at every workgroup size."""
    g = S.make_config("grid-100k")
    beta = 0.01 * abar(g)
    _, st, _ = oracle_run(g, 10, beta)
    ref = pack(st)
    for prec in ("fp64", "fp32"):
        got, _, _ = gpu_run(pgo, g, 10, beta, precision=prec, schedule="phase")
        check("grid-100k/phase", prec, got, ref, beta, floor(g, 10, beta, ref, prec))
        for block in (128, 512, 1024):
            co, _, _ = gpu_run(pgo, g, 10, beta, precision=prec, schedule="coop", block=block)
            assert np.array_equal(co, got), (prec, block)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replays_equal_eager_launches(pgo, prec):
    """The per-phase schedule captures a k-sweep call into a HIP graph once
    and replays it: three replays from the same state, with eager library
    work (reductions, state transfers) and synchronisations in between, each
    equal bit for bit to k single-sweep (uncaptured) calls."""
    g = S.make_config("sphere-2.5k")
    beta = 0.01 * abar(g)
    with pgo.PoseGraph.from_graph(g, precision=prec, schedule="phase") as h:
        s0 = h.state()
        for _ in range(5):
            h.iterate(1, beta, GAMMA)
        eager = h.state()
        for _ in range(3):
            h.set_state(s0)
            h.iterate(5, beta, GAMMA)
            h.cost()
            assert np.array_equal(h.state(), eager)


def test_lds_residency_thresholds_bitwise(pgo):
    """Graphs on both sides of every LDS residency threshold of the per-graph
    kernel (160 KiB; FP32 quaternions take 16 bytes a pose, 3-vectors 12:
    all six state arrays up to 1950 poses, five to 2275, four to 2925, three
    to 3723, two to 5120, one above; FP64 arrays are twice as wide; the
    chordal model's arrays have their own widths) and of every register
    variant of the quaternion kernel (owner-only values of up to 3 vertices
    per thread with the slot between phases, up to 5 without it, at 1024
    threads: 3072 and 5120 poses in FP32; 1 and 2 vertices in FP64: 1024 and
    2048) give the same bits as the per-phase schedule, whose state stays in
    memory, for every model and both precisions."""
    sizes = [1024, 1025, 1950, 1951, 2048, 2049, 2275, 2276, 2925, 2926, 3072, 3073, 3723, 3724,
             5120, 5121]
    graphs = [S.circle(n, n_closures=n // 2, sigma_R=0.05, sigma_t=0.05, seed=k)
              for k, n in enumerate(sizes)]
    b = S.Batch(graphs)
    betas = np.array([0.05 * abar(gr) for gr in graphs])
    voff, _ = b.offsets()
    infos = np.concatenate([S.random_info(gr.m, gr.tau, 10.0, seed=k) for k, gr in enumerate(graphs)])
    for model in ("quat", "chordal", "info"):
        for prec in ("fp32", "fp64"):
            got = {}
            for sched, block in (("phase", 256), ("graph", 512 if model == "info" else 1024)):
                kw = dict(precision=prec, schedule=sched, block=block)
                if model == "info":
                    h = pgo.PoseGraph.from_batch(b, info=infos, **kw)
                else:
                    h = pgo.PoseGraph.from_batch(b, model=model, **kw)
                with h:
                    h.iterate(6, betas, GAMMA)
                    got[sched] = h.state()
                    if sched == "graph":
                        assert h.info()["lds"] == 1
            assert np.array_equal(got["phase"], got["graph"]), (model, prec)
            assert np.isfinite(got["graph"]).all()


@pytest.mark.parametrize("gamma", [1.0, 1.5, 1.9])
def test_relaxation_steps_of_the_sphere_workload(pgo, gamma):
    """The sphere workload at the relaxation steps its configuration sweeps
    (gamma in {1.0, 1.5, 1.9}): FP64 and FP32 against the oracle after 10
    sweeps."""
    g = S.make_config("sphere-2.5k")
    beta = 0.01 * abar(g)
    _, st, _ = oracle_run(g, 10, beta, gamma)
    ref = pack(st)
    for prec in ("fp64", "fp32"):
        got, _, _ = gpu_run(pgo, g, 10, beta, gamma, precision=prec)
        check(f"sphere-2.5k/gamma={gamma}", prec, got, ref, beta, floor(g, 10, beta, ref, prec, gamma))


def test_degenerate_graphs_in_a_batch(pgo):
    """A batch holding a single pose without edges, a two-pose graph with one
    edge and an ordinary graph: the per-graph kernel (state in LDS) and the
    per-phase schedule agree bit for bit, and each graph matches the oracle
    run alone."""
    single = S.tree(3, seed=4)
    single.n = 1
    single.R0, single.t0 = single.R0[:1], single.t0[:1]
    single.R_gt, single.t_gt = single.R_gt[:1], single.t_gt[:1]
    single.ei, single.ej = single.ei[:0], single.ej[:0]
    single.Rm, single.tm, single.kappa, single.tau = (single.Rm[:0], single.tm[:0],
                                                      single.kappa[:0], single.tau[:0])
    graphs = [single, S.tree(2, seed=5), S.make_config("circle-100")]
    b = S.Batch(graphs)
    betas = np.array([1.0, 0.05 * abar(graphs[1]), 0.01 * abar(graphs[2])])
    voff, _ = b.offsets()
    for prec in ("fp64", "fp32"):
        got = {}
        for sched, block in (("phase", 64), ("graph", 128), ("coop", 64)):
            with pgo.PoseGraph.from_batch(b, precision=prec, schedule=sched, block=block) as h:
                h.iterate(10, betas, GAMMA)
                got[sched] = h.state()
        assert np.array_equal(got["phase"], got["graph"]), prec
        assert np.array_equal(got["phase"], got["coop"]), prec
        for k, gr in enumerate(graphs):
            _, st, _ = oracle_run(gr, 10, betas[k])
            ref = pack(st)
            check(f"degenerate batch/graph {k}", prec, got["graph"][voff[k]:voff[k + 1]], ref,
                  betas[k], floor(gr, 10, betas[k], ref, prec))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cooperative_schedule_in_the_solve_loop(pgo, prec):
    """The cooperative schedule under pgo_solve's per-graph penalties and run
    mask (graphs that stop or are undone skip their vertices while every
    workgroup still meets every barrier): the same penalties, sweep counts
    and bits as the per-phase schedule, on a batch of uneven graphs."""
    b = S.batched(4096, first=40, count=12)
    betas = np.array([0.002 * abar(gr) for gr in b.graphs])   # low: some chunks are undone
    out = {}
    for sched in ("phase", "coop"):
        with pgo.PoseGraph.from_batch(b, precision=prec, schedule=sched) as h:
            beta, done, conv = h.solve(200, 20, GAMMA, betas.copy(), tol=1e-3)
            out[sched] = (beta, done, conv, h.state())
    for a, c in zip(out["phase"], out["coop"]):
        assert np.array_equal(a, c)
    assert np.any(out["coop"][0] > betas) or np.any(out["coop"][1] < 200)


def test_cooperative_schedule_refuses_other_models(pgo):
    g = S.make_config("circle-100")
    with pytest.raises(pgo.PgoError) as ex:
        pgo.PoseGraph.from_graph(g, model="chordal", schedule="coop")
    assert ex.value.name == "PGO_EINVAL"
