"""GPU parity of the rotation-matrix (chordal) rendering of the sweep: the
HIP library with PGO_MODEL_CHORDAL, through its C ABI, against the FP64 CPU
oracle of oracle/chordal.py on the same seeded inputs.

Tolerances are those of the quaternion tests (tests/tolerance.py): the
state after 10 sweeps, max-abs per block (P, Q, t, s, Lambda/beta, z/beta),
unscaled; FP64 1e-10, FP32 max(1e-4, 4 x the departure of this model's
oracle run in float32 from its float64 run on the same input)."""
import numpy as np
import pytest
import torch

import pgo_synth as S
from oracle import chordal as C
from tests import tolerance as T

pytestmark = pytest.mark.gpu

GAMMA = 1.4
KEYS = ("P", "Q", "t", "s", "L", "z")
SL = dict(P=slice(0, 9), Q=slice(9, 18), t=slice(18, 21), s=slice(21, 24), L=slice(24, 33),
          z=slice(33, 36))


def abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def pack(st):
    n = st["t"].shape[0]
    return np.concatenate([st[k].reshape(n, -1).numpy() for k in KEYS], 1)


def unpack(a):
    n = a.shape[0]
    return {k: torch.as_tensor(a[:, SL[k]].reshape((n, 3, 3) if k in ("P", "Q", "L") else (n, 3)).copy())
            for k in KEYS}


def oracle_run(g, k, beta, gamma=GAMMA, st=None):
    Pb, P0, t0 = C.prepare_graph(g)
    st0 = C.init_state(P0, t0) if st is None else st
    st, prev = C.iterate(Pb, st0, k, beta, gamma, return_prev=True)
    return Pb, st, prev


def floor(g, k, beta, ref, prec, gamma=GAMMA):
    """What the arithmetic costs on this input (tests/tolerance.py)."""
    Pb, P0, t0 = C.prepare_graph(g)
    return T.chordal_floor(Pb, C.init_state(P0, t0), beta, gamma, k, ref=ref,
                           dtype=torch.float64 if prec == "fp64" else torch.float32)


def check(label, prec, got, ref, beta, floor=None):
    T.assert_within("chordal " + label, prec, T.block_errors(got, ref, beta, T.CHORDAL_BLOCKS),
                    floor)


def chordal(pgo, g, **opt):
    return pgo.PoseGraph.from_graph(g, model="chordal", **opt)


def gpu_run(pgo, g, k, beta, gamma=GAMMA, **opt):
    with chordal(pgo, g, **opt) as h:
        h.iterate(k, beta, gamma)
        return h.state(), h.cost()[0], h.residuals()[0]


def test_prepared_rotations_match_oracle(pgo):
    g = S.make_config("grid-1k")
    Pb, P0, _ = C.prepare_graph(g)
    with chordal(pgo, g) as h:
        Re, Pv = h.prepared()
        assert h.info()["model"] == pgo.MODEL_CHORDAL and h.info()["width"] == 36
    assert np.abs(Pv - P0.numpy()).max() < 1e-14
    assert np.abs(Re - Pb["Rm"].numpy()).max() < 1e-14


@pytest.mark.parametrize("name", ["circle-100", "grid-1k", "sphere-2.5k"])
@pytest.mark.parametrize("sched", ["phase", "graph"])
def test_fp64_state_parity_10_sweeps(pgo, name, sched):
    g = S.make_config(name)
    beta = 0.01 * abar(g)
    _, st, _ = oracle_run(g, 10, beta)
    got, _, _ = gpu_run(pgo, g, 10, beta, precision="fp64", schedule=sched)
    ref = pack(st)
    check(f"{name}/{sched}", "fp64", got, ref, beta, floor(g, 10, beta, ref, "fp64"))


@pytest.mark.parametrize("name", ["circle-100", "grid-1k", "sphere-2.5k"])
def test_fp32_state_parity_10_sweeps(pgo, name):
    g = S.make_config(name)
    beta = 0.01 * abar(g)
    _, st, _ = oracle_run(g, 10, beta)
    ref = pack(st)
    f32 = floor(g, 10, beta, ref, "fp32")
    for sched in ("phase", "graph"):
        got, _, _ = gpu_run(pgo, g, 10, beta, precision="fp32", schedule=sched)
        check(f"{name}/{sched}", "fp32", got, ref, beta, f32)


def test_edge_cases_fp64(pgo):
    rng = np.random.default_rng(11)
    cases = []
    g = S.random_small(6, 4, seed=3, sigma_R=0.05, sigma_t=0.05)
    dup = np.array([0, 1], np.int64)
    g2 = S._measure(
        np.concatenate([g.R_gt, S.so3_exp(rng.standard_normal((1, 3)))]),
        np.concatenate([g.t_gt, rng.standard_normal((1, 3))]),
        np.concatenate([g.ei, g.ei[dup], g.ej[dup]]), np.concatenate([g.ej, g.ej[dup], g.ei[dup]]),
        0.05, 0.05, rng, init="gt")
    g2.R0 = g2.R0 @ S.so3_exp(rng.standard_normal((g2.n, 3)) * 0.1)
    g2.t0 = g2.t0 + 0.1 * rng.standard_normal((g2.n, 3))
    cases.append(("dup-reverse-isolated", g2))
    g3 = S.tree(3, seed=1)
    g3.ei, g3.ej = g3.ei[:0], g3.ej[:0]
    g3.Rm, g3.tm, g3.kappa, g3.tau = g3.Rm[:0], g3.tm[:0], g3.kappa[:0], g3.tau[:0]
    cases.append(("no-edges", g3))
    cases.append(("single-edge", S.tree(2, seed=2)))
    cases.append(("ragged-grid", S.grid(7, 11, 9, p=0.4, sigma_R=0.05, sigma_t=0.1, seed=5)))
    for label, g in cases:
        beta = 0.05 * abar(g) if g.m else 1.0
        _, st, _ = oracle_run(g, 10, beta)
        for sched in ("phase", "graph"):
            for block in (64, 256):
                got, _, _ = gpu_run(pgo, g, 10, beta, precision="fp64", schedule=sched, block=block)
                check(f"{label}/{sched}/{block}", "fp64", got, pack(st), beta)


def test_schedules_and_block_sizes_bitwise_identical(pgo):
    g = S.make_config("sphere-2.5k")
    beta = 0.01 * abar(g)
    for prec in ("fp64", "fp32"):
        ref = None
        for sched in ("phase", "graph"):
            for block in (64, 256, 1024):
                got, _, _ = gpu_run(pgo, g, 6, beta, precision=prec, schedule=sched, block=block)
                if ref is None:
                    ref = got
                assert np.array_equal(got, ref), (prec, sched, block)


def test_batched_equals_single_and_oracle(pgo):
    b = S.batched(4096, first=40, count=7)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    voff, _ = b.offsets()
    for prec in ("fp64", "fp32"):
        with pgo.PoseGraph.from_batch(b, precision=prec, model="chordal") as h:
            h.iterate(8, betas, GAMMA)
            allst = h.state()
            costs = h.cost()
        for k, gr in enumerate(b.graphs):
            got, F, _ = gpu_run(pgo, gr, 8, betas[k], precision=prec)
            assert np.array_equal(allst[voff[k]:voff[k + 1]], got), (prec, k)
            assert costs[k] == F
            if prec == "fp64":
                _, st, _ = oracle_run(gr, 8, betas[k])
                ref = pack(st)
                check(gr.name, "fp64", got, ref, betas[k], floor(gr, 8, betas[k], ref, "fp64"))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cost_residuals_and_merit_match_oracle(pgo, prec):
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    Pb, st, prev = oracle_run(g, 7, beta)
    ref = np.array(C.residuals(Pb, prev, st, beta))
    a1 = abs(1 - GAMMA) / (1 - abs(1 - GAMMA))
    L_ref = float(C.aug_lagrangian(Pb, st, beta))
    psi_ref = L_ref + a1 / (GAMMA * beta) * float(((st["L"] - prev["L"]) ** 2).sum())
    with chordal(pgo, g, precision=prec) as h:
        h.iterate(7, beta, GAMMA)
        F, res, mer = h.cost()[0], h.residuals()[0], h.merit()[0]
    rtol = 1e-12 if prec == "fp64" else 1e-4
    assert abs(F - ref[5]) <= rtol * ref[5]
    assert np.allclose(res, ref, rtol=rtol if prec == "fp64" else 2e-3, atol=1e-12)
    assert abs(mer[0] - L_ref) <= (1e-10 if prec == "fp64" else 1e-4) * abs(L_ref)
    assert abs(mer[1] - psi_ref) <= (1e-10 if prec == "fp64" else 1e-4) * abs(psi_ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_final_cost_500_sweeps(pgo, prec):
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    Pb, st, _ = oracle_run(g, 500, beta)
    F_ref = float(C.cost(Pb, st["P"], st["t"]))
    _, F, _ = gpu_run(pgo, g, 500, beta, precision=prec)
    assert abs(F - F_ref) <= 1e-6 * F_ref


def test_so3_after_every_sweep(pgo):
    g = S.make_config("sphere-2.5k")
    beta = 0.01 * abar(g)
    for prec, tol in (("fp64", 1e-14), ("fp32", 2e-6)):
        with chordal(pgo, g, precision=prec) as h:
            for _ in range(5):
                h.iterate(1, beta, GAMMA)
                R, _ = h.poses()
                assert np.abs(np.transpose(R, (0, 2, 1)) @ R - np.eye(3)).max() < tol, prec
                assert np.abs(np.linalg.det(R) - 1).max() < 2 * tol, prec
                assert np.array_equal(R.reshape(g.n, 9), h.state()[:, 0:9])


def test_noise_free_fixed_point(pgo):
    g = S.grid(5, 5, 4, p=0.5, sigma_R=0.0, sigma_t=0.0, init="gt")
    beta = 0.01 * abar(g)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        with chordal(pgo, g, precision=prec) as h:
            s0 = h.state()
            h.iterate(5, beta, GAMMA)
            err = T.block_errors(h.state(), s0, beta, T.CHORDAL_BLOCKS)
            assert max(err.values()) <= tol, (prec, err)


def test_fp32_polar_island(pgo):
    """Multipliers chosen so that every M_i of the next P update is
    c_i U_i diag(1, 1e-3, -1e-4) V_i^T: a reflection whose SO(3) factor has
    a small denominator sigma_2 - sigma_3 = 9e-4 c_i.  Summed and factored in
    float the factor would be off by ~1e-4; the double island keeps the FP32
    P within 1e-6 of the oracle run on the same float32 inputs (the state,
    beta, and the edge records tau t~ and kappa R~ as the FP32 path stores
    them)."""
    g = S.make_config("grid-1k")
    beta = float(np.float32(0.01 * abar(g)))
    Pb, st, _ = oracle_run(g, 3, beta)
    with chordal(pgo, g, precision="fp32") as h:
        R9, _ = h.prepared()
    kap, tau = Pb["kappa"].numpy(), Pb["tau"].numpy()
    Rm32 = (kap[:, None, None] * R9).astype(np.float32).astype(np.float64) / kap[:, None, None]
    tm32 = (tau[:, None] * Pb["tm"].numpy()).astype(np.float32).astype(np.float64) / tau[:, None]
    Pb = dict(Pb, Rm=torch.as_tensor(Rm32), tm=torch.as_tensor(tm32))
    h1 = C.DEFAULT_H[0]
    # M_i of the P update at st (the oracle's P-update sum, retyped to build the input)
    ei, ej = torch.as_tensor(g.ei), torch.as_tensor(g.ej)
    r = st["t"][ej] - st["s"][ei]
    M = torch.zeros(g.n, 3, 3, dtype=torch.float64)
    M.index_add_(0, ei, 2 * Pb["tau"][:, None, None] * (r.unsqueeze(-1) @ Pb["tm"].unsqueeze(-2)))
    M.index_add_(0, ej, 2 * Pb["kappa"][:, None, None] * (st["Q"][ei] @ Pb["Rm"]))
    M += beta * st["Q"] + st["L"] + h1 * st["P"]
    rng = np.random.default_rng(7)
    U = torch.as_tensor(S.so3_exp(rng.standard_normal((g.n, 3))))
    V = torch.as_tensor(S.so3_exp(rng.standard_normal((g.n, 3))))
    c = torch.linalg.matrix_norm(M)[:, None, None]
    E = c * (U @ torch.diag(torch.tensor([1.0, 1e-3, -1e-4], dtype=torch.float64)) @ V.transpose(1, 2))
    st2 = dict(st, L=st["L"] - M + E)
    x32 = pack(st2).astype(np.float32).astype(np.float64)   # the state the FP32 path holds
    ref = pack(C.iterate(Pb, unpack(x32), 1, beta, GAMMA))
    with chordal(pgo, g, precision="fp32") as h:
        h.set_state(x32)
        assert np.array_equal(h.state(), x32)
        h.iterate(1, beta, GAMMA)
        got = h.state()
    assert np.abs(got[:, 0:9] - ref[:, 0:9]).max() < 1e-6
    check("grid-1k/polar island", "fp32", got, ref, beta)


def test_full_size_grid_100k_parity(pgo):
    """The 100k-pose grid in the per-phase schedule, FP64 and FP32 (the
    multipliers carry the accumulated rounding of every sweep's P - Q and
    t - s; the float32 oracle's own departure sets their bound)."""
    g = S.make_config("grid-100k")
    beta = 0.01 * abar(g)
    _, st, _ = oracle_run(g, 10, beta)
    ref = pack(st)
    for prec in ("fp64", "fp32"):
        got, _, _ = gpu_run(pgo, g, 10, beta, precision=prec, schedule="phase")
        check("grid-100k/phase", prec, got, ref, beta, floor(g, 10, beta, ref, prec))


def test_solve_and_quaternion_only_calls(pgo):
    b = S.batched(4096, first=60, count=5)
    betas = np.array([0.01 * abar(gr) for gr in b.graphs])
    voff, _ = b.offsets()
    with pgo.PoseGraph.from_batch(b, precision="fp64", model="chordal") as h:
        F0 = h.cost()
        beta, done, _ = h.solve(200, 50, GAMMA, betas, tol=0.0, beta_growth=2.0)
        allst = h.state()
        assert np.all(done == 200) and np.all(h.cost() < F0)
        dstate = torch.zeros((h.info()["n"], 21), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        for call in (lambda: pgo.pgo_forward_record(h.h, 5, 1.0, GAMMA, 2),
                     lambda: pgo.pgo_adjoint(h.h, dstate.data_ptr()),
                     lambda: pgo.pgo_set_edge_params(h.h, 0, 0, 0, 0)):
            with pytest.raises(pgo.PgoError) as ex:
                call()
            assert ex.value.name == "PGO_ESTATE"
    for k, gr in enumerate(b.graphs):  # the batched solve equals each graph's own solve
        with chordal(pgo, gr, precision="fp64") as h:
            bk, dk, _ = h.solve(200, 50, GAMMA, np.array([betas[k]]), tol=0.0, beta_growth=2.0)
            assert bk[0] == beta[k] and dk[0] == done[k]
            assert np.array_equal(h.state(), allst[voff[k]:voff[k + 1]])


def test_fp32_large_lever_arms(pgo):
    """A 4336-pose circle of the batch (b3891: radius ~700 m, loop closures
    spanning up to ~1.4 km) from the chordal start at the batch penalty:
    M_i of the P update then has entries of ~1e9, whose squared column norms
    overflow FP32 unless the polar factor scales its input.  The FP32 path
    after 5 sweeps against the FP64 oracle, within the FP32 bounds."""
    from oracle import chordal_init as CI
    g = S.batched(4096, first=3891, count=1).graphs[0]
    beta = 0.01 * abar(g)
    Rc, tc = CI.chordal_init_graph(g)
    g.R0, g.t0 = np.asarray(Rc), np.asarray(tc)
    Pb, P0, t0 = C.prepare_graph(g)
    st0 = C.init_state(P0, t0)
    ref = T.pack_chordal(C.iterate(Pb, st0, 5, beta, GAMMA))
    assert np.abs(ref[:, 18:21]).max() > 500.0
    got, _, _ = gpu_run(pgo, g, 5, beta, precision="fp32", schedule="phase")
    f32 = T.chordal_floor(Pb, st0, beta, GAMMA, 5, ref=ref)
    check("b3891-circle-4336 (large lever arms)", "fp32", got, ref, beta, f32)
