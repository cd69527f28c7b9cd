"""GPU tests of the hand-written adjoint of K unrolled sweeps, through the
C ABI and the torch.autograd.Function: against the oracle's reference
adjoint (automatic differentiation of the FP64 CPU sweeps) and against FP64
central finite differences of the library's own FP64 forward pass
(h = 1e-6, parameters log kappa, log tau, omega, t~)."""
import numpy as np
import pytest
import torch

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


def cuda(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def gpu_grads(pgo, g, K, beta, C, prec, omega=None, schedule="auto"):
    from paper_2601_15684_amd.autograd import unrolled_pradmm
    kappa = cuda(g.kappa).requires_grad_()
    tau = cuda(g.tau).requires_grad_()
    tm = cuda(g.tm).requires_grad_()
    om = cuda(np.zeros((g.m, 3)) if omega is None else omega).requires_grad_()
    with pgo.PoseGraph.from_graph(g, precision=prec, schedule=schedule) as h:
        state = unrolled_pradmm(h, kappa, tau, tm, om, K, beta, GAMMA, C)
        loss = ((state[:, 8:11] - cuda(g.t_gt)) ** 2).sum()
        loss.backward()
    torch.cuda.synchronize()
    return float(loss), dict(kappa=kappa.grad.cpu().numpy(), tau=tau.grad.cpu().numpy(),
                             tm=tm.grad.cpu().numpy(), omega=om.grad.cpu().numpy())


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("sched", ["phase", "graph"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-3)])
@pytest.mark.parametrize("K,C", [(10, 3), (6, 6)])
def test_adjoint_matches_oracle(pgo, prec, tol, K, C, sched):
    g = S.grid(4, 3, 3, all_pairs=True, sigma_R=0.05, sigma_t=0.1, seed=0)
    beta = 0.05 * abar(g)
    P, p0, t0 = prep.prepare_graph(g)
    L_ref, ref = O.unrolled_grad(P, p0, t0, K, beta, GAMMA, torch.as_tensor(g.t_gt))
    L, got = gpu_grads(pgo, g, K, beta, C, prec, schedule=sched)
    assert abs(L - L_ref) <= (1e-10 if prec == "fp64" else 1e-4) * L_ref
    for k in ("kappa", "tau", "tm", "omega"):
        assert rel(got[k], ref[k].numpy()) <= tol, (k, rel(got[k], ref[k].numpy()))


@pytest.mark.parametrize("sched,C", [("phase", 10), ("phase", 50), ("graph", 10)])
def test_adjoint_fp32_matches_fp64_grid_1k(pgo, sched, C):
    """K = 50 sweeps of the 1000-pose grid: the FP32 adjoint against the FP64
    one in each schedule, with several checkpoint segments (C = 10) and one
    (C = 50).  A float32 run of the oracle's own automatic differentiation
    departs from its float64 run by ~5e-6 here."""
    g = S.make_config("grid-1k")
    beta = 0.01 * abar(g)
    _, g64 = gpu_grads(pgo, g, 50, beta, C, "fp64", schedule=sched)
    _, g32 = gpu_grads(pgo, g, 50, beta, C, "fp32", schedule=sched)
    errs = {k: rel(g32[k], g64[k]) for k in g64}
    assert max(errs.values()) <= 1e-4, errs


def test_autograd_on_a_side_stream_matches_default_stream(pgo):
    """The autograd wrapper orders its library calls with torch's current
    stream: run under a non-default stream it gives the same bits."""
    g = S.grid(4, 3, 3, all_pairs=True, sigma_R=0.05, sigma_t=0.1, seed=0)
    beta = 0.05 * abar(g)
    L0, g0 = gpu_grads(pgo, g, 10, beta, 3, "fp32", schedule="phase")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        L1, g1 = gpu_grads(pgo, g, 10, beta, 3, "fp32", schedule="phase")
    torch.cuda.synchronize()
    assert L0 == L1
    for k in g0:
        assert np.array_equal(g0[k], g1[k]), k


def test_adjoint_state_gradient_matches_oracle(pgo):
    g = S.random_small(6, 5, seed=4, sigma_R=0.05, sigma_t=0.1)
    beta, K = 0.05 * abar(g), 7
    P, p0, t0 = prep.prepare_graph(g)
    st = O.init_state(p0, t0)
    leaves = {k: v.clone().requires_grad_() for k, v in st.items()}
    s = dict(leaves)
    for _ in range(K):
        s = O.sweep(P, s, beta, GAMMA)
    w = torch.as_tensor(np.random.default_rng(0).standard_normal((g.n, 21)))
    packed = torch.cat([s[k] for k in ("p", "q", "t", "s", "lam", "z")], 1)
    (packed * w).sum().backward()
    ref = torch.cat([leaves[k].grad for k in ("p", "q", "t", "s", "lam", "z")], 1).numpy()
    with pgo.PoseGraph.from_graph(g) as h:
        pgo.pgo_forward_record(h.h, K, beta, GAMMA, 3)
        wd = cuda(w.numpy())
        torch.cuda.synchronize()  # the library runs on the handle's own stream
        d0 = torch.empty((g.n, 21), dtype=torch.float64, device="cuda")
        pgo.pgo_adjoint(h.h, wd.data_ptr(), 0, 0, 0, 0, d0.data_ptr())
        torch.cuda.synchronize()
        got = d0.cpu().numpy()
    assert rel(got, ref) <= 1e-9


def _fd_t(pgo, h, base, K, beta, C):
    torch.cuda.synchronize()  # parameters written by torch, read on the handle's own stream
    pgo.pgo_set_edge_params(h.h, base["kappa"].data_ptr(), base["tau"].data_ptr(),
                            base["tm"].data_ptr(), base["omega"].data_ptr())
    pgo.pgo_reset_state(h.h)
    pgo.pgo_forward_record(h.h, K, beta, GAMMA, C)
    return h.state()[:, 8:11]


def _central(tp, tm_, t_gt, hstep):
    """(L(+h) - L(-h)) / 2h for L = sum |t - t_gt|^2, formed from the state
    difference so the large loss does not cancel:
    L+ - L- = sum (t+ - t-) . (t+ + t- - 2 t_gt)."""
    return float(((tp - tm_) * (tp + tm_ - 2 * t_gt)).sum()) / (2 * hstep)


@pytest.mark.parametrize("omega_scale", [0.0, 0.02])
def test_adjoint_vs_central_differences_diff_20k(pgo, omega_scale):
    """The 20k-pose grid, K = 50 unrolled sweeps, checkpoint every 10: FP32
    and FP64 adjoints against FP64 central differences on 64 random edges."""
    g = S.make_config("diff-20k")
    K, C, hstep = 50, 10, 1e-6
    beta = 0.01 * abar(g)
    rng = np.random.default_rng(0)
    omega = omega_scale * rng.standard_normal((g.m, 3))
    _, g32 = gpu_grads(pgo, g, K, beta, C, "fp32", omega)
    _, g64 = gpu_grads(pgo, g, K, beta, C, "fp64", omega)
    edges = rng.choice(g.m, size=64, replace=False)
    fd = {k: [] for k in ("log_kappa", "log_tau", "omega", "tm")}
    with pgo.PoseGraph.from_graph(g, precision="fp64") as h:
        base = dict(kappa=cuda(g.kappa), tau=cuda(g.tau), tm=cuda(g.tm), omega=cuda(omega))

        def t_with(name, idx, delta, mul=False):
            b = {k: v.clone() for k, v in base.items()}
            if mul:
                b[name][idx] = b[name][idx] * float(np.exp(delta))
            else:
                b[name][idx] = b[name][idx] + delta
            return _fd_t(pgo, h, b, K, beta, C)

        def central(name, idx, mul=False, hh=hstep):
            return _central(t_with(name, idx, hh, mul), t_with(name, idx, -hh, mul), g.t_gt, hh)

        fd_wide = {k: [] for k in fd}   # the same at h = 1e-4
        for e in edges:
            e = int(e)
            for store, hh in ((fd, hstep), (fd_wide, 1e-4)):
                store["log_kappa"].append(central("kappa", e, True, hh))
                store["log_tau"].append(central("tau", e, True, hh))
                for c in range(3):
                    store["omega"].append(central("omega", (e, c), hh=hh))
                    store["tm"].append(central("tm", (e, c), hh=hh))
    # Tolerances: at h = 1e-6 the central difference of the FP64 forward
    # carries the forward's rounding divided by h, a few 1e-5 relative on
    # this 20k-pose problem; at h = 1e-4 that noise is 100x smaller and the
    # O(h^2) truncation still below it, so there the FP64 adjoint is held to
    # 1e-5 (the bound the method's adjoint check asks), at h = 1e-6 to 1e-4.
    # FP32 adds its own rounding: 1e-3.
    errs = {}
    for name, grads in (("fp64", g64), ("fp32", g32)):
        ad = {"log_kappa": grads["kappa"][edges] * g.kappa[edges],
              "log_tau": grads["tau"][edges] * g.tau[edges],
              "omega": grads["omega"][edges].ravel(), "tm": grads["tm"][edges].ravel()}
        for k in fd:
            errs[(name, k)] = rel(ad[k], fd[k])
            errs[(name + "@h=1e-4", k)] = rel(ad[k], fd_wide[k])
    for k in ("kappa", "tau", "tm", "omega"):
        errs[("fp32-vs-fp64", k)] = rel(g32[k], g64[k])
    print("adjoint vs central differences:", {f"{a}/{b}": f"{v:.2e}" for (a, b), v in errs.items()})
    bound = {"fp64": 1e-4, "fp64@h=1e-4": 1e-5}
    bad = {kk: v for kk, v in errs.items() if v > bound.get(kk[0], 1e-3)}
    assert not bad, bad


def test_adjoint_diff_20k_matches_oracle_adjoint(pgo):
    """The 20k-pose grid, K = 50 unrolled sweeps, checkpoint every 10: the
    FP64 and FP32 adjoints against the oracle's reference adjoint (automatic
    differentiation of the FP64 CPU sweeps) at full size."""
    g = S.make_config("diff-20k")
    K, C = 50, 10
    beta = 0.01 * abar(g)
    P, p0, t0 = prep.prepare_graph(g)
    L_ref, ref = O.unrolled_grad(P, p0, t0, K, beta, GAMMA, torch.as_tensor(g.t_gt))
    for prec, tol in (("fp64", 1e-8), ("fp32", 1e-3)):
        L, got = gpu_grads(pgo, g, K, beta, C, prec)
        assert abs(L - L_ref) <= (1e-10 if prec == "fp64" else 1e-4) * L_ref, (prec, L, L_ref)
        errs = {k: rel(got[k], ref[k].numpy()) for k in ("kappa", "tau", "tm", "omega")}
        print(f"diff-20k {prec} adjoint vs oracle adjoint:", {k: f"{v:.2e}" for k, v in errs.items()})
        assert all(v <= tol for v in errs.values()), (prec, errs)


def test_adjoint_requires_a_recorded_pass(pgo):
    g = S.make_config("circle-100")
    with pgo.PoseGraph.from_graph(g) as h:
        d = torch.zeros((g.n, 21), dtype=torch.float64, device="cuda")
        with pytest.raises(pgo.PgoError) as ex:
            pgo.pgo_adjoint(h.h, d.data_ptr())
        assert ex.value.name == "PGO_ESTATE"
        bad = cuda(g.kappa)
        bad[3] = -1.0
        torch.cuda.synchronize()
        with pytest.raises(pgo.PgoError) as ex:
            pgo.pgo_set_edge_params(h.h, bad.data_ptr(), 0, 0, 0)
        assert ex.value.name == "PGO_EINVAL" and "kappa entry 3" in str(ex.value)


def test_backward_of_a_replaced_forward_raises(pgo):
    """Two forward passes on one handle: the handle keeps only the latest
    recording, so the first pass's backward raises instead of returning the
    second pass's gradients; the second pass's backward works, and equals a
    lone forward/backward with its parameters."""
    from paper_2601_15684_amd.autograd import unrolled_pradmm
    g = S.grid(4, 3, 3, all_pairs=True, sigma_R=0.05, sigma_t=0.1, seed=1)
    beta = 0.05 * abar(g)
    t_gt = cuda(g.t_gt)

    def leaves(scale):
        return [cuda(g.kappa * scale).requires_grad_(), cuda(g.tau).requires_grad_(),
                cuda(g.tm).requires_grad_(), cuda(np.zeros((g.m, 3))).requires_grad_()]

    with pgo.PoseGraph.from_graph(g, precision="fp64") as h:
        a, b = leaves(1.0), leaves(2.0)
        sa = unrolled_pradmm(h, *a, 6, beta, GAMMA, 3)
        id_a = pgo.pgo_record_id(h.h)
        sb = unrolled_pradmm(h, *b, 6, beta, GAMMA, 3)
        assert pgo.pgo_record_id(h.h) == id_a + 1
        with pytest.raises(RuntimeError, match="no longer this one"):
            ((sa[:, 8:11] - t_gt) ** 2).sum().backward()
        ((sb[:, 8:11] - t_gt) ** 2).sum().backward()
        got = b[0].grad.cpu().numpy()
        pgo.pgo_set_edge_params(h.h, b[0].data_ptr(), 0, 0, 0)
        assert pgo.pgo_record_id(h.h) == -1        # new edges: the recording is void
    torch.cuda.synchronize()
    with pgo.PoseGraph.from_graph(g, precision="fp64") as h:
        c = leaves(2.0)
        sc = unrolled_pradmm(h, *c, 6, beta, GAMMA, 3)
        ((sc[:, 8:11] - t_gt) ** 2).sum().backward()
    torch.cuda.synchronize()
    assert np.array_equal(got, c[0].grad.cpu().numpy())
