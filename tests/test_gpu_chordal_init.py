"""GPU chordal initialisation (pgo_chordal_init) against the oracle's sparse
direct solves (oracle/chordal_init.py): rotations and translations of the
new initial point, both models, batches, several components, exact recovery
without noise, and the sign alignment redone for the new quaternions.
Tolerances: the device solves stop at a relative preconditioned residual of
1e-13; the conditioning of these graph Laplacians (<= ~1e4) leaves the
solution within ~1e-9, checked at 1e-8 (rotations, unitless) and 1e-8 L
(translations, L = max(1, max|t| / 10 m))."""
import numpy as np
import pytest
import torch

import pgo_synth as S
from oracle import chordal as C
from oracle import chordal_init as CI

pytestmark = pytest.mark.gpu


def poses_after_init(pgo, g, **opt):
    with pgo.PoseGraph.from_graph(g, **opt) as h:
        its = h.chordal_init(5000, 1e-13)
        R, t = h.poses()
        return R, t, its, h.state()


def check(R, t, Rr, tr):
    L = max(1.0, float(np.abs(tr).max()) / 10.0)
    assert np.abs(R - Rr).max() < 1e-8
    assert np.abs(t - tr).max() < 1e-8 * L


@pytest.mark.parametrize("model", ["quat", "chordal"])
@pytest.mark.parametrize("name", ["grid-1k", "sphere-2.5k"])
def test_matches_oracle(pgo, name, model):
    g = S.make_config(name)
    Rr, tr = CI.chordal_init_graph(g)
    R, t, its, _ = poses_after_init(pgo, g, model=model)
    check(R, t, Rr, tr)
    assert 0 < its[0, 0] < 5000 and 0 < its[0, 1] < 5000


def test_batched_each_graph_matches_oracle(pgo):
    """A batch in FP32: the new initial rotations p^0 are kept in FP64 and
    compared at 1e-8; the state holds the translations rounded to float."""
    from oracle.quat import rotmat
    # graphs of the batch small enough for the oracle's sparse direct solves
    # (a circle's random closures make their factors dense)
    pick = (203, 205, 213, 232, 237, 239)
    b = S.Batch([S.batched(4096, first=k, count=1).graphs[0] for k in pick])
    voff, _ = b.offsets()
    with pgo.PoseGraph.from_batch(b, precision="fp32") as h:
        its = h.chordal_init(5000, 1e-13)
        _, p0 = h.prepared()
        t0 = h.state()[:, 8:11]
    assert its.shape == (6, 2)
    for k, gr in enumerate(b.graphs):
        Rr, tr = CI.chordal_init_graph(gr)
        R = rotmat(torch.as_tensor(p0[voff[k]:voff[k + 1]])).numpy()
        assert np.abs(R - Rr).max() < 1e-8, gr.name
        L = max(1.0, float(np.abs(tr).max()) / 10.0)
        assert np.abs(t0[voff[k]:voff[k + 1]] - tr).max() < 1e-6 * L, gr.name


def test_components_keep_their_anchors_and_noise_free_recovers_truth(pgo):
    rng = np.random.default_rng(3)
    g = S.grid(4, 3, 3, p=0.6, sigma_R=0.0, sigma_t=0.0, init="gt", seed=2)
    h_ = S.tree(5, seed=7, sigma_R=0.0, sigma_t=0.0, init="gt")
    n = g.n + h_.n
    R_gt = np.concatenate([g.R_gt, h_.R_gt]); t_gt = np.concatenate([g.t_gt, h_.t_gt])
    R0 = R_gt @ S.so3_exp(0.3 * rng.standard_normal((n, 3)))
    t0 = t_gt + 0.3 * rng.standard_normal((n, 3))
    R0[0], t0[0] = R_gt[0], t_gt[0]
    R0[g.n], t0[g.n] = R_gt[g.n], t_gt[g.n]
    ei = np.concatenate([g.ei, h_.ei + g.n]); ej = np.concatenate([g.ej, h_.ej + g.n])
    Rm = np.concatenate([g.Rm, h_.Rm]); tm = np.concatenate([g.tm, h_.tm])
    kap = np.concatenate([g.kappa, h_.kappa]); tau = np.concatenate([g.tau, h_.tau])
    for model in ("quat", "chordal"):
        o = pgo.pgo_default_options(model=model)
        hd = pgo.pgo_create(n, R0.reshape(-1, 9), t0, ei, ej, Rm.reshape(-1, 9), tm, kap, tau, o)
        try:
            pgo.pgo_chordal_init(hd, 5000, 1e-14)
            R, t = pgo.pgo_get_poses(hd)
            assert np.abs(R - R_gt).max() < 1e-9 and np.abs(t - t_gt).max() < 1e-9, model
            assert pgo.pgo_cost(hd)[0] < 1e-16
            pgo.pgo_iterate(hd, 5, 100.0, 1.4)  # ground truth is a fixed point of the sweep
            R2, t2 = pgo.pgo_get_poses(hd)
            assert np.abs(R2 - R_gt).max() < 1e-9 and np.abs(t2 - t_gt).max() < 1e-9, model
        finally:
            pgo.pgo_destroy(hd)


def test_quaternion_signs_realigned(pgo):
    """After the new p^0 every edge keeps <p_i^0 q~_e, p_j^0> >= 0, the sign rule of the boundary preparation."""
    from oracle.quat import qmul
    g = S.make_config("sphere-2.5k")
    with pgo.PoseGraph.from_graph(g) as h:
        h.chordal_init(5000, 1e-12)
        qe, p0 = h.prepared()
        s = h.state()
    a = qmul(torch.as_tensor(p0[g.ei]), torch.as_tensor(qe)).numpy()
    assert (np.einsum("kc,kc->k", a, p0[g.ej]) >= 0).all()
    assert np.array_equal(s[:, 0:4], p0) and np.array_equal(s[:, 4:8], p0)
    assert np.abs(s[:, 14:]).max() == 0.0


def test_argument_checks(pgo):
    g = S.make_config("circle-100")
    with pgo.PoseGraph.from_graph(g) as h:
        for mi, tol in ((0, 1e-8), (10, 0.0), (10, 1.5), (10, np.nan)):
            with pytest.raises(pgo.PgoError) as ex:
                pgo.pgo_chordal_init(h.h, mi, tol)
            assert ex.value.name == "PGO_EINVAL"
