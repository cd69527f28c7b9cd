"""pgo_evaluate_noalloc (the reductions with their scratch in the library's
static device array, results on the device) against pgo_evaluate on the same
handle: bit for bit, on two calls in a row, the second on a smaller handle,
and its refusals."""
import numpy as np
import pytest
import torch

import pgo_synth as S

pytestmark = pytest.mark.gpu

GAMMA = 1.4


def abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def evaluate_both(pgo, h, betas):
    F, res, mer = pgo.pgo_evaluate(h)
    G = len(betas)
    b = torch.tensor(betas, dtype=torch.float64, device="cuda")
    out = torch.full((G, 8), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    pgo.pgo_set_stream(h, stream.cuda_stream)
    pgo.pgo_evaluate_noalloc(h, b.data_ptr(), GAMMA, out.data_ptr())
    torch.cuda.synchronize()
    pgo.pgo_set_stream(h, 0)
    ref = np.concatenate([F[:, None], res[:, :5], mer], 1)
    return out.cpu().numpy(), ref


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_evaluate_on_two_calls(pgo, prec):
    big = S.batched(4096, first=200, count=12)
    small = S.batched(4096, first=300, count=3)
    for b in (big, small):            # the second call on a smaller input
        betas = np.array([0.01 * abar(gr) for gr in b.graphs])
        with pgo.PoseGraph.from_batch(b, precision=prec) as h:
            h.iterate(7, betas, GAMMA)
            got, ref = evaluate_both(pgo, h.h, betas)
        assert got.shape == ref.shape and np.isfinite(got).all()
        assert np.array_equal(got, ref), np.abs(got - ref).max()


def test_noalloc_refusals(pgo):
    g = S.make_config("circle-100")
    with pgo.PoseGraph.from_graph(g) as h:
        b = torch.ones(1, dtype=torch.float64, device="cuda")
        out = torch.empty(8, dtype=torch.float64, device="cuda")
        with pytest.raises(pgo.PgoError) as ex:
            pgo.pgo_evaluate_noalloc(h.h, b.data_ptr(), 2.0, out.data_ptr())
        assert ex.value.name == "PGO_EINVAL"
        with pytest.raises(pgo.PgoError):
            pgo.pgo_evaluate_noalloc(h.h, 0, GAMMA, out.data_ptr())
    with pgo.PoseGraph.from_graph(g, model="chordal") as h:
        with pytest.raises(pgo.PgoError) as ex:
            pgo.pgo_evaluate_noalloc(h.h, b.data_ptr(), GAMMA, out.data_ptr())
        assert ex.value.name == "PGO_ESTATE"
    # 14000 single-pose graphs need 20 doubles each: more than the array holds
    G = 14000
    voff, eoff = np.arange(G + 1, dtype=np.int64), np.zeros(G + 1, np.int64)
    R0, t0 = np.tile(np.eye(3).reshape(1, 9), (G, 1)), np.zeros((G, 3))
    e0i, e0f = np.zeros(0, np.int32), np.zeros(0)
    h = pgo.pgo_create_batched(voff, eoff, R0, t0, e0i, e0i, np.zeros((0, 9)), np.zeros((0, 3)),
                               e0f, e0f)
    try:
        bb = torch.ones(G, dtype=torch.float64, device="cuda")
        oo = torch.empty(G * 8, dtype=torch.float64, device="cuda")
        with pytest.raises(pgo.PgoError) as ex:
            pgo.pgo_evaluate_noalloc(h, bb.data_ptr(), GAMMA, oo.data_ptr())
        assert ex.value.name == "PGO_EINVAL" and "static scratch" in str(ex.value)
    finally:
        pgo.pgo_destroy(h)
