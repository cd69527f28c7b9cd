"""The stored reference minimum of grid-1k (tests/golden/fstar_grid1k.json,
written by tests/golden/make_fstar.py from the oracle only) against what the
oracle says about the same problem: it lies below the cost of both start
points, and no oracle PRADMM iterate from the odometry start goes below it."""
import json
import os

import numpy as np

import pgo_synth as S
from oracle import gn, prep
from oracle import pradmm as O

REC = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                  "fstar_grid1k.json")))


def abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def test_reference_minimum_bounds_the_oracle_iterates():
    F_star = REC["F_star"]
    assert REC["workload"] == "grid-1k"
    assert 0 < F_star < REC["F_chordal_start"] < REC["F_odometry_start"]
    g = S.make_config("grid-1k")
    P, p0, t0 = prep.prepare_graph(g)
    args = (P["ei"].numpy(), P["ej"].numpy(), P["qm"].numpy(), P["tm"].numpy(),
            P["kappa"].numpy(), P["tau"].numpy())
    assert abs(gn.model_cost(p0.numpy(), t0.numpy(), *args) - REC["F_odometry_start"]) <= \
        1e-9 * REC["F_odometry_start"]
    st = O.init_state(p0, t0)
    beta = 0.01 * abar(g)
    for _ in range(4):
        st = O.iterate(P, st, 50, beta, 1.4)
        F = float(O.cost(P, st["p"], st["t"]))
        assert F >= F_star * (1 - 1e-12)
