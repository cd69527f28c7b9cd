"""Writes fstar_grid1k.json: the reference minimum F* of model (1) on the
grid-1k workload (pgo_synth.make_config("grid-1k"), odometry start, edge
quaternion signs aligned against it), used as the target of the
time-to-1e-6-relative-cost measurement.  Computed by the oracle only: its
chordal initialisation, then the model-(1) residuals of oracle/gn.py
minimised by scipy's trust-region least squares with the residuals' sparse
Jacobian pattern.

    python tests/golden/make_fstar.py        # a few minutes on one CPU
"""
import json
import os
import sys

import numpy as np
import scipy.sparse as sp
import torch
from scipy.optimize import least_squares

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pgo_synth as S  # noqa: E402
from oracle import chordal_init as CI  # noqa: E402
from oracle import gn, prep  # noqa: E402


def jac_pattern(n, ei, ej):
    """Residual rows of edge e (3 translation, 4 rotation) depend on the 7
    unknowns (x_v in R^4, t_v) of its two ends."""
    m = len(ei)
    rows, cols = [], []
    for e in range(m):
        r = list(range(3 * e, 3 * e + 3)) + list(range(3 * m + 4 * e, 3 * m + 4 * e + 4))
        for v in (ei[e], ej[e]):
            c = list(range(4 * v, 4 * v + 4)) + list(range(4 * n + 3 * v, 4 * n + 3 * v + 3))
            for rr in r:
                rows += [rr] * len(c)
                cols += c
    return sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(7 * m, 7 * n)).tocsr()


def main():
    g = S.make_config("grid-1k")
    P, p0, t0 = prep.prepare_graph(g)
    ei, ej = P["ei"].numpy(), P["ej"].numpy()
    args = (g.n, ei, ej, P["qm"].numpy(), P["tm"].numpy(), P["kappa"].numpy(), P["tau"].numpy())
    F_odo = gn.model_cost(p0.numpy(), t0.numpy(), *args[1:])
    Rc, tc = CI.chordal_init_graph(g)
    pc = prep.rot_to_quat(torch.tensor(Rc)).numpy()
    s = np.where((pc * p0.numpy()).sum(1) < 0, -1.0, 1.0)  # each vertex on p0's side
    pc = pc * s[:, None]
    F_chordal = gn.model_cost(pc, tc, *args[1:])
    sol = least_squares(gn.residual, np.concatenate([pc.ravel(), tc.ravel()]), args=args,
                        jac_sparsity=jac_pattern(g.n, ei, ej), method="trf", tr_solver="lsmr",
                        x_scale="jac", xtol=1e-15, ftol=1e-15, gtol=1e-10, max_nfev=3000)
    r = gn.residual(sol.x, *args)
    out = {"workload": "grid-1k", "F_star": float(r @ r), "F_odometry_start": F_odo,
           "F_chordal_start": F_chordal, "optimality": float(sol.optimality),
           "function_evaluations": int(sol.nfev),
           "method": "oracle chordal initialisation, then scipy least_squares (trf, sparse "
                     "Jacobian pattern) on the model (1) residuals of oracle/gn.py"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fstar_grid1k.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
