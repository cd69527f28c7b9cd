"""Writes fstar_configs.json: the reference minimum F* of model (1) for the
single-graph workloads (the 100-pose circle, the 2500-pose sphere and the
100k-pose grid), the targets of their time-to-1e-6-relative-cost
measurements.  Computed by the oracle only, for the problem the library
solves from the odometry start (edge quaternions sign-aligned against the
odometry start, oracle/prep.py): the oracle's chordal initialisation
(oracle/chordal_init.py) as the starting point of the sparse damped Newton
method of oracle/gn.py on the model (1) residuals, to a relative cost
decrease below 1e-12 in the quadratic regime.  The edge signs stay those of
the odometry start, so F* is the minimum of the same objective the sweeps
run on.

    python tests/golden/make_fstar_configs.py [names...]   # minutes on one CPU
"""
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pgo_synth as S  # noqa: E402
from oracle import chordal_init as CI  # noqa: E402
from oracle import gn, prep  # noqa: E402

NAMES = ["circle-100", "sphere-2.5k", "grid-100k"]


def solve(name):
    g = S.make_config(name)
    t0 = time.time()
    P, p0, t0v = prep.prepare_graph(g)      # edge signs aligned against the odometry start
    args = (P["ei"].numpy(), P["ej"].numpy(), P["qm"].numpy(), P["tm"].numpy(),
            P["kappa"].numpy(), P["tau"].numpy())
    F_odo = gn.model_cost(p0.numpy(), t0v.numpy(), *args)
    Rc, tc = CI.chordal_init_graph(g)
    pc = prep.rot_to_quat(torch.as_tensor(Rc)).numpy()
    pc = pc * np.where((pc * p0.numpy()).sum(1) < 0, -1.0, 1.0)[:, None]   # p0's hemisphere
    F_chordal = gn.model_cost(pc, tc, *args)
    F, _, _, info = gn.sparse_local_min(pc, tc, *args)
    rec = {"workload": name, "n": g.n, "m": g.m, "F_odometry_start": F_odo,
           "F_chordal_start": F_chordal, "F_star": F, "iterations": int(info["iterations"]),
           "last_rel_decrease": float(info["last_rel_decrease"]), "stop": info["stop"],
           "grad_max": float(info["grad_max"]), "seconds": time.time() - t0}
    print(json.dumps(rec), flush=True)
    return rec


def main():
    names = sys.argv[1:] or NAMES
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fstar_configs.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        out[name] = solve(name)
        json.dump(out, open(path, "w"), indent=1)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
