"""Writes fstar_configs.json: the reference minima F* of model (1) for the
single-graph workloads (the 100-pose circle, the 2500-pose sphere), the
targets of their time-to-1e-6-relative-cost measurements.  Computed by the
oracle only.  The edge quaternions' signs are aligned against the start
point of the run they serve (oracle/prep.py), which fixes the objective:
  * "odometry": signs aligned against the odometry start (the library's
    handle as created);
  * "chordal": signs aligned against the chordal start (the handle after
    pgo_chordal_init, which aligns them again).
Either minimum is taken by the sparse damped Newton method of oracle/gn.py
from the oracle's chordal initialisation (oracle/chordal_init.py; with the
odometry signs, each rotation on the odometry start's hemisphere), to a
relative cost decrease below 1e-12 in the quadratic regime.

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

NAMES = ["circle-100", "sphere-2.5k"]


def minimum(P, p_start, t_start):
    args = (P["ei"].numpy(), P["ej"].numpy(), P["qm"].numpy(), P["tm"].numpy(),
            P["kappa"].numpy(), P["tau"].numpy())
    F0 = gn.model_cost(p_start, t_start, *args)
    F, _, _, info = gn.sparse_local_min(p_start, t_start, *args)
    return {"F_start": F0, "F_star": F, "iterations": int(info["iterations"]),
            "last_rel_decrease": float(info["last_rel_decrease"]), "stop": info["stop"],
            "grad_max": float(info["grad_max"])}


def solve(name):
    g = S.make_config(name)
    t0 = time.time()
    Rc, tc = CI.chordal_init_graph(g)
    # signs against the odometry start; Newton from the chordal start on its hemisphere
    P, p0, t0v = prep.prepare_graph(g)
    args = (P["ei"].numpy(), P["ej"].numpy(), P["qm"].numpy(), P["tm"].numpy(),
            P["kappa"].numpy(), P["tau"].numpy())
    pc = prep.rot_to_quat(torch.as_tensor(Rc)).numpy()
    pc = pc * np.where((pc * p0.numpy()).sum(1) < 0, -1.0, 1.0)[:, None]
    odo = minimum(P, pc, tc)
    odo["F_odometry_start"] = gn.model_cost(p0.numpy(), t0v.numpy(), *args)
    # signs against the chordal start, Newton from it
    Pc, pcc, tcc = prep.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau, Rc, tc)
    cho = minimum(Pc, pcc.numpy(), tcc.numpy())
    rec = {"workload": name, "n": g.n, "m": g.m, "odometry": odo, "chordal": cho,
           "seconds": time.time() - t0}
    print(json.dumps(rec), flush=True)
    return rec


def main():
    names = sys.argv[1:] or NAMES
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fstar_configs.json")
    out = {}
    if os.path.exists(path):
        out = {k: v for k, v in json.load(open(path)).items() if "odometry" in v}
    for name in names:
        out[name] = solve(name)
        json.dump(out, open(path, "w"), indent=1)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
