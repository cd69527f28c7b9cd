"""Writes fstar_batch_sample.json: the reference minimum F* of model (1) for a
seeded sample of 32 graphs of the batched-4096 workload, the target of the
batch's time-to-1e-6-relative-cost measurement.  Computed by the oracle
only, for the problem the library solves after pgo_chordal_init: the
oracle's chordal initial point (oracle/chordal_init.py), the edge
quaternions sign-aligned against it (oracle/prep.py), then the sparse
Newton method of oracle/gn.py (exact Hessian, Levenberg-Marquardt damping)
on the model (1) residuals from that point, to a relative cost decrease
below 1e-12 in the quadratic regime.

The sample: the batch's graphs except the circles above 2000 poses, sorted
by pose count, cut into 32 strata, one graph drawn from each by a seeded
generator, so sizes from 50 to 5000 poses and the three topologies are all
represented.  The large circles are left out because their loop closures
join uniformly random pose pairs: the oracle's Newton system is then
effectively dense (above 12000 unknowns, a dense Cholesky factorisation
per step, hours per graph on one host), while grids and spheres of 5000
poses factorise sparsely in seconds.

    python tests/golden/make_fstar_batch.py [--workers 2 --threads 4]   # tens of minutes on 8 CPUs
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pgo_synth as S  # noqa: E402

G = 4096
SAMPLE = 32


CIRCLE_MAX_N = 2000


def sample_indices():
    graphs = S.batched(G, workers=8).graphs
    sizes = np.array([g.n for g in graphs])
    keep = np.array([not (g.meta["kind"] == "circle" and g.n > CIRCLE_MAX_N) for g in graphs])
    pool = np.flatnonzero(keep)
    order = pool[np.argsort(sizes[pool], kind="stable")]
    rng = np.random.default_rng(2026)
    strata = np.array_split(order, SAMPLE)
    return sorted(int(rng.choice(s)) for s in strata), graphs


def solve(job):
    k, threads = job
    import torch
    from threadpoolctl import threadpool_limits
    torch.set_num_threads(threads)
    threadpool_limits(threads)
    from oracle import chordal_init as CI
    from oracle import gn, prep
    g = S.batched(G, first=k, count=1).graphs[0]
    t0 = time.time()
    Rc, tc = CI.chordal_init_graph(g)
    P, pc, tcc = prep.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau, Rc, tc)
    args = (P["ei"].numpy(), P["ej"].numpy(), P["qm"].numpy(), P["tm"].numpy(),
            P["kappa"].numpy(), P["tau"].numpy())
    F_chordal = gn.model_cost(pc.numpy(), tcc.numpy(), *args)
    F, _, _, info = gn.sparse_local_min(pc.numpy(), tcc.numpy(), *args)
    rec = {"index": k, "name": g.name, "kind": g.meta["kind"], "n": g.n, "m": g.m,
           "F_chordal_start": F_chordal, "F_star": F, "iterations": int(info["iterations"]),
           "last_rel_decrease": float(info["last_rel_decrease"]), "stop": info["stop"],
           "grad_max": float(info["grad_max"]), "seconds": time.time() - t0}
    print(json.dumps(rec), flush=True)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=2)
    ap.add_argument("--threads", type=int, default=4, help="BLAS threads per worker")
    ap.add_argument("--cache", default=None,
                    help="JSON-lines file of finished graphs: appended to, and read to skip them")
    args = ap.parse_args()
    idx, graphs = sample_indices()
    print(f"sampled graphs: {idx}", flush=True)
    import multiprocessing as mp
    # largest first, so the long solves do not end up last
    done = {}
    if args.cache and os.path.exists(args.cache):
        for line in open(args.cache):
            r = json.loads(line)
            done[r["index"]] = r
    todo = [k for k in idx if k not in done]
    sizes = {k: graphs[k].m for k in todo}
    del graphs
    with mp.get_context("fork").Pool(args.workers) as pool:
        jobs = [(k, args.threads) for k in sorted(todo, key=lambda k: -sizes[k])]
        for r in pool.imap_unordered(solve, jobs, chunksize=1):
            done[r["index"]] = r
            if args.cache:
                with open(args.cache, "a") as f:
                    f.write(json.dumps(r) + "\n")
    recs = [done[k] for k in idx]
    out = {"workload": "batched-4096", "graphs": recs,
           "start": "oracle chordal initialisation; edge signs aligned against it",
           "method": "damped Newton of oracle/gn.py on the model (1) residuals (analytic "
                     "Jacobian and second-order terms), relative cost decrease below 1e-12",
           "sample": "the batch's graphs except circles above 2000 poses, sorted by pose "
                     "count, 32 strata, one drawn from each (numpy default_rng(2026))"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fstar_batch_sample.json")
    json.dump(out, open(path, "w"), indent=1)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
