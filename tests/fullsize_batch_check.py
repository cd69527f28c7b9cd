"""Full-size check of the batched-4096 workload in the launch configuration
bench.py times: one handle over all 4096 graphs, per-graph schedule with
1024-thread workgroups and the multipliers in LDS (FP32; FP64 as well), one
beta per graph (0.01 x the graph's mean diagonal weight), 10 sweeps.
Sampled graphs (the largest, the smallest, and six seeded picks) are run
one by one through the FP64 oracle and compared block by block, with the
tolerances of the parity tests (FP64 1e-10, FP32 1e-4, multipliers over
beta, everything over L = max(1, max|t| / 10 m)).

Run as a child process by tests/test_gpu_fullsize.py: the generator forks
worker processes, which has to happen before the process touches the GPU.
Prints one JSON line and exits non-zero on a failure.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import pgo_synth as S  # noqa: E402

GAMMA = 1.4
SWEEPS = 10


def abar(g):
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


def scaled_err(a, b, beta):
    sl = dict(p=slice(0, 4), q=slice(4, 8), t=slice(8, 11), s=slice(11, 14), lam=slice(14, 18),
              z=slice(18, 21))
    L = max(1.0, float(np.abs(b[:, 8:11]).max()) / 10.0)
    return {k: float(np.abs(a[:, s] - b[:, s]).max()) / (beta if k in ("lam", "z") else 1.0) / L
            for k, s in sl.items()}


def main():
    batch = S.batched(4096, workers=int(os.environ.get("PGO_GEN_WORKERS", "16")))
    voff, eoff = batch.offsets()
    cat = batch.concat()
    betas = np.array([0.01 * abar(g) for g in batch.graphs])
    sizes = np.diff(voff)
    rng = np.random.default_rng(7)
    pick = [int(np.argmax(sizes)), int(np.argmin(sizes))] + \
        [int(k) for k in rng.choice(len(sizes), 6, replace=False)]
    print(f"batch: {int(voff[-1])} poses, {int(eoff[-1])} edges; sampled graphs {pick}", flush=True)

    import torch

    import paper_2601_15684_amd as P
    from oracle import prep
    from oracle import pradmm as O

    refs = {}
    for k in pick:
        Pr, p0, t0 = prep.prepare_graph(batch.graphs[k])
        st = O.iterate(Pr, O.init_state(p0, t0), SWEEPS, betas[k], GAMMA)
        refs[k] = np.concatenate([st[c].numpy() for c in ("p", "q", "t", "s", "lam", "z")], 1)
    print("oracle done", flush=True)
    torch.cuda.init()
    report, ok = {}, True
    for prec, tol in (("fp32", 1e-4), ("fp64", 1e-10)):
        opt = P.pgo_default_options(precision=prec, schedule="graph", block=1024)
        h = P.pgo_create_batched(voff, eoff, cat["R0"].reshape(-1, 9), cat["t0"], cat["ei"],
                                 cat["ej"], cat["Rm"].reshape(-1, 9), cat["tm"], cat["kappa"],
                                 cat["tau"], opt)
        try:
            info = P.pgo_info(h)
            P.pgo_iterate_graphs(h, SWEEPS, betas, GAMMA)
            state = P.pgo_get_state(h)
        finally:
            P.pgo_destroy(h)
        worst = {}
        for k in pick:
            e = scaled_err(state[voff[k]:voff[k + 1]], refs[k], betas[k])
            for c, v in e.items():
                worst[c] = max(worst.get(c, 0.0), v)
            if not all(v <= tol for v in e.values()):
                ok = False
                print(f"{prec}: graph {k} ({batch.graphs[k].name}) exceeds {tol}: {e}", flush=True)
        report[prec] = {"tol": tol, "lds": info["lds"], "schedule": info["schedule"],
                        "block": info["block"], "worst": worst}
        print(f"{prec} done", flush=True)
    print(json.dumps({"graphs": pick, "ok": ok, **report}), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
