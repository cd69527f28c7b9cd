"""Full-size check of the batched-4096 workload in the launch configuration
bench.py times: one handle over all 4096 graphs, per-graph schedule with
1024-thread workgroups and the multipliers in LDS (FP32; FP64 as well), one
beta per graph (0.01 x the graph's mean diagonal weight), 10 sweeps.
The rotation-matrix rendering and the information model (random
information matrices, seed 0) run the same way in their bench legs'
configuration (FP32, 1024 and 512 threads).  Sampled graphs (the largest,
the smallest, and six seeded picks) are run one by one through the FP64
oracle of each model and compared block by block, with the
bounds of the parity tests (tests/tolerance.py: raw max-abs per block,
multipliers over beta; FP64 1e-10, FP32 max(1e-4, 4 x the float32 oracle's
own departure on that graph)); the raw errors of every sampled graph are in
the JSON line.

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
    from tests import tolerance as T

    refs, floors = {}, {"fp32": {}, "fp64": {}}
    for k in pick:
        Pr, p0, t0 = prep.prepare_graph(batch.graphs[k])
        st0 = O.init_state(p0, t0)
        refs[k] = T.pack_quat(O.iterate(Pr, st0, SWEEPS, betas[k], GAMMA))
        floors["fp32"][k] = T.quat_floor(Pr, st0, betas[k], GAMMA, SWEEPS, ref=refs[k])
        floors["fp64"][k] = T.quat_floor(Pr, st0, betas[k], GAMMA, SWEEPS, ref=refs[k],
                                         dtype=torch.float64)
    print("oracle done", flush=True)
    torch.cuda.init()
    report, ok = {}, True
    for prec in ("fp32", "fp64"):
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
        worst, per_graph = {}, {}
        for k in pick:
            e = T.block_errors(state[voff[k]:voff[k + 1]], refs[k], betas[k])
            bad = T.check(batch.graphs[k].name, prec, e, floors[prec][k])
            per_graph[batch.graphs[k].name] = {c: float(f"{v:.3e}") for c, v in e.items()}
            for c, v in e.items():
                worst[c] = max(worst.get(c, 0.0), v)
            if bad:
                ok = False
                print(f"{prec}: graph {k} ({batch.graphs[k].name}) over its bound: {bad}", flush=True)
        report[prec] = {"lds": info["lds"], "schedule": info["schedule"], "block": info["block"],
                        "worst_raw": worst, "raw_per_graph": per_graph,
                        "floor_per_graph": {batch.graphs[k].name: {c: float(f"{v:.3e}") for c, v in floors[prec][k].items()} for k in pick}}
        print(f"{prec} done", flush=True)

    # the rotation-matrix rendering and the information model in the launch
    # configuration of their bench legs (FP32, per graph, LDS residency;
    # 1024 and 512 threads), the same sampled graphs against their oracles
    from oracle import aniso as A
    from oracle import chordal as C
    infos = S.random_info(int(eoff[-1]), cat["tau"], 10.0, seed=0)
    legs = {
        "chordal_fp32": dict(model="chordal", block=1024, blocks=T.CHORDAL_BLOCKS),
        "info_fp32": dict(model="info", block=512, blocks=T.QUAT_BLOCKS),
    }
    for leg, cfg in legs.items():
        refs_m, floors_m = {}, {}
        for k in pick:
            g = batch.graphs[k]
            if cfg["model"] == "chordal":
                Pb, P0, t0c = C.prepare_graph(g)
                st0 = C.init_state(P0, t0c)
                refs_m[k] = T.pack_chordal(C.iterate(Pb, st0, SWEEPS, betas[k], GAMMA))
                floors_m[k] = T.chordal_floor(Pb, st0, betas[k], GAMMA, SWEEPS, ref=refs_m[k])
            else:
                info_k = infos[eoff[k]:eoff[k + 1]]
                Pa, pa0, ta0 = A.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, info_k, g.R0, g.t0)
                st0 = O.init_state(pa0, ta0)
                refs_m[k] = T.pack_quat(A.iterate(Pa, st0, SWEEPS, betas[k], GAMMA))
                floors_m[k] = T.info_floor(Pa, st0, betas[k], GAMMA, SWEEPS, ref=refs_m[k])
        if cfg["model"] == "chordal":
            opt = P.pgo_default_options(precision="fp32", schedule="graph", block=cfg["block"],
                                        model="chordal")
            h = P.pgo_create_batched(voff, eoff, cat["R0"].reshape(-1, 9), cat["t0"], cat["ei"],
                                     cat["ej"], cat["Rm"].reshape(-1, 9), cat["tm"],
                                     cat["kappa"], cat["tau"], opt)
        else:
            opt = P.pgo_default_options(precision="fp32", schedule="graph", block=cfg["block"])
            h = P.pgo_create_info(voff, eoff, cat["R0"].reshape(-1, 9), cat["t0"], cat["ei"],
                                  cat["ej"], cat["Rm"].reshape(-1, 9), cat["tm"], cat["kappa"],
                                  infos, opt)
        try:
            info = P.pgo_info(h)
            P.pgo_iterate_graphs(h, SWEEPS, betas, GAMMA)
            state = P.pgo_get_state(h)
        finally:
            P.pgo_destroy(h)
        worst, per_graph = {}, {}
        for k in pick:
            e = T.block_errors(state[voff[k]:voff[k + 1]], refs_m[k], betas[k], cfg["blocks"])
            bad = T.check(f"{cfg['model']} {batch.graphs[k].name}", "fp32", e, floors_m[k])
            per_graph[batch.graphs[k].name] = {c: float(f"{v:.3e}") for c, v in e.items()}
            for c, v in e.items():
                worst[c] = max(worst.get(c, 0.0), v)
            if bad:
                ok = False
                print(f"{leg}: graph {k} ({batch.graphs[k].name}) over its bound: {bad}", flush=True)
        report[leg] = {"lds": info["lds"], "schedule": info["schedule"], "block": info["block"],
                       "worst_raw": worst, "raw_per_graph": per_graph}
        print(f"{leg} done", flush=True)
    print(json.dumps({"graphs": pick, "ok": ok, **report}), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
