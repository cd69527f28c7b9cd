#!/usr/bin/env python3
"""Benchmark of the PRADMM sweep on one MI355X.

Workload (headline, ``batched-4096``): 4096 independent SE(3) pose graphs of
uneven size (poses uniform in [50, 5000], edges/poses uniform in [1.2, 4],
circle / grid / sphere topologies, sigma_R ~ U[0.01, 0.1] rad, sigma_t ~
U[0.01, 0.2] m), FP32 state, one persistent launch of 50 sweeps per step,
one penalty per graph, from the chordal initialisation of every graph (the
experiments start every method from it).  Warm-up: --warmup chunks of the
merit-checked solve (a graph whose merit rose redoes its chunk with a
doubled penalty).  One timed step
is one chunk of that solve over the whole batch: 50 sweeps of the four
phases (p, q, t, s with the multiplier updates) for every graph, the FP64
cost, residual and merit reductions of every graph (one pass) read back,
and the rerun of any graph whose merit rose; the value counts accepted
sweeps only.  The run exits with status 1 when any batch leg leaves a
graph above its starting cost.

Printed: one JSON line with edge-iterations/s (sum over graphs of edges x
accepted sweeps / wall time of the timed steps), the same hot path without
the merit check, the HBM roofline of the sweep kernel (hipEvent-timed
launches of every graph on the stream the kernel runs on), the plain FP64
path (with its own roofline), the rotation-matrix rendering and the
information model on the same batch, the chordal initialisation of the
batch, the differentiation workload (forward and hand-written adjoint of 50
unrolled sweeps of the 20000-pose grid), the in-kernel stopping rule, time
to a 1e-6 relative cost gap on the 1000-pose grid and on 32 sampled graphs
of the batch for both precisions, the single-graph workloads (100-pose
circle in FP64, 2500-pose sphere and 100k-pose grid in FP32 at three
relaxation steps), and the CPU oracle timed on a bounded sample over a
process pool (which also checks sampled graphs of the batch against the GPU
result).

    python bench.py [--gpus 1] [--steps 10] [--warmup 4]
    python bench.py --steps 0 ...   # only the roofline launches (profiling)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import pgo_synth as S  # noqa: E402

HBM_PEAK_GBS = 8000.0
B_EDGE = 44     # algorithmic bytes per edge per sweep (q~ 16, t~ 12, kappa+tau 8, two indices 8)
B_VERTEX = 168  # algorithmic bytes per pose per sweep (21-word FP32 state read and written)
# the same in FP64: edge q~ 32, t~ 24, kappa+tau 16, two indices 8; 21 doubles
# per pose read and written
B_EDGE_F64, B_VERTEX_F64 = 80, 336
# the rotation-matrix rendering: edge (kappa, tau 8, t~ 12, R~ 36, two indices
# 8) = 64 B; pose state P, Q, Lambda, t, s, z = 36 words read and written
B_EDGE_CHORDAL, B_VERTEX_CHORDAL = 64, 288
# the information model: the isotropic edge plus the 6 unique entries of S_e
B_EDGE_INFO = B_EDGE + 24
GAMMA = 1.4
BETA_SCALE = 0.01


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def abar(g):
    """Mean over poses of the diagonal weight 2 sum_out (tau |t~|^2 + kappa) + 2 sum_in kappa."""
    d = np.zeros(g.n)
    np.add.at(d, g.ei, 2 * (g.tau * (g.tm ** 2).sum(1) + g.kappa))
    np.add.at(d, g.ej, 2 * g.kappa)
    return float(d.mean())


KERNEL_SOURCES = {  # device sources each profiled sweep kernel is built from
    "k_graph_sweeps<false, float>": ("sweep_graph.hip", "sweep_core.hpp", "qmath.hpp",
                                     "internal.hpp"),
    "k_graph_sweeps<false, double>": ("sweep_graph.hip", "sweep_core.hpp", "qmath.hpp",
                                      "internal.hpp"),
    "k_graph_sweeps_c<float>": ("chordal.hip", "polar.hpp", "qmath.hpp", "internal.hpp"),
    "k_graph_sweeps_a<float>": ("aniso.hip", "qmath.hpp", "internal.hpp"),
}


def source_sha(kernel):
    """Hash of a sweep kernel's device sources without their comments and
    white space (the byte counters of profiles/traffic.json hold only for the
    code they were taken on)."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2601_15684_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel, ()):
        code = open(os.path.join(csrc, f)).read()
        code = re.sub(r"/\*.*?\*/", "", code, flags=re.S)
        code = re.sub(r"//[^\n]*", "", code)
        h.update(re.sub(r"\s+", "", code).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/traffic.json), or None when it is missing or was taken on
    other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[kernel]
    except (OSError, KeyError, ValueError):
        return None
    if kernel not in KERNEL_SOURCES or rec.get("source_sha") != source_sha(kernel):
        return None
    return rec["bytes_per_launch"]


def measured_rate(kernel, kern_ms, copy_gbs=None):
    """Bytes per launch between the L2 and the memory fabric from the
    committed counters (FETCH_SIZE and WRITE_SIZE scaled by a device copy of
    known size; or None when they were taken on other sources), the rate
    they give over the measured launch time, and its fractions of the peak
    and of a plain device copy's rate (the measured-traffic figures; the
    roofline frac uses algorithmic bytes)."""
    t = load_traffic(kernel)
    if t is None:
        return {"traffic": None}
    gbs = t / (kern_ms * 1e-3) / 1e9
    out = {"traffic": t, "traffic_GBs": gbs, "traffic_frac": gbs / HBM_PEAK_GBS}
    if copy_gbs:
        out["traffic_over_copy_rate"] = gbs / copy_gbs
    return out


def copy_rate(torch, gib=2, reps=5):
    """GB/s of a plain device-to-device copy (bytes read + written), timed
    with hipEvents: the bandwidth a streaming kernel reaches in practice."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        b.copy_(a)
        e1.record()
    torch.cuda.synchronize()
    ms = min(e0.elapsed_time(e1) for e0, e1 in ev)
    del a, b
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def copy_calibration(torch, gib=1):
    """A plain device copy of known size, so that rocprofv3 byte counters can
    be scaled (FETCH_SIZE/WRITE_SIZE of this copy vs its 2 x size bytes)."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def run_batch(P, torch, cat, voff, eoff, prec, betas, sweeps, steps, warmup, tune, sched, block,
              edges_per_graph, model="quat", info=None, plain_steps=0):
    """One handle over the whole batch.

    Warm-up: `warmup` chunks of the merit-checked solve (per graph, a chunk
    of `sweeps` sweeps whose merit rose is undone and rerun with its beta
    doubled), which settle most graphs' beta.
    Timed steps: `steps` chunks of the merit-checked solve -- a step is one
    pass of the hot path over the batch: one persistent launch of `sweeps`
    sweeps for every graph at its beta, the FP64 reductions of every graph
    (cost, residuals and merit, one pass, read back), the merit check, and
    for a graph whose merit rose its chunk undone and rerun; value =
    accepted edge-iterations / wall.
    Then `plain_steps` steps of the hot path without the check (one
    persistent launch + one pass of the reductions, read back) as a second
    figure, and the persistent launch alone timed with hipEvents on the
    handle's stream for the roofline (3 launches of `sweeps` sweeps, after
    an untimed one)."""
    stream = torch.cuda.Stream()
    opt = P.pgo_default_options(precision=prec, schedule=sched, block=block,
                                model=model if info is None else "quat")
    t0 = time.perf_counter()
    if info is None:
        h = P.pgo_create_batched(voff, eoff, cat["R0"].reshape(-1, 9), cat["t0"], cat["ei"], cat["ej"],
                                 cat["Rm"].reshape(-1, 9), cat["tm"], cat["kappa"], cat["tau"], opt)
    else:
        h = P.pgo_create_info(voff, eoff, cat["R0"].reshape(-1, 9), cat["t0"], cat["ei"], cat["ej"],
                              cat["Rm"].reshape(-1, 9), cat["tm"], cat["kappa"], info, opt)
    create_s = time.perf_counter() - t0
    P.pgo_set_stream(h, stream.cuda_stream)
    # the start: chordal initialisation, as the experiments start every method
    P.pgo_chordal_init(h, 4000, 1e-10)
    info = P.pgo_autotune(h, float(np.median(betas)), GAMMA, sweeps=10) if tune else P.pgo_info(h)
    log(f"[{model}/{prec}] created in {create_s:.2f}s, schedule={info['schedule']} block={info['block']}")
    F0 = P.pgo_cost(h)
    beta = betas.copy()
    accepted = np.zeros(len(betas), np.int64)
    warm_chunks, warm_rejected = 0, None
    for _ in range(warmup):
        b0 = beta.copy()
        beta, done, _ = P.pgo_solve(h, sweeps, sweeps, GAMMA, 0.0, 2.0, beta)
        accepted += done
        warm_chunks += 1
        warm_rejected = int(np.sum(beta > b0))
    if warmup:
        log(f"[{model}/{prec}] warm-up: {warm_chunks} chunks, {warm_rejected} graphs rejected in the last")
    wall = plain_wall = 0.0
    edge_iters = 0
    timed_rejected = 0
    if steps:
        b0 = beta.copy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            beta, done, _ = P.pgo_solve(h, steps * sweeps, sweeps, GAMMA, 0.0, 2.0, beta)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        accepted += done
        edge_iters = int(np.dot(done.astype(np.int64), edges_per_graph))
        timed_rejected = int(np.sum(beta > b0))
    m_total = int(np.sum(edges_per_graph))
    # the result of the run: after the merit-checked chunks
    res = P.pgo_residuals(h)
    state = P.pgo_get_state(h)
    if plain_steps:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(plain_steps):
                P.pgo_iterate_graphs(h, sweeps, beta, GAMMA)
                P.pgo_evaluate(h)
        torch.cuda.synchronize()
        plain_wall = time.perf_counter() - t0
    # the persistent launch alone, timed with hipEvents on the handle's stream
    # (after one untimed launch, so that the timed ones start warm also when
    # nothing ran before them, as in a profiling run with --steps 0)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(3)]
    with torch.cuda.stream(stream):
        P.pgo_iterate_graphs(h, sweeps, beta, GAMMA)
        for a, bb in evs:
            a.record(stream)
            P.pgo_iterate_graphs(h, sweeps, beta, GAMMA)
            bb.record(stream)
    torch.cuda.synchronize()
    kern_ms = float(np.mean([a.elapsed_time(bb) for a, bb in evs]))
    P.pgo_destroy(h)
    return dict(wall=wall, kern_ms=kern_ms, info=info, create_s=create_s, F0=F0, res=res,
                state=state, accepted=accepted, edge_iters=edge_iters, beta=beta,
                plain_wall=plain_wall, plain_edge_iters=m_total * sweeps * plain_steps,
                warm_chunks=warm_chunks, warm_rejected=warm_rejected,
                timed_rejected=timed_rejected, steps=steps)


def plain_figure(r, plain_steps):
    """The hot path without the merit check, timed after the steps."""
    if not plain_steps or not r["plain_wall"]:
        return None
    return {"value": r["plain_edge_iters"] / r["plain_wall"], "unit": "edge-iter/s",
            "ms_per_step": r["plain_wall"] / plain_steps * 1e3, "steps": plain_steps,
            "note": "one persistent launch of the sweeps for every graph + one pass of the FP64 "
                    "reductions read back, at the settled penalties, without the merit check"}


def stopping_leg(P, torch, cat, voff, eoff, betas, edges_per_graph, max_sweeps=1000, check=10,
                 tol=1e-4):
    """The experiments' stopping rule e < tol (App. E.1, tol 1e-4 as in the
    experiments section) on the batch from its chordal start at the
    penalties the headline leg's merit check settled, chunks of
    `check` sweeps, at most `max_sweeps`: evaluated inside the persistent
    kernel (pgo_iterate_until, one launch) against the host loop of
    pgo_solve without penalty control (one launch, reduction and host check
    per chunk).  Both stop every graph after the same sweeps."""
    opt = P.pgo_default_options(precision="fp32", schedule="graph", block=1024)
    h = P.pgo_create_batched(voff, eoff, cat["R0"].reshape(-1, 9), cat["t0"], cat["ei"], cat["ej"],
                             cat["Rm"].reshape(-1, 9), cat["tm"], cat["kappa"], cat["tau"], opt)
    P.pgo_chordal_init(h, 4000, 1e-10)
    s0 = P.pgo_get_state(h)
    P.pgo_iterate_until(h, check, check, betas, GAMMA, tol)  # warm-up of the launch path
    out = {"workload": "batched-4096", "tol": tol, "check_every": check, "max_sweeps": max_sweeps}
    for label in ("in_kernel", "host_loop"):
        P.pgo_set_state(h, s0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if label == "in_kernel":
            done = P.pgo_iterate_until(h, max_sweeps, check, betas, GAMMA, tol)
        else:
            _, done, _ = P.pgo_solve(h, max_sweeps, check, GAMMA, tol, 1.0, betas.copy())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[label] = {"seconds": wall, "graphs_stopped": int(np.sum(done < max_sweeps)),
                      "sweeps_median": float(np.median(done)), "sweeps_max": int(done.max()),
                      "edge_iters_per_s": float(np.dot(done.astype(np.int64), edges_per_graph)) / wall}
        out[label + "_sweeps"] = done
    out["same_sweeps"] = bool(np.array_equal(out.pop("in_kernel_sweeps"), out.pop("host_loop_sweeps")))
    P.pgo_destroy(h)
    return out


def cinit_leg(P, torch, cat, voff, eoff, steps):
    """Chordal initialisation of the whole batch on the device (FP64 CG per
    graph, tolerance 1e-10): wall time of the call, iterations, and the cost
    of the new initial point against the odometry start."""
    opt = P.pgo_default_options(precision="fp32")
    h = P.pgo_create_batched(voff, eoff, cat["R0"].reshape(-1, 9), cat["t0"], cat["ei"], cat["ej"],
                             cat["Rm"].reshape(-1, 9), cat["tm"], cat["kappa"], cat["tau"], opt)
    F_odo = P.pgo_cost(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = P.pgo_chordal_init(h, 4000, 1e-10)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    F_ch = P.pgo_cost(h)
    P.pgo_destroy(h)
    return {"workload": "batched-4096", "seconds": sec, "tol": 1e-10,
            "iterations_max": [int(its[:, 0].max()), int(its[:, 1].max())],
            "iterations_median": [float(np.median(its[:, 0])), float(np.median(its[:, 1]))],
            "median_cost_chordal_over_odometry": float(np.median(F_ch / F_odo))}


def adjoint_leg(P, torch, reps=3):
    """The differentiation workload (diff-20k, K = 50 unrolled sweeps,
    checkpoints every C = 10): forward, the loss sum |t_i - t_i^gt|^2 and the
    hand-written adjoint into kappa, tau, t~ and the rotation perturbation,
    through the torch.autograd.Function; wall time per forward + backward."""
    from paper_2601_15684_amd.autograd import unrolled_pradmm
    g = S.make_config("diff-20k")
    beta = BETA_SCALE * abar(g)
    K, C = 50, 10
    out = {"workload": "diff-20k", "poses": g.n, "edges": g.m, "K": K, "C": C}

    def leaf(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64,
                               device="cuda").requires_grad_()

    t_gt = torch.as_tensor(g.t_gt, dtype=torch.float64, device="cuda")
    for prec in ("fp32", "fp64"):
        with P.PoseGraph.from_graph(g, precision=prec) as h:
            ms = []
            for rep in range(reps + 1):
                kappa, tau, tm, om = leaf(g.kappa), leaf(g.tau), leaf(g.tm), leaf(np.zeros((g.m, 3)))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                state = unrolled_pradmm(h, kappa, tau, tm, om, K, beta, GAMMA, C)
                loss = ((state[:, 8:11] - t_gt) ** 2).sum()
                loss.backward()
                torch.cuda.synchronize()
                if rep:  # the first call builds the captured launch sequences
                    ms.append((time.perf_counter() - t0) * 1e3)
        out[prec] = {"ms_forward_and_adjoint": float(np.mean(ms)),
                     "edge_iters_per_s": g.m * K / (np.mean(ms) * 1e-3)}
    out["speedup_fp32_over_fp64"] = (out["fp64"]["ms_forward_and_adjoint"] /
                                     out["fp32"]["ms_forward_and_adjoint"])
    out["note"] = "edge_iters_per_s counts the K forward sweeps per forward + adjoint"
    return out


def health(r, betas, sizes=None):
    F0, F1 = r["F0"], r["res"][:, 5]
    w = int(np.argmax(F1 / F0))
    worst = {"graph": w, "F_initial": float(F0[w]), "F_final": float(F1[w]),
             "beta_over_initial": float(r["beta"][w] / betas[w])}
    if sizes is not None:
        worst["poses"], worst["edges"] = int(sizes[0][w]), int(sizes[1][w])
    return {"graphs_cost_up": int(np.sum(~(F1 <= F0))), "worst_graph": worst,
            "warmup_chunks": r["warm_chunks"], "graphs_rejected_in_last_warmup_chunk": r["warm_rejected"],
            "graphs_rejected_in_timed_steps": r["timed_rejected"],
            "graphs_nonfinite": int(np.sum(~np.isfinite(F1))),
            "median_final_over_initial": float(np.median(F1 / F0)),
            "worst_final_over_initial": float(np.max(F1 / F0)),
            "graphs_beta_raised": int(np.sum(r["beta"] > betas)),
            "max_beta_over_initial": float(np.max(r["beta"] / betas)),
            "accepted_sweeps_per_graph": [int(r["accepted"].min()), int(r["accepted"].max())]}


def time_to_tol(P, g, prec, beta, F_star, tol=1e-6, check_every=10, cap=20000):
    """Wall time (s) and sweeps until cost <= F*(1 + tol), cost checked every
    check_every sweeps (the reductions are inside the timed region), with the
    schedule the autotuner picks; returns (seconds, sweeps, schedule)."""
    with P.PoseGraph.from_graph(g, precision=prec) as h:
        s0 = h.state()
        sched = h.autotune(beta, GAMMA, sweeps=check_every)["schedule"]
        h.set_state(s0)
        h.iterate(check_every, beta, GAMMA)  # first call builds the captured launch sequence
        h.set_state(s0)
        t0 = time.perf_counter()
        done = 0
        while done < cap:
            h.iterate(check_every, beta, GAMMA)
            done += check_every
            F = h.cost()[0]
            if F <= F_star * (1 + tol):
                return time.perf_counter() - t0, done, sched
        return None, done, sched


def reference_minimum(name="grid-1k"):
    """F* of the time-to-tolerance target, written by the oracle
    (tests/golden/make_fstar.py: chordal initialisation, then least squares
    on model (1))."""
    rec = json.load(open(os.path.join(ROOT, "tests", "golden", "fstar_grid1k.json")))
    assert rec["workload"] == name
    return rec["F_star"]


def cpu_topology():
    """lscpu's model name, sockets, cores per socket and threads per core."""
    import subprocess
    out = {"model": None, "sockets": None, "cores_per_socket": None, "threads_per_core": None}
    try:
        text = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return out
    keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
            "Thread(s) per core": "threads_per_core"}
    for line in text.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keys and out[keys[k.strip()]] is None:
            v = v.strip()
            out[keys[k.strip()]] = int(v) if v.isdigit() else v
    return out


def host_workers(cap=16):
    """Worker processes for the CPU oracle: the CPUs this process may run on,
    at most `cap` (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def _oracle_worker_init():
    import torch
    torch.set_num_threads(1)


def _oracle_sweeps(job):
    """One graph of the batch through the FP64 oracle (a pool task): the
    graph is rebuilt from its seed in the worker, prepared, and run for
    `sweeps` sweeps; returns (edges, seconds of sweep time)."""
    k, graphs, sweeps, beta = job
    from oracle import prep
    from oracle import pradmm as O
    g = S.batched(graphs, first=k, count=1).graphs[0]
    Pr, p0, t0 = prep.prepare_graph(g)
    st = O.init_state(p0, t0)
    t = time.perf_counter()
    O.iterate(Pr, st, sweeps, beta, GAMMA)
    return g.m, time.perf_counter() - t


def cpu_leg(pool, workers, batch, betas, voff, gpu32, gpu64, g1k, beta1k, F_star, budget_s=8.0,
            sweeps=5):
    """The FP64 CPU oracle: (1) one thread on the first graphs of the batch
    for about budget_s seconds of sweep time; (2) the same graphs and as
    many again over all workers of a process pool (forked before the GPU was
    touched), wall time of the pool; (3) its time to a 1e-6 relative cost
    gap on grid-1k (cost checked every 10 sweeps, as the GPU leg); (4) run on
    sampled small graphs for as many sweeps as the GPU ran, to state the GPU
    error per result."""
    import torch

    from oracle import prep
    from oracle import pradmm as O

    threads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        e1, used, t1 = 0, 0, 0.0
        for g, b in zip(batch.graphs, betas):
            Pr, p0, t0 = prep.prepare_graph(g)
            st = O.init_state(p0, t0)
            t = time.perf_counter()
            O.iterate(Pr, st, sweeps, b, GAMMA)
            t1 += time.perf_counter() - t
            e1 += g.m
            used += 1
            if t1 > budget_s:
                break
    finally:
        torch.set_num_threads(threads)
    G = len(batch.graphs)
    count = min(G, max(used * workers, used))
    jobs = [(k, G, sweeps, float(betas[k])) for k in range(count)]
    t = time.perf_counter()
    done = pool.map(_oracle_sweeps, jobs, chunksize=1)
    t_pool = time.perf_counter() - t
    e_pool = sum(e for e, _ in done)
    topo = cpu_topology()
    base = dict(value=e_pool * sweeps / t_pool, unit="edge-iter/s", cores=workers,
                kind="oracle",
                sample=f"first {count} graphs of the batch, {sweeps} FP64 sweeps each "
                       f"({e_pool} edges), one graph per task over {workers} worker processes "
                       f"(one thread each), {t_pool:.1f} s wall",
                cpu=topo, workers=workers,
                value_1_thread=e1 * sweeps / t1,
                sample_1_thread=f"first {used} graphs, {sweeps} sweeps each, {t1:.1f} s",
                pool_speedup_over_1_thread=(e_pool * sweeps / t_pool) / (e1 * sweeps / t1))
    if F_star is not None:
        Pr, p0, t0 = prep.prepare_graph(g1k)
        st = O.init_state(p0, t0)
        t = time.perf_counter()
        done, reached = 0, None
        while done < 2000:
            st = O.iterate(Pr, st, 10, beta1k, GAMMA)
            done += 10
            if float(O.cost(Pr, st["p"], st["t"])) <= F_star * (1 + 1e-6):
                reached = time.perf_counter() - t
                break
        base["time_to_1e-6"] = {"workload": "grid-1k", "seconds": reached, "sweeps": done,
                                "cores": threads}
    # sampled parity: the three smallest graphs of the batch whose penalty the
    # merit check left unchanged; the oracle starts from its own chordal
    # initialisation (as the GPU legs start from the device's) and runs the
    # plain iteration for the GPU's accepted sweeps
    from oracle import chordal_init as CI
    order = np.argsort([g.n for g in batch.graphs])
    pick = [k for k in order if gpu32["beta"][k] == betas[k]
            and (gpu64 is None or gpu64["beta"][k] == betas[k])][:3]

    errs = {}
    starts = {}
    for prec, run in (("fp32", gpu32), ("fp64", gpu64)):
        if run is None:
            continue
        worst = {}
        for k in pick:
            g = batch.graphs[k]
            if k not in starts:
                Rc, tc = CI.chordal_init_graph(g)
                starts[k] = prep.prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau, Rc, tc)
            Pr, p0, t0 = starts[k]
            st = O.iterate(Pr, O.init_state(p0, t0), int(run["accepted"][k]), betas[k], GAMMA)
            ref = np.concatenate([st[q].numpy() for q in ("p", "q", "t", "s", "lam", "z")], 1)
            got = run["state"][voff[k]:voff[k + 1]]
            for name, sl, sc in (("p", slice(0, 4), 1), ("q", slice(4, 8), 1), ("t", slice(8, 11), 1),
                                 ("s", slice(11, 14), 1), ("lam/beta", slice(14, 18), betas[k]),
                                 ("z/beta", slice(18, 21), betas[k])):
                e = float(np.abs(got[:, sl] - ref[:, sl]).max()) / sc
                worst[name] = max(worst.get(name, 0.0), e)
        errs[prec] = worst
    base["sampled_parity"] = {"graphs": [batch.graphs[k].name for k in pick],
                              "sweeps": [int(gpu32["accepted"][k]) for k in pick],
                              "max_abs_err": errs,
                              "note": "raw max-abs per block after the GPU's accepted sweeps "
                                      "from the chordal start (multipliers over beta); the "
                                      "oracle's and the device's chordal starts agree to the "
                                      "CG tolerance, 1e-10 relative"}
    return base


def load_golden(name):
    path = os.path.join(ROOT, "tests", "golden", name)
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return None


def config_legs(P, torch, fstar, tol=1e-6, check=10, cap=20000):
    """The single-graph workloads, plain PRADMM at beta = 0.01 x mean
    diagonal weight (fixed): the 100-pose circle in FP64 for 200 sweeps from
    the odometry start; the 2500-pose sphere and the 100k-pose grid in FP32
    for 1000 sweeps at gamma 1.0, 1.5 and 1.9 from the device chordal
    initialisation (the experiments' start).  Per run: the schedule the
    autotuner picked, edge-iter/s of the whole sweep count in one call, the
    rate of the algorithmic bytes against the HBM peak, the final cost
    against F* (the oracle's minimum of the same objective, when stored) and
    the time to cost <= F*(1 + tol), the cost checked every `check` sweeps
    inside the timed region, at most `cap` sweeps."""
    legs = [("circle-100", "fp64", 200, (GAMMA,), "odometry"),
            ("sphere-2.5k", "fp32", 1000, (1.0, 1.5, 1.9), "chordal"),
            ("grid-100k", "fp32", 1000, (1.0, 1.5, 1.9), "chordal")]
    out = {}
    for name, prec, iters, gammas, start in legs:
        g = S.make_config(name)
        beta = BETA_SCALE * abar(g)
        F_star = ((fstar or {}).get(name) or {}).get(start, {}).get("F_star")
        be, bv = (B_EDGE_F64, B_VERTEX_F64) if prec == "fp64" else (B_EDGE, B_VERTEX)
        rec = {"poses": g.n, "edges": g.m, "dtype": "f64" if prec == "fp64" else "f32",
               "sweeps": iters, "beta": beta, "start": start, "F_star": F_star,
               "bytes_model": f"{be} B/edge + {bv} B/pose per sweep"}
        with P.PoseGraph.from_graph(g, precision=prec) as h:
            if start == "chordal":
                h.chordal_init(4000, 1e-10)
            s0 = h.state()
            F0 = float(h.cost()[0])
            info = h.autotune(beta, gammas[0], sweeps=10)
            rec["schedule"] = ["auto", "phase", "graph", "coop"][info["schedule"]]
            rec["block"] = info["block"]
            rec["F_start"] = F0
            for gm in gammas:
                h.set_state(s0)
                h.iterate(iters, beta, gm)  # builds the captured launch sequence
                h.set_state(s0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h.iterate(iters, beta, gm)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                F = float(h.cost()[0])
                e = float(h.residuals()[0, 2])
                h.set_state(s0)
                h.iterate(check, beta, gm)
                h.set_state(s0)
                reached, done = None, 0
                if F_star is not None:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    while done < cap:
                        h.iterate(check, beta, gm)
                        done += check
                        if float(h.cost()[0]) <= F_star * (1 + tol):
                            reached = time.perf_counter() - t0
                            break
                gbs = (be * g.m + bv * g.n) * iters / wall / 1e9
                rec[f"gamma={gm}"] = {
                    "seconds": wall, "us_per_sweep": wall / iters * 1e6,
                    "edge_iters_per_s": g.m * iters / wall,
                    "roofline": {"bound": "latency" if gbs < 0.05 * HBM_PEAK_GBS else "hbm",
                                 "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": gbs / HBM_PEAK_GBS},
                    "final_over_start_cost": F / F0,
                    "final_rel_gap": (F / F_star - 1) if F_star else None,
                    "residual_e": e,
                    "time_to_tol": {"seconds": reached, "sweeps": done if reached else None,
                                    "tol": tol, "check_every": check, "cap_sweeps": cap}}
        out[name] = rec
    return out


def batch_ttt_leg(P, torch, cat, voff, eoff, betas, sample, sched, block, chunk=50, cap=30000,
                  tol=1e-6):
    """Time for the batch to bring every sampled graph within tol of its F*
    (the oracle's minimum of model (1) from its chordal start): chordal
    initialisation of the whole batch on the device, then chunks of the
    merit-checked solve for all graphs, the sampled graphs' costs read back
    after every chunk (inside the timed region), FP32 and FP64."""
    idx = np.array([r["index"] for r in sample["graphs"]])
    Fs = np.array([r["F_star"] for r in sample["graphs"]])
    out = {"workload": "batched-4096", "sampled_graphs": int(len(idx)), "tol": tol,
           "chunk_sweeps": chunk, "cap_sweeps": cap,
           "start": "pgo_chordal_init on the device (FP64 CG, tolerance 1e-10)",
           "F_star_from": "oracle: chordal initialisation + damped Newton on model (1), "
                          "tests/golden/fstar_batch_sample.json"}
    for prec in ("fp32", "fp64"):
        opt = P.pgo_default_options(precision=prec, schedule=sched, block=block)
        h = P.pgo_create_batched(voff, eoff, cat["R0"].reshape(-1, 9), cat["t0"], cat["ei"], cat["ej"],
                                 cat["Rm"].reshape(-1, 9), cat["tm"], cat["kappa"], cat["tau"], opt)
        P.pgo_solve(h, chunk, chunk, GAMMA, 0.0, 2.0, betas.copy())  # warm-up of the launch path
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.pgo_chordal_init(h, 4000, 1e-10)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        F_init = P.pgo_cost(h)
        beta = betas.copy()
        done, reached = 0, None
        first = np.full(len(idx), -1)   # sweeps at which each sampled graph first got within tol
        first_s = np.full(len(idx), np.nan)   # and the wall time since the sweeps started
        t1 = time.perf_counter()
        while done < cap:
            beta, _, _ = P.pgo_solve(h, chunk, chunk, GAMMA, 0.0, 2.0, beta)
            done += chunk
            F = P.pgo_cost(h)
            within = F[idx] <= Fs * (1 + tol)
            now = time.perf_counter() - t1
            first_s[(first < 0) & within] = now
            first[(first < 0) & within] = done
            if np.all(within):
                reached = now
                break
        t_run = time.perf_counter() - t1
        gap = F[idx] / Fs - 1
        out[prec] = {"seconds_init": t_init, "seconds_sweeps": reached,
                     "seconds_total": t_init + reached if reached is not None else None,
                     "sweeps": done if reached is not None else None,
                     "seconds_run": t_run, "sweeps_run": done,
                     "graphs_within_tol": int(np.sum(gap <= tol)),
                     "sweeps_to_tol_per_graph": [int(x) if x >= 0 else None for x in first],
                     "seconds_to_tol_per_graph": [float(x) if np.isfinite(x) else None
                                                  for x in first_s],
                     "max_rel_gap": float(gap.max()), "min_rel_gap": float(gap.min()),
                     "graphs_cost_up_from_init": int(np.sum(~(F <= F_init))),
                     "graphs_beta_raised": int(np.sum(beta > betas))}
        P.pgo_destroy(h)
    if out["fp32"]["seconds_total"] and out["fp64"]["seconds_total"]:
        out["speedup_fp32_over_fp64"] = out["fp64"]["seconds_total"] / out["fp32"]["seconds_total"]
    # equal accuracy: the sampled graphs both precisions bring within tol,
    # and the time until the last of them is
    both = [k for k in range(len(idx)) if out["fp32"]["seconds_to_tol_per_graph"][k] is not None
            and out["fp64"]["seconds_to_tol_per_graph"][k] is not None]
    if both:
        t32 = max(out["fp32"]["seconds_to_tol_per_graph"][k] for k in both)
        t64 = max(out["fp64"]["seconds_to_tol_per_graph"][k] for k in both)
        out["common"] = {"graphs": len(both),
                         "fp32_seconds": out["fp32"]["seconds_init"] + t32,
                         "fp64_seconds": out["fp64"]["seconds_init"] + t64,
                         "speedup_fp32_over_fp64": (out["fp64"]["seconds_init"] + t64) /
                                                   (out["fp32"]["seconds_init"] + t32),
                         "note": "chordal initialisation + merit-checked chunks until every sampled "
                                 "graph that both precisions bring within tol is"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps (0: only the hipEvent-timed plain launches)")
    ap.add_argument("--warmup", type=int, default=4,
                    help="least number of untimed chunks of the merit-checked solve; the warm-up "
                         "goes on until a chunk rejects no graph")
    ap.add_argument("--sweeps", type=int, default=50, help="sweeps per persistent launch (one step)")
    ap.add_argument("--graphs", type=int, default=4096)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-chordal", action="store_true", help="skip the rotation-matrix model leg")
    ap.add_argument("--skip-cinit", action="store_true", help="skip the chordal-initialisation leg")
    ap.add_argument("--skip-info", action="store_true", help="skip the information-model leg")
    ap.add_argument("--skip-ttt", action="store_true", help="skip the time-to-tolerance legs")
    ap.add_argument("--skip-configs", action="store_true", help="skip the single-graph workloads")
    ap.add_argument("--skip-adjoint", action="store_true", help="skip the differentiation leg")
    ap.add_argument("--skip-stop", action="store_true", help="skip the stopping-rule leg")
    ap.add_argument("--no-tune", action="store_true", help="use --schedule/--block as given")
    ap.add_argument("--schedule", default="auto", choices=["auto", "phase", "graph", "coop"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a 1 GiB device copy first (byte-counter calibration for rocprofv3)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the batched sweep would shard by whole graphs with "
              "no exchange between GPUs, and no multi-GPU leg is measured here (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    # inputs first, and the CPU oracle's process pool: both fork worker
    # processes, which must happen before this process touches the GPU
    t0 = time.perf_counter()
    batch = S.batched(args.graphs, workers=args.workers)
    voff, eoff = batch.offsets()
    cat = batch.concat()
    n, m = int(voff[-1]), int(eoff[-1])
    betas = np.array([BETA_SCALE * abar(g) for g in batch.graphs])
    g1k = S.make_config("grid-1k")
    beta1k = BETA_SCALE * abar(g1k)
    log(f"generated {args.graphs} graphs: n={n} m={m} in {time.perf_counter() - t0:.1f}s")
    pool, workers = None, host_workers(args.workers)
    if not args.skip_cpu and args.steps:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(workers, initializer=_oracle_worker_init)

    import torch

    import paper_2601_15684_amd as P
    P.lib()
    torch.cuda.init()
    if args.copy_calib:
        copy_calibration(torch)
    tune = not args.no_tune
    copy_gbs = copy_rate(torch)
    epg = (eoff[1:] - eoff[:-1]).astype(np.int64)
    sizes = (voff[1:] - voff[:-1], epg)
    r32 = run_batch(P, torch, cat, voff, eoff, "fp32", betas, args.sweeps, args.steps, args.warmup,
                    tune, args.schedule, args.block, epg, plain_steps=args.steps)
    value = r32["edge_iters"] / r32["wall"] if args.steps else None
    algo_bytes = (B_EDGE * m + B_VERTEX * n) * args.sweeps
    achieved = algo_bytes / (r32["kern_ms"] * 1e-3) / 1e9
    sched_names = ["auto", "phase", "graph", "coop"]
    kname = ("k_graph_sweeps<false, float>"
             if r32["info"]["schedule"] == 2 else "k_phase<*,float>")
    out = {
        "metric": "edge-iters/s + time to 1e-6 rel cost; FP32/batched vs plain FP64, 1 GPU",
        "value": value,
        "unit": "edge-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["wall"] / args.steps * 1e3 if args.steps else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched-4096", "graphs": args.graphs, "poses": n, "edges": m,
                   "sweeps_per_step": args.sweeps,
                   "step": "one chunk of the merit-checked solve: one persistent launch of the "
                           "sweeps for all graphs, FP64 cost, residual and merit reductions per "
                           "graph (one pass) read back, a graph whose merit rose undone and rerun "
                           "with its beta doubled; value counts accepted sweeps",
                   "beta": f"per graph: {BETA_SCALE} x mean diagonal weight, raised by the "
                           f"merit check",
                   "start": "chordal initialisation on the device (pgo_chordal_init, tol 1e-10)",
                   "gamma": GAMMA, "schedule": sched_names[r32["info"]["schedule"]],
                   "block": r32["info"]["block"], "lds_state": bool(r32["info"]["lds"]),
                   "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, **measured_rate(kname, r32["kern_ms"], copy_gbs),
                     "device_copy_GBs": copy_gbs,
                     "frac_of_device_copy": achieved / copy_gbs,
                     "kernel": kname, "kernel_ms_per_launch": r32["kern_ms"],
                     "bytes_per_launch": algo_bytes,
                     "bytes_model": f"{B_EDGE} B/edge + {B_VERTEX} B/pose per sweep x {args.sweeps} sweeps"},
        "batch_health": health(r32, betas, sizes),
        "plain_path": plain_figure(r32, args.steps),
    }
    legs = {"fp32": r32}
    r64 = None
    if not args.skip_fp64:
        steps64 = max(2, args.steps // 2) if args.steps else 0
        r64 = run_batch(P, torch, cat, voff, eoff, "fp64", betas, args.sweeps, steps64, args.warmup,
                        tune, args.schedule, args.block, epg, plain_steps=steps64)
        legs["fp64"] = r64
        v64 = r64["edge_iters"] / r64["wall"] if steps64 else None
        b64 = (B_EDGE_F64 * m + B_VERTEX_F64 * n) * args.sweeps
        a64 = b64 / (r64["kern_ms"] * 1e-3) / 1e9
        k64 = ("k_graph_sweeps<false, double>" if r64["info"]["schedule"] == 2
               else "k_phase<*,double>")
        out["fp64"] = {"value": v64, "unit": "edge-iter/s", "steps": steps64, "dtype": "f64",
                       "kernel": k64, "kernel_ms_per_launch": r64["kern_ms"],
                       "schedule": sched_names[r64["info"]["schedule"]],
                       "roofline": {"bound": "hbm", "achieved": a64, "peak": HBM_PEAK_GBS,
                                    "unit": "GB/s", "frac": a64 / HBM_PEAK_GBS,
                                    **measured_rate(k64, r64["kern_ms"], copy_gbs),
                                    "bytes_per_launch": b64,
                                    "bytes_model": f"{B_EDGE_F64} B/edge + {B_VERTEX_F64} B/pose per "
                                                   f"sweep x {args.sweeps} sweeps"},
                       "speedup_fp32_over_fp64": value / v64 if v64 else None,
                       "kernel_speedup_fp32_over_fp64": r64["kern_ms"] / r32["kern_ms"],
                       "batch_health": health(r64, betas, sizes),
                       "plain_path": plain_figure(r64, steps64)}
    if not args.skip_chordal:
        # the rotation-matrix rendering on the same batch (FP32): state
        # P, Q, Lambda (9 words each), t, s, z; edges kappa R~ (9), tau t~, tau
        stc = max(2, args.steps // 2) if args.steps else 0
        rc = run_batch(P, torch, cat, voff, eoff, "fp32", betas, args.sweeps, stc,
                       args.warmup if args.steps else 0, tune, args.schedule,
                       args.block, epg, model="chordal")
        legs["chordal"] = rc
        cb = (B_EDGE_CHORDAL * m + B_VERTEX_CHORDAL * n) * args.sweeps
        ca = cb / (rc["kern_ms"] * 1e-3) / 1e9
        ckern = "k_graph_sweeps_c<float>" if rc["info"]["schedule"] == 2 else "k_phase_c<*,float>"
        out["chordal"] = {
            "value": rc["edge_iters"] / rc["wall"] if stc else None, "unit": "edge-iter/s",
            "steps": stc, "dtype": "f32", "kernel": ckern,
            "kernel_ms_per_launch": rc["kern_ms"],
            "roofline": {"bound": "hbm", "achieved": ca, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ca / HBM_PEAK_GBS, **measured_rate(ckern, rc["kern_ms"], copy_gbs),
                         "bytes_model": f"{B_EDGE_CHORDAL} B/edge + {B_VERTEX_CHORDAL} B/pose per "
                                        f"sweep x {args.sweeps} sweeps"},
            "batch_health": health(rc, betas, sizes)}
    if not args.skip_info:
        # the information model on the same batch: S_e = tau_e R diag(a) R^T
        # with eigenvalue ratios up to 10 (FP32)
        info = S.random_info(m, cat["tau"], 10.0, seed=0)
        sti = max(2, args.steps // 2) if args.steps else 0
        ri = run_batch(P, torch, cat, voff, eoff, "fp32", betas, args.sweeps, sti,
                       args.warmup if args.steps else 0, tune,
                       "auto" if args.schedule in ("auto", "coop") else args.schedule,
                       min(args.block, 512 if args.schedule == "graph" else 256), epg, info=info)
        legs["information_model"] = ri
        del info
        ib = (B_EDGE_INFO * m + B_VERTEX * n) * args.sweeps
        ia = ib / (ri["kern_ms"] * 1e-3) / 1e9
        ikern = "k_graph_sweeps_a<float>" if ri["info"]["schedule"] == 2 else "k_phase_a<*,float>"
        out["information_model"] = {
            "value": ri["edge_iters"] / ri["wall"] if sti else None, "unit": "edge-iter/s",
            "steps": sti, "dtype": "f32", "kernel": ikern,
            "kernel_ms_per_launch": ri["kern_ms"],
            "roofline": {"bound": "hbm", "achieved": ia, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ia / HBM_PEAK_GBS, **measured_rate(ikern, ri["kern_ms"], copy_gbs),
                         "bytes_model": f"{B_EDGE_INFO} B/edge + {B_VERTEX} B/pose per sweep x {args.sweeps} sweeps"},
            "batch_health": health(ri, betas, sizes)}
    if not args.skip_cinit:
        out["chordal_init"] = cinit_leg(P, torch, cat, voff, eoff, args.steps)
    if not args.skip_adjoint and args.steps:
        out["differentiation"] = adjoint_leg(P, torch)
    if not args.skip_stop and args.steps:
        out["stopping_rule"] = stopping_leg(P, torch, cat, voff, eoff, r32["beta"], epg)
    if not args.skip_ttt:
        F_star = reference_minimum()
        ttt = {"workload": "grid-1k", "F_star": F_star,
               "F_star_from": "oracle: chordal initialisation + least squares on model (1), "
                              "tests/golden/fstar_grid1k.json"}
        for prec in ("fp64", "fp32"):
            s, k, sch = time_to_tol(P, g1k, prec, beta1k, F_star)
            ttt[prec] = {"seconds": s, "sweeps": k, "schedule": sched_names[sch],
                         "us_per_sweep_incl_checks": s / k * 1e6 if s else None}
        if ttt["fp64"]["seconds"] and ttt["fp32"]["seconds"]:
            ttt["speedup_fp32_over_fp64"] = ttt["fp64"]["seconds"] / ttt["fp32"]["seconds"]
        out["time_to_1e-6"] = ttt
        sample = load_golden("fstar_batch_sample.json")
        if sample is not None and args.graphs == 4096:
            out["batch_time_to_1e-6"] = batch_ttt_leg(
                P, torch, cat, voff, eoff, betas, sample, sched_names[r32["info"]["schedule"]],
                r32["info"]["block"])
    if not args.skip_configs and args.steps:
        out["single_graph_workloads"] = config_legs(P, torch, load_golden("fstar_configs.json"))
    if pool is not None:
        out["cpu_baseline"] = cpu_leg(pool, workers, batch, betas, voff, r32, r64, g1k, beta1k,
                                      None if args.skip_ttt else reference_minimum())
        pool.close()
        pool.join()
    bad = {k: health(r, betas)["graphs_cost_up"] for k, r in legs.items()}
    bad = {k: v for k, v in bad.items() if v}
    out["all_legs_descend"] = not bad
    print(json.dumps(out), flush=True)
    if bad:
        log(f"graphs whose final cost is above their starting cost: {bad}")
        sys.exit(1)


if __name__ == "__main__":
    main()
